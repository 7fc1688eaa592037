// plan.hip -- device-side batching: length-bucketed task formation.
//
// Pairs of one pass are sorted by a key (band class, padded query height,
// reference length) with a device radix sort and cut into tasks of `slots`
// consecutive pairs, so that the pairs sharing a wave have nearly the same
// dimensions and little padding.  Task sizes and buffer offsets are derived on
// the device; the host only reads back the totals it must allocate.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

// n_dev (may be null): the number of valid ids, read on the device; entries
// beyond it get the largest key (they sort last and form empty tasks)
__global__ void k_plan_keys(int64_t n, const int64_t *n_dev, const int64_t *ids, const int32_t *qlen,
                            const int64_t *rlen, const int32_t *band, int32_t R, uint64_t *keys,
                            int64_t *vals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (n_dev && k >= *n_dev) {
    keys[k] = ~0ull;
    vals[k] = -1;
    return;
  }
  const int64_t p = ids ? ids[k] : k;
  int64_t q = qlen[p];
  if (q < 1) q = 1;
  const uint64_t qc = (uint64_t)((q + R / 2 - 1) / (R / 2));   // half-strip buckets
  uint64_t r = (uint64_t)rlen[p];
  if (r > 0xFFFFFFFull) r = 0xFFFFFFFull;
  // band class: the band half-width, except that pairs whose band spans
  // nearly the whole reference (2 * band + R >= rlen: a strip's window then
  // leaves out few columns) are grouped by size alone, after the banded ones,
  // and unbanded pairs come last
  uint64_t b = 0;
  if (band) {
    if (band[p] < 0) b = 0xFFFFFull;
    else if (2 * (int64_t)band[p] + R >= (int64_t)rlen[p]) b = 0xFFFFEull;
    else b = (uint64_t)(band[p] > 0xFFFFD ? 0xFFFFD : band[p]);
  }
  keys[k] = (b << 44) | ((qc > 0xFFFF ? 0xFFFF : qc) << 28) | r;
  vals[k] = p;
}

__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// one wave per task: the lanes take the task's slots in turn, and the
// maxima are reduced across the wave
__global__ void k_plan_tasks(int64_t n, const int64_t *n_dev, int64_t ntasks, int32_t slots,
                             int32_t R, int64_t qdata_per_row, const int64_t *sorted,
                             const int32_t *qlen, const int64_t *rlen, const int32_t *band,
                             const int32_t *band_q, InterTask *tasks, int64_t *bnd_size,
                             int64_t *qdata_size) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= ntasks) return;
  if (n_dev) n = *n_dev;
  const int64_t s0 = t * slots;
  int64_t s1 = (s0 + slots < n) ? s0 + slots : n;
  if (s1 < s0) s1 = s0;   // a task past the valid ids is empty
  // mb, mbq: a negative band (none) counts as the largest
  int64_t mq = 1, mr = 1, mb = 0, mbq = 0;
  for (int64_t k = s0 + lane; k < s1; k += 64) {
    const int64_t p = sorted[k];
    if (qlen[p] > mq) mq = qlen[p];
    if (rlen[p] > mr) mr = rlen[p];
    if (band) {
      const int64_t b = band[p] < 0 ? INT64_MAX : band[p];
      mb = b > mb ? b : mb;
      const int64_t bq = band_q ? (band_q[p] < 0 ? INT64_MAX : band_q[p]) : b;
      mbq = bq > mbq ? bq : mbq;
    }
  }
  mq = wave_max_i64(mq);
  mr = wave_max_i64(mr);
  mb = wave_max_i64(mb);
  mbq = wave_max_i64(mbq);
  if (lane != 0) return;
  if (t == 0) {   // the totals' slots of the two scans
    bnd_size[ntasks] = 0;
    qdata_size[ntasks] = 0;
  }
  InterTask tk{};
  tk.nslots = (int32_t)(s1 - s0);
  // without a query profile the last strip may be half high: rows are
  // padded to a multiple of R / 2 (an odd multiple leaves a half strip last)
  const int64_t unit = qdata_per_row == 0 ? R / 2 : R;
  tk.qp = (int32_t)((mq + unit - 1) / unit * unit);
  tk.rp = (int32_t)((mr + 7) / 8 * 8);
  tk.band = band ? (mb == INT64_MAX ? -1 : (int32_t)mb) : -1;
  tk.band_q = (band && mbq != INT64_MAX && tk.band >= 0) ? (int32_t)mbq : tk.band;
  tk.slot_base = s0;
  tasks[t] = tk;
  bnd_size[t] = 3 * (int64_t)tk.rp * 64;
  // qdata_per_row < 0: a profile shared by every task (whole strips, no bytes per task)
  qdata_size[t] = qdata_per_row > 0 ? ((int64_t)tk.qp * qdata_per_row + 15) / 16 * 16 : 0;
}

__global__ void k_plan_offsets(int64_t ntasks, InterTask *tasks, const int64_t *bnd_off,
                               const int64_t *qdata_off) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  tasks[t].bnd_off = bnd_off[t];
  tasks[t].qdata_off = qdata_off[t];
}

// flagged compaction: out[k] = the k-th pair with flag != 0 (in pair order)
// f64[0 .. n) = flags as 0/1 and f64[n] = 0 (the total's slot of the scan)
__global__ void k_flag_to_i64(int64_t n, const uint8_t *flag, int64_t *f64) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) f64[p] = flag[p] ? 1 : 0;
  else if (p == n) f64[n] = 0;
}

__global__ void k_compact(int64_t n, const uint8_t *flag, const int64_t *pos, int64_t *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && flag[p]) out[pos[p]] = p;
}

__global__ void k_count_classes(int64_t n, const uint8_t *cls, int64_t *counts) {
  __shared__ int64_t c[8];
  if (threadIdx.x < 8) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    atomicAdd((unsigned long long *)&c[cls[p] & 7], 1ull);
  __syncthreads();
  if (threadIdx.x < 8 && c[threadIdx.x]) atomicAdd((unsigned long long *)&counts[threadIdx.x],
                                                   (unsigned long long)c[threadIdx.x]);
}

// reversed pass setup: drift band per pair and the lane width it runs at.
// Every alignment of score score1 in the reversed region starts at the
// reversed corner (T1 leaves no other cell of that value there).  A path
// that drifts d diagonals off the corner's diagonal holds at least d gap
// symbols, so score1 <= smax*min(qend+1, rend+1) - o - (d-1)e: d <= G'.
// When the drift is towards the query (i - j = d) those d symbols are
// insertions, which also leave at most qend+1-d rows for matches:
// score1 <= smax*(qend+1-d) - o - (d-1)e, so d <= Gq =
// (smax*(qend+1) - o + e - score1) / (smax + e); towards the reference
// likewise with rend+1 (Gr).  band = max(min(G', Gq), min(G', Gr)) bounds
// both sides, band_q = min(G', Gq) the query side (e > 0; with e == 0 no band
// is used).
__device__ __forceinline__ int64_t rev_drift(int64_t num, int64_t den) {
  const int64_t g = num / den;
  return g < 0 ? 0 : (g > (1 << 30) ? (1 << 30) : g);
}

__global__ void k_rev_prepare(int64_t n, const int32_t *score, const int32_t *qend,
                              const int64_t *rend, const uint8_t *lanebits, int32_t smax,
                              int32_t o, int32_t e, int32_t *band, int32_t *band_q, uint8_t *f16,
                              uint8_t *f32) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const bool ok = score[p] > 0;
  int32_t b = 0, bq = 0;
  if (ok) {
    if (e > 0) {
      const int64_t rows = (int64_t)qend[p] + 1, cols = rend[p] + 1;
      const int64_t base = -(int64_t)o + e - score[p];
      const int64_t g = rev_drift((int64_t)smax * (rows < cols ? rows : cols) + base, e);
      int64_t gq = rev_drift((int64_t)smax * rows + base, (int64_t)smax + e);
      int64_t gr = rev_drift((int64_t)smax * cols + base, (int64_t)smax + e);
      gq = gq < g ? gq : g;
      gr = gr < g ? gr : g;
      b = (int32_t)(gq > gr ? gq : gr);
      bq = (int32_t)gq;
    } else {
      b = bq = -1;
    }
  }
  band[p] = b;
  band_q[p] = bq;
  f16[p] = (ok && lanebits[p] == 16) ? 1 : 0;
  f32[p] = (ok && lanebits[p] == 32) ? 1 : 0;
}

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Eager sorts go by digit passes (onesweep) at every size: rocprim's default
// sorts up to 2^20 items by block sorts and about ten merge passes instead,
// which took ~0.2 ms per sort of 10^6 pairs (two kernels per merge pass).
// Both are stable, so the order is the same.  Sorts recorded into a graph
// take the merge form at every size: onesweep clears its lookback states with
// a memset, which must not become a graph node.
using OnesweepConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                  rocprim::default_config, 0>;
using MergeConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                               rocprim::default_config, SIZE_MAX>;

template <class K, class V>
static hipError_t radix_pairs(bool graph, void *tmp, size_t &bytes, rocprim::double_buffer<K> &kb,
                              rocprim::double_buffer<V> &vb, size_t n, unsigned end_bit,
                              hipStream_t st) {
  if (graph) return rocprim::radix_sort_pairs<MergeConfig>(tmp, bytes, kb, vb, n, 0u, end_bit, st);
  return rocprim::radix_sort_pairs<OnesweepConfig>(tmp, bytes, kb, vb, n, 0u, end_bit, st);
}

hipError_t count_classes(int64_t n, const uint8_t *cls, int64_t *counts, hipStream_t st) {
  if (!n) return hipSuccess;
  unsigned blocks = nb(n, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_count_classes, dim3(blocks), dim3(256), 0, st, n, cls, counts);
  return hipGetLastError();
}

hipError_t sort_keys(int64_t n, uint64_t *keys, uint64_t *keys_alt, int64_t *vals,
                     int64_t *vals_alt, void *tmp, size_t *tmp_bytes, int64_t **sorted_out,
                     hipStream_t st, int end_bit, bool graph) {
  rocprim::double_buffer<uint64_t> kb(keys, keys_alt);
  rocprim::double_buffer<int64_t> vb(vals, vals_alt);
  hipError_t e = radix_pairs(graph, tmp, *tmp_bytes, kb, vb, (size_t)n, (unsigned)end_bit, st);
  if (tmp) *sorted_out = vb.current();
  return e;
}

hipError_t rev_prepare(int64_t npairs, const int32_t *score, const int32_t *qend,
                       const int64_t *rend, const uint8_t *lanebits, int32_t smax, int32_t o,
                       int32_t e, int32_t *band, int32_t *band_q, uint8_t *f16, uint8_t *f32,
                       hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_rev_prepare, dim3(nb(npairs, 256)), dim3(256), 0, st, npairs, score, qend,
                     rend, lanebits, smax, o, e, band, band_q, f16, f32);
  return hipGetLastError();
}

hipError_t plan_sort(int64_t n, const int64_t *n_dev, const int64_t *ids, const int32_t *qlen,
                     const int64_t *rlen, const int32_t *band, int32_t R, uint64_t *keys,
                     uint64_t *keys_alt, int64_t *vals, int64_t *vals_alt, void *tmp,
                     size_t *tmp_bytes, int64_t **sorted_out, hipStream_t st, bool graph) {
  // without a band the top field is zero: sort the low 44 bits only.  The
  // size query covers both bit ranges, so one buffer serves either pass.
  const int end_bit = band ? 64 : 44;
  if (tmp == nullptr) {
    rocprim::double_buffer<uint64_t> kb(keys, keys_alt);
    rocprim::double_buffer<int64_t> vb(vals, vals_alt);
    size_t b44 = 0, b64 = 0;
    hipError_t e = radix_pairs(graph, nullptr, b44, kb, vb, (size_t)n, 44u, st);
    if (e == hipSuccess) e = radix_pairs(graph, nullptr, b64, kb, vb, (size_t)n, 64u, st);
    *tmp_bytes = b44 > b64 ? b44 : b64;
    return e;
  }
  if (n == 0) { *sorted_out = vals; return hipSuccess; }
  hipLaunchKernelGGL(k_plan_keys, dim3(nb(n, 256)), dim3(256), 0, st, n, n_dev, ids, qlen, rlen,
                     band, R, keys, vals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  rocprim::double_buffer<uint64_t> kb(keys, keys_alt);
  rocprim::double_buffer<int64_t> vb(vals, vals_alt);
  e = radix_pairs(graph, tmp, *tmp_bytes, kb, vb, (size_t)n, (unsigned)end_bit, st);
  *sorted_out = vb.current();
  return e;
}

hipError_t plan_tasks_dev(int64_t n, const int64_t *n_dev, int64_t ntasks, int32_t slots, int32_t R,
                          int64_t qdata_per_row, const int64_t *sorted, const int32_t *qlen,
                          const int64_t *rlen, const int32_t *band, const int32_t *band_q,
                          InterTask *tasks, int64_t *bnd_size, int64_t *qdata_size,
                          hipStream_t st) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_tasks, dim3(nb(ntasks, 4)), dim3(256), 0, st, n, n_dev, ntasks,
                     slots, R, qdata_per_row, sorted, qlen, rlen, band, band_q, tasks, bnd_size,
                     qdata_size);
  return hipGetLastError();
}

hipError_t plan_offsets_dev(int64_t ntasks, InterTask *tasks, const int64_t *bnd_off,
                            const int64_t *qdata_off, hipStream_t st) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_offsets, dim3(nb(ntasks, 128)), dim3(128), 0, st, ntasks, tasks,
                     bnd_off, qdata_off);
  return hipGetLastError();
}

hipError_t flags_to_i64(int64_t n, const uint8_t *flag, int64_t *f64, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_to_i64, dim3(nb(n + 1, 256)), dim3(256), 0, st, n, flag, f64);
  return hipGetLastError();
}

hipError_t compact_flags(int64_t n, const uint8_t *flag, const int64_t *pos, int64_t *out,
                         hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3(nb(n, 256)), dim3(256), 0, st, n, flag, pos, out);
  return hipGetLastError();
}

// ---- plain fills (graph-capturable in place of memset nodes) ------------------
__global__ void k_fill_u8(int64_t n, uint8_t *p, uint8_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void k_fill_i64(int64_t n, int64_t *p, int64_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

hipError_t fill_u8(int64_t n, uint8_t *p, uint8_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(nb(n, 256)), dim3(256), 0, st, n, p, v);
  return hipGetLastError();
}

hipError_t fill_i64(int64_t n, int64_t *p, int64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(nb(n, 256)), dim3(256), 0, st, n, p, v);
  return hipGetLastError();
}

// ranges[2c], ranges[2c+1]: positions of class c in the class-sorted list
__global__ void k_class_ranges(const int64_t *counts, int64_t *ranges) {
  if (threadIdx.x != 0) return;
  int64_t pos = 0;
  for (int c = 0; c < 8; ++c) {
    ranges[2 * c] = pos;
    pos += counts[c];
    ranges[2 * c + 1] = pos;
  }
}

hipError_t class_ranges(const int64_t *counts, int64_t *ranges, hipStream_t st) {
  hipLaunchKernelGGL(k_class_ranges, dim3(1), dim3(64), 0, st, counts, ranges);
  return hipGetLastError();
}

}  // namespace swx
