// aux_kernels.hip -- the steps of the method after the forward fill:
//   * pair views (forward, and reversed prefixes for the begin search),
//   * the banded global DP and traceback that produce the CIGAR
//     (method section: "the banded SW (whose band is defined by the beginning
//     and ending positions) generates the detailed alignment"),
//   * the suboptimal score from the masked max array (method section, (2);
//     Figure 1 caption),
//   * CIGAR compaction and result records.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_scan.hpp>

#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

// ---- pair views -----------------------------------------------------------
// Views of the pairs.  Every index and range is clamped into the arrays
// (pair indices into [0, nq) and [0, nr), a sequence into its code array, its
// length to the caps): input that the validation kernel flags still drives
// every later kernel inside its buffers, where a caller's device buffers
// (the graph's) are checked only by that kernel, in the same launch order.
__global__ void k_views(int64_t npairs, const int64_t *qoff, const int64_t *roff,
                        const int64_t *pair_q, const int64_t *pair_r, ViewCaps caps,
                        int64_t *qstart, int32_t *qlen, int64_t *rstart, int64_t *rlen) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  auto clamp = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
  const int64_t qi = clamp(pair_q[p], 0, caps.nq - 1), ri = clamp(pair_r[p], 0, caps.nr - 1);
  const int64_t q0 = clamp(qoff[qi], 0, caps.qcat_len);
  const int64_t q1 = clamp(qoff[qi + 1], q0, caps.qcat_len);
  const int64_t r0 = clamp(roff[ri], 0, caps.rcat_len);
  const int64_t r1 = clamp(roff[ri + 1], r0, caps.rcat_len);
  qstart[p] = q0;
  qlen[p] = (int32_t)(q1 - q0 < caps.max_qlen ? q1 - q0 : caps.max_qlen);
  rstart[p] = r0;
  rlen[p] = r1 - r0 < caps.max_rlen ? r1 - r0 : caps.max_rlen;
}

// Reversed prefixes q[0..qend] and r[0..rend] (read backwards by the fill).
__global__ void k_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                            const int32_t *qlen, const int64_t *rlen,
                            const int32_t *score, const int32_t *qend, const int64_t *rend,
                            int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                            int32_t *target, uint8_t *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  bool ok = score[p] > 0;
  if (ok && (qend[p] < 0 || qend[p] >= qlen[p] || rend[p] < 0 || rend[p] >= rlen[p])) {
    err[p] = 1;   // an end outside the pair: never read past the sequences
    ok = false;
  }
  rqstart[p] = qstart[p];
  rrstart[p] = rstart[p];
  rqlen[p] = ok ? qend[p] + 1 : 0;
  rrlen[p] = ok ? rend[p] + 1 : 0;
  target[p] = ok ? score[p] : 0;
}

// ---- banded global DP and traceback (one thread per pair) ------------------
// Safe band: with m = qend-qbeg+1, w = rend-rbeg+1, D = w - m and
//   G = floor((smax*(m+w) - 2o + 2e - 2*score1) / (smax + 2e)),
// every path of score score1 has at most G gap symbols, so it stays on the
// diagonals min(0,D) - hw .. max(0,D) + hw with hw = floor((G - |D|)/2).
// Inside the band the DP values on such paths equal the unbanded ones, so the
// traceback (rule T3: M, then D, then I; open before extend) is the same.
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ void band_of(int64_t m, int64_t w, int64_t score1, int32_t smax,
                                        int32_t o, int32_t e, int64_t *dlo, int64_t *dhi) {
  const int64_t D = w - m;
  const int64_t num = (int64_t)smax * (m + w) - 2 * o + 2 * e - 2 * score1;
  const int64_t den = (int64_t)smax + 2 * e;
  const int64_t G = den > 0 ? floor_div(num, den) : (m + w);
  const int64_t aD = D < 0 ? -D : D;
  int64_t hw = (G - aD) >= 0 ? (G - aD) / 2 : 0;
  *dlo = (D < 0 ? D : 0) - hw;
  *dhi = (D > 0 ? D : 0) + hw;
}

__device__ __forceinline__ bool coords_ok(int64_t p, const int32_t *qbeg, const int32_t *qend,
                                          const int64_t *rbeg, const int64_t *rend,
                                          const int32_t *qlen, const int64_t *rlen) {
  return qbeg[p] >= 0 && qbeg[p] <= qend[p] && qend[p] < qlen[p] && rbeg[p] >= 0 &&
         rbeg[p] <= rend[p] && rend[p] < rlen[p];
}

__global__ void k_band_sizes(int64_t npairs, const int32_t *score, const int32_t *qbeg,
                             const int32_t *qend, const int64_t *rbeg, const int64_t *rend,
                             const int32_t *qlen, const int64_t *rlen, const uint8_t *only,
                             int32_t smax, int32_t o, int32_t e, int64_t *dir_size,
                             int64_t *cig_cap, int64_t *row_cap) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  if (score[p] <= 0 || (only && only[p] != 5) || !coords_ok(p, qbeg, qend, rbeg, rend, qlen, rlen)) {
    dir_size[p] = 0; cig_cap[p] = 0; row_cap[p] = 0; return;
  }
  const int64_t m = qend[p] - qbeg[p] + 1, w = rend[p] - rbeg[p] + 1;
  int64_t dlo, dhi;
  band_of(m, w, score[p], smax, o, e, &dlo, &dhi);
  const int64_t bw = dhi - dlo + 1;
  dir_size[p] = (m + 1) * bw;
  cig_cap[p] = m + w + 2;
  row_cap[p] = bw + 2;
}



constexpr int32_t kNegInf = -(1 << 29);

__global__ void k_band_tb(BandArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npairs) return;
  const int32_t s1 = a.score[p];
  if (a.only && a.only[p] != 5) return;
  if (s1 <= 0) { a.cig_len[p] = 0; return; }
  if (!coords_ok(p, a.qbeg, a.qend, a.rbeg, a.rend, a.qlen, a.rlen)) {
    a.cig_len[p] = 0;
    a.err[p] = 1;
    return;
  }
  const int64_t qb = a.qbeg[p], qe = a.qend[p], rb = a.rbeg[p], re = a.rend[p];
  const int64_t m = qe - qb + 1, w = re - rb + 1;
  int64_t dlo, dhi;
  band_of(m, w, s1, a.smax, a.o, a.e, &dlo, &dhi);
  const int64_t bw = dhi - dlo + 1;
  uint8_t *dir = a.dir + a.dir_off[p];
  int32_t *hrow = a.rowbuf + 2 * a.row_off[p];      // H of the previous row, by band index
  int32_t *frow = hrow + (bw + 2);                   // F of the previous row
  const int8_t *q = a.qcat + a.qstart[p] + qb;
  const int8_t *r = a.rcat + a.rstart[p] + rb;
  const int32_t o = a.o, e = a.e;
  // band index k = j - i - dlo; row i covers j in [max(0, i+dlo), min(w, i+dhi)]
  // row 0
  for (int64_t k = 0; k < bw; ++k) { hrow[k] = kNegInf; frow[k] = kNegInf; }
  {
    int32_t ev = kNegInf;
    const int64_t jhi = dhi < w ? dhi : w;
    for (int64_t j = 0; j <= jhi; ++j) {
      const int64_t k = j - dlo;
      if (j == 0) { hrow[k] = 0; dir[k] = 0; continue; }
      const int32_t open = hrow[k - 1] - o, ext = ev - e;
      ev = open > ext ? open : ext;
      hrow[k] = ev;
      dir[k] = (uint8_t)(1 | (open >= ext ? 4 : 0));
    }
  }
  for (int64_t i = 1; i <= m; ++i) {
    const int64_t jlo = (i + dlo) > 0 ? (i + dlo) : 0;
    const int64_t jhi = (i + dhi) < w ? (i + dhi) : w;
    uint8_t *drow = dir + i * bw;
    int32_t ev = kNegInf;        // E(i, j-1)
    int32_t hleft = kNegInf;     // H(i, j-1)
    // the previous row's entries are read at band index k (diag) and k+1 (up);
    // they are overwritten in place at index k after use
    for (int64_t j = jlo; j <= jhi; ++j) {
      const int64_t k = j - i - dlo;
      const int32_t hup = (k + 1 < bw) ? hrow[k + 1] : kNegInf;
      const int32_t fup = (k + 1 < bw) ? frow[k + 1] : kNegInf;
      const int32_t hdg = hrow[k];
      const int32_t fopen = hup - o, fext = fup - e;
      const int32_t fij = fopen > fext ? fopen : fext;
      int32_t h, c;
      if (j == 0) {
        h = fij;
        c = 2 | (fopen >= fext ? 8 : 0);
        ev = kNegInf;
      } else {
        const int32_t eopen = hleft - o, eext = ev - e;
        const int32_t eij = eopen > eext ? eopen : eext;
        const int32_t diag = hdg + a.matrix[q[i - 1] * a.n + r[j - 1]];
        h = diag;
        if (eij > h) h = eij;
        if (fij > h) h = fij;
        c = (h == diag) ? 0 : (h == eij ? 1 : 2);
        if (eopen >= eext) c |= 4;
        if (fopen >= fext) c |= 8;
        ev = eij;
      }
      drow[k] = (uint8_t)c;
      hrow[k] = h;
      frow[k] = fij;
      hleft = h;
    }
    // cells of the previous row outside this row's range must not leak
    // into the next row: the next row reads indices k and k+1 for its j
    for (int64_t k = 0; k < bw; ++k) {
      const int64_t j = i + dlo + k;
      if (j < jlo || j > jhi) { hrow[k] = kNegInf; frow[k] = kNegInf; }
    }
  }
  // global optimum check: H(m, w)
  const int32_t hend = hrow[w - m - dlo];
  if (hend != s1) a.err[p] = 1;
  // traceback from (m, w) in state H, runs written end -> begin then reversed
  uint32_t *out = a.cig + a.cig_off[p];
  int32_t nruns = 0;
  int64_t i = m, j = w;
  int state = 0;
  uint32_t cur_op = 0xFF, cur_len = 0;
  int64_t guard = 2 * (m + w) + 4;
  while ((i > 0 || j > 0) && guard-- > 0) {
    const int64_t k = j - i - dlo;
    if (k < 0 || k >= bw) { a.err[p] = 1; break; }
    const uint8_t c = dir[i * bw + k];
    uint32_t op = 0xFF;
    if (state == 0) {
      const int src = c & 3;
      if (src == 0 && i > 0 && j > 0) { op = 0; --i; --j; }
      else if (src == 1) state = 1;
      else state = 2;
    } else if (state == 1) {
      op = 2;
      state = (c & 4) ? 0 : 1;
      --j;
    } else {
      op = 1;
      state = (c & 8) ? 0 : 2;
      --i;
    }
    if (op != 0xFF) {
      if (op == cur_op) ++cur_len;
      else {
        if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
        cur_op = op; cur_len = 1;
      }
    }
  }
  if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
  for (int32_t x = 0, y = nruns - 1; x < y; ++x, --y) {
    uint32_t t = out[x]; out[x] = out[y]; out[y] = t;
  }
  a.cig_len[p] = nruns;
}

// ---- CIGAR compaction -----------------------------------------------------
// 16 lanes per pair (most CIGARs have few runs), 16 pairs per block
__global__ void k_cigar_compact(int64_t npairs, const uint32_t *src, const int64_t *src_off,
                                const int32_t *len, const int64_t *dst_off, uint32_t *dst) {
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16;
  if (p >= npairs) return;
  const int32_t n = len[p];
  const int64_t so = src_off[p], d = dst_off[p];
  for (int32_t k = threadIdx.x & 15; k < n; k += 16) dst[d + k] = src[so + k];
}

// ---- score2 on inter tasks (max array = final CM plane) -------------------


__global__ __launch_bounds__(256) void k_score2_inter(Score2InterArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t tid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tid >= a.ntasks) return;
  const InterTask tk = a.tasks[tid];
  const uint32_t *bC = a.bnd + tk.bnd_off + 2 * (int64_t)tk.rp * 64;
  // a lane owns slots lane and lane + 64 (16-bit halves of one word): both
  // scans share one pass over the plane
  int64_t pr[2], lr[2], padr[2], lo[2], hi[2], at[2];
  int32_t best[2];
  int64_t gfirst = tk.rp / 4;
  for (int h = 0; h < 2; ++h) {
    const int s = lane + 64 * h;
    pr[h] = (h < a.halves && s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
    best[h] = 0;
    at[h] = -1;
    lr[h] = 0;
    padr[h] = tk.rp;
    lo[h] = hi[h] = 0;
    if (pr[h] >= 0 && a.score1[pr[h]] > 0) {
      const int64_t p = pr[h];
      lr[h] = a.rlen[p];
      padr[h] = tk.rp - lr[h];
      int64_t m = a.mask_len;
      if (m < 0) { m = a.qlen[p] / 2; if (m < 15) m = 15; }
      lo[h] = a.rbeg[p] - m;
      hi[h] = a.rend[p] + m;
      gfirst = min(gfirst, padr[h] / 4);
    }
  }
  // the plane holds 4 columns per 16-byte word: 4 words (16 columns) are
  // read at a time, all in flight together, and scanned in column order
  const uint4 *w4 = reinterpret_cast<const uint4 *>(bC);
  const int64_t gend = tk.rp / 4;
  for (int64_t g0 = gfirst; g0 < gend; g0 += 4) {
    uint4 wd[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) wd[u] = w4[min(g0 + u, gend - 1) * 64 + lane];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t ws[4] = {wd[u].x, wd[u].y, wd[u].z, wd[u].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t c = 4 * (g0 + u) + k;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t j = c - padr[h];
          const bool in = g0 + u < gend && j >= 0 && j < lr[h] && (j < lo[h] || j > hi[h]);
          const int32_t v = (a.halves == 2) ? (int32_t)(h ? (ws[k] >> 16) : (ws[k] & 0xFFFFu))
                                            : (int32_t)ws[k];
          if (in && v > best[h]) { best[h] = v; at[h] = j; }
        }
      }
    }
  }
  for (int h = 0; h < 2; ++h) {
    if (pr[h] < 0) continue;
    a.score2[pr[h]] = best[h];
    a.rend2[pr[h]] = best[h] > 0 ? at[h] : -1;
  }
}

// score2 on a plain per-pair max array (long pairs)
__global__ void k_score2_plain(int64_t p, const int32_t *maxcol, int64_t lr, const int32_t *score1,
                               const int64_t *rbeg, const int64_t *rend, int32_t mask_len,
                               const int32_t *qlen, int32_t *score2, int64_t *rend2) {
  __shared__ int32_t sv[256];
  __shared__ int64_t sj[256];
  int32_t best = 0;
  int64_t at = INT64_MAX;
  if (score1[p] > 0) {
    int64_t m = mask_len;
    if (m < 0) { m = qlen[p] / 2; if (m < 15) m = 15; }
    const int64_t lo = rbeg[p] - m, hi = rend[p] + m;
    for (int64_t j = threadIdx.x; j < lr; j += blockDim.x) {
      if (j >= lo && j <= hi) continue;
      const int32_t v = maxcol[j];
      if (v > best) { best = v; at = j; }
    }
  }
  sv[threadIdx.x] = best;
  sj[threadIdx.x] = at;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const int32_t v2 = sv[threadIdx.x + off];
      const int64_t j2 = sj[threadIdx.x + off];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && j2 < sj[threadIdx.x])) {
        sv[threadIdx.x] = v2; sj[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    score2[p] = sv[0];
    rend2[p] = sv[0] > 0 ? sj[0] : -1;
  }
}

// ---- result records -------------------------------------------------------
__global__ void k_records(int64_t npairs, const int32_t *score1, const int32_t *score2,
                          const int32_t *qbeg, const int32_t *qend, const int64_t *rbeg,
                          const int64_t *rend, const int64_t *rend2, const int64_t *cig_off,
                          const int32_t *cig_len, const uint8_t *lane_bits, uint32_t flags,
                          swx_rec_dev *recs) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  swx_rec_dev r;
  const bool ok = score1[p] > 0;
  const bool beg = (flags & 1u) && ok;
  r.score1 = score1[p];
  r.score2 = (ok && (flags & 4u)) ? score2[p] : 0;
  r.read_begin1 = beg ? qbeg[p] : -1;
  r.read_end1 = ok ? qend[p] : -1;
  r.ref_begin1 = beg ? rbeg[p] : -1;
  r.ref_end1 = ok ? rend[p] : -1;
  r.ref_end2 = (ok && (flags & 4u)) ? rend2[p] : -1;
  r.cigar_off = (ok && (flags & 2u)) ? cig_off[p] : 0;
  r.cigar_len = (ok && (flags & 2u)) ? cig_len[p] : 0;
  r.lane_bits = lane_bits[p];
  recs[p] = r;
}

// begin coordinates from the reversed pass: begin = end - reversed end
__global__ void k_begins(int64_t npairs, const int32_t *score1, const int32_t *qend,
                         const int64_t *rend, const int32_t *rscore, const int32_t *rqend,
                         const int64_t *rrend, int32_t *qbeg, int64_t *rbeg, uint8_t *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  if (score1[p] <= 0) { qbeg[p] = -1; rbeg[p] = -1; return; }
  if (rscore[p] != score1[p]) err[p] = 1;
  qbeg[p] = qend[p] - rqend[p];
  rbeg[p] = rend[p] - rrend[p];
}

// ---- input validation -------------------------------------------------------
// Any byte of p[0, len) outside [0, n), 1 <= n <= 32.  The 16-byte-aligned
// body is read in 16-byte words and tested four bytes at a time: a byte b is
// bad when its top bit is set (negative) or when (b & 0x7F) + 128 - n reaches
// 128 (no carry leaves the byte, since 127 + 127 < 256).
__device__ __forceinline__ bool symbols_bad(const int8_t *p, int64_t len, int32_t n, int64_t tid,
                                            int64_t stride) {
  const uint32_t add = (uint32_t)(128 - n) * 0x01010101u;
  const int64_t head = (int64_t)((16 - ((uintptr_t)p & 15)) & 15);
  const int64_t h = head < len ? head : len;
  const int64_t nw = (len - h) / 16;
  bool bad = false;
  for (int64_t k = tid; k < h; k += stride) bad |= p[k] < 0 || p[k] >= n;
  const uint4 *w = reinterpret_cast<const uint4 *>(p + h);
  for (int64_t k = tid; k < nw; k += stride) {
    const uint4 v = w[k];
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) bad |= ((x[i] | ((x[i] & 0x7F7F7F7Fu) + add)) & 0x80808080u) != 0;
  }
  for (int64_t k = h + 16 * nw + tid; k < len; k += stride) bad |= p[k] < 0 || p[k] >= n;
  return bad;
}

__global__ void k_validate(ValidateArgs a) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (int64_t k = tid; k <= a.nq; k += stride) {
    const int64_t v = a.qoff[k];
    if (v < 0 || v > a.qcat_len || (k > 0 && a.qoff[k - 1] > v)) bad |= 1u;
  }
  for (int64_t k = tid; k <= a.nr; k += stride) {
    const int64_t v = a.roff[k];
    if (v < 0 || v > a.rcat_len || (k > 0 && a.roff[k - 1] > v)) bad |= 1u;
  }
  for (int64_t k = tid; k < a.npairs; k += stride) {
    if (a.pair_q[k] < 0 || a.pair_q[k] >= a.nq || a.pair_r[k] < 0 || a.pair_r[k] >= a.nr) bad |= 2u;
  }
  if (symbols_bad(a.qcat, a.qcat_len, a.n, tid, stride)) bad |= 4u;
  if (symbols_bad(a.rcat, a.rcat_len, a.n, tid, stride)) bad |= 8u;
  if (bad) atomicOr(a.bad, bad);
}

// ---- small helpers ------------------------------------------------------------
// stats[0] = max over pairs of min(qlen, rlen); stats[1] = sum of qlen * rlen
__global__ void k_pair_stats(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t *stats) {
  int64_t best = 0, cells = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int64_t m = qlen[p] < rlen[p] ? qlen[p] : rlen[p];
    best = m > best ? m : best;
    cells += (int64_t)qlen[p] * rlen[p];
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
    cells += __shfl_xor(cells, off, 64);
  }
  // one pair of atomics per block, not per wave: they all meet at two words
  __shared__ int64_t s_best[4], s_cells[4];
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) { s_best[wv] = best; s_cells[wv] = cells; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      best = s_best[k] > best ? s_best[k] : best;
      cells += s_cells[k];
    }
    if (best > 0) atomicMax((unsigned long long *)&stats[0], (unsigned long long)best);
    if (cells > 0) atomicAdd((unsigned long long *)&stats[1], (unsigned long long)cells);
  }
}

__global__ void k_lens_to_i64(int64_t n, const int32_t *len, int64_t *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = len[p];
}

__global__ void k_mark_lanes(int64_t n, const int64_t *n_dev, const int64_t *ids, uint8_t *lanebits,
                             uint8_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n_dev) n = *n_dev;
  if (k < n) lanebits[ids[k]] = v;
}

__global__ void k_any_flag(int64_t n, const uint8_t *flag, int64_t *count) {
  int64_t c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    c += flag[p] ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd((unsigned long long *)count, (unsigned long long)c);
}

// ---- launchers --------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_pair_stats(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t *stats,
                             hipStream_t st) {
  if (!n) return hipSuccess;
  unsigned b = blocks_for(n, 256);
  if (b > 256) b = 256;
  hipLaunchKernelGGL(k_pair_stats, dim3(b), dim3(256), 0, st, n, qlen, rlen, stats);
  return hipGetLastError();
}

hipError_t lens_to_i64(int64_t n, const int32_t *len, int64_t *out, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_lens_to_i64, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, len, out);
  return hipGetLastError();
}

hipError_t mark_lanes(int64_t n, const int64_t *ids, uint8_t *lanebits, int v, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mark_lanes, dim3(blocks_for(n, 256)), dim3(256), 0, st, n,
                     (const int64_t *)nullptr, ids, lanebits, (uint8_t)v);
  return hipGetLastError();
}

hipError_t mark_lanes_dev(int64_t cap, const int64_t *n_dev, const int64_t *ids, uint8_t *lanebits,
                          int v, hipStream_t st) {
  if (!cap) return hipSuccess;
  hipLaunchKernelGGL(k_mark_lanes, dim3(blocks_for(cap, 256)), dim3(256), 0, st, cap, n_dev, ids,
                     lanebits, (uint8_t)v);
  return hipGetLastError();
}

hipError_t launch_any_flag(int64_t n, const uint8_t *flag, int64_t *count, hipStream_t st) {
  if (!n) return hipSuccess;
  unsigned b = blocks_for(n, 256);
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_any_flag, dim3(b), dim3(256), 0, st, n, flag, count);
  return hipGetLastError();
}

// ---- the query profile of one query (method section: built once per query) --
// fwd[sym][x], x in [0, qp): the biased score S(q[x - pad], sym) + bias, with
// pad = qp - qlen rows on top scoring 0 (and every byte of sym == n, the
// padding symbol, 0), laid out as the batched fill's forward strips read it.
// rev[c][sym][k], c in [0, 16), k in [0, rev_row): the biased score of query
// position qlen - 1 - (k + c), 0 for k + c >= qlen (the reversed pass's
// padding rows at the bottom): copy c serves rows that start c bytes past a
// 16-byte boundary.
__global__ void k_build_qprof(const int8_t *q, int32_t qlen, const int8_t *matrix, int32_t n,
                              int32_t bias, int32_t qp, uint8_t *fwd, int64_t rev_row,
                              uint8_t *rev) {
  const int64_t nf = (int64_t)(n + 1) * qp;
  const int64_t nr = 16 * (int64_t)(n + 1) * rev_row;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nf + nr; k += stride) {
    int64_t i;
    int32_t sym;
    if (k < nf) {
      sym = (int32_t)(k / qp);
      i = k % qp - (qp - qlen);
    } else {
      const int64_t u = k - nf;
      const int64_t c = u / ((int64_t)(n + 1) * rev_row);
      const int64_t rest = u % ((int64_t)(n + 1) * rev_row);
      sym = (int32_t)(rest / rev_row);
      const int64_t pos = rest % rev_row + c;
      i = pos < qlen ? qlen - 1 - pos : -1;
    }
    uint8_t b = 0;
    if (sym < n && i >= 0 && i < qlen) {
      const int32_t qc = q[i];
      if (qc >= 0 && qc < n) b = (uint8_t)(matrix[qc * n + sym] + bias);   // codes checked before
    }
    if (k < nf) fwd[k] = b;
    else rev[k - nf] = b;
  }
}

hipError_t build_qprof(const int8_t *q, int32_t qlen, const int8_t *matrix, int32_t n, int32_t bias,
                       int32_t qp, uint8_t *fwd, int64_t rev_row, uint8_t *rev, hipStream_t st) {
  const int64_t total = (int64_t)(n + 1) * qp + 16 * (int64_t)(n + 1) * rev_row;
  unsigned b = blocks_for(total, 256);
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_build_qprof, dim3(b), dim3(256), 0, st, q, qlen, matrix, n, bias, qp, fwd,
                     rev_row, rev);
  return hipGetLastError();
}

hipError_t launch_validate(const ValidateArgs &a, hipStream_t st) {
  const int64_t work = a.qcat_len + a.rcat_len + a.npairs + a.nq + a.nr + 2;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                                 size_t *tmp_bytes, hipStream_t st) {
  return rocprim::exclusive_scan(tmp, *tmp_bytes, in, out, (int64_t)0, (size_t)n,
                                 rocprim::plus<int64_t>(), st);
}

hipError_t launch_views(int64_t npairs, const int64_t *qoff, const int64_t *roff,
                        const int64_t *pair_q, const int64_t *pair_r, const ViewCaps &caps,
                        int64_t *qstart, int32_t *qlen, int64_t *rstart, int64_t *rlen,
                        hipStream_t st) {
  if (!npairs) return hipSuccess;
  if (caps.nq < 1 || caps.nr < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_views, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, qoff, roff,
                     pair_q, pair_r, caps, qstart, qlen, rstart, rlen);
  return hipGetLastError();
}

hipError_t launch_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                            const int32_t *qlen, const int64_t *rlen,
                            const int32_t *score, const int32_t *qend, const int64_t *rend,
                            int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                            int32_t *target, uint8_t *err, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_rev_views, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, qstart,
                     rstart, qlen, rlen, score, qend, rend, rqstart, rqlen, rrstart, rrlen, target,
                     err);
  return hipGetLastError();
}

hipError_t launch_band_sizes(int64_t npairs, const int32_t *score, const int32_t *qbeg,
                             const int32_t *qend, const int64_t *rbeg, const int64_t *rend,
                             const int32_t *qlen, const int64_t *rlen, const uint8_t *only,
                             int32_t smax, int32_t o, int32_t e, int64_t *dir_size,
                             int64_t *cig_cap, int64_t *row_cap, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_band_sizes, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, score,
                     qbeg, qend, rbeg, rend, qlen, rlen, only, smax, o, e, dir_size, cig_cap,
                     row_cap);
  return hipGetLastError();
}

hipError_t launch_band_tb(const BandArgs &a, hipStream_t st) {
  if (!a.npairs) return hipSuccess;
  hipLaunchKernelGGL(k_band_tb, dim3(blocks_for(a.npairs, 64)), dim3(64), 0, st, a);
  return hipGetLastError();
}

// the CIGAR of pair 0 of a one-pair call: its final offsets (0 and its
// length) and its words, in one launch
__global__ void k_cigar_one(const uint32_t *src, const int64_t *src_off, const int32_t *len,
                            int64_t *dst_off, uint32_t *dst) {
  const int32_t n = len[0];
  if (threadIdx.x == 0) {
    dst_off[0] = 0;
    dst_off[1] = n;
  }
  const int64_t so = src_off[0];
  for (int32_t k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[so + k];
}

hipError_t cigar_one(const uint32_t *src, const int64_t *src_off, const int32_t *len,
                     int64_t *dst_off, uint32_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_cigar_one, dim3(1), dim3(256), 0, st, src, src_off, len, dst_off, dst);
  return hipGetLastError();
}

// Clears of many buffers in one launch (graph capture records no memset):
// entry k sets f.n[k] elements of f.size[k] bytes at f.p[k] to f.v[k].
__global__ void k_fill_set(FillSet f) {
  const int64_t gs = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < f.count; ++k) {
    const int64_t n = f.n[k];
    if (f.size[k] == 1) {
      uint8_t *q = static_cast<uint8_t *>(f.p[k]);
      for (int64_t i = gt; i < n; i += gs) q[i] = (uint8_t)f.v[k];
    } else if (f.size[k] == 4) {
      uint32_t *q = static_cast<uint32_t *>(f.p[k]);
      for (int64_t i = gt; i < n; i += gs) q[i] = (uint32_t)f.v[k];
    } else {
      int64_t *q = static_cast<int64_t *>(f.p[k]);
      for (int64_t i = gt; i < n; i += gs) q[i] = f.v[k];
    }
  }
}

hipError_t fill_set(const FillSet &f, hipStream_t st) {
  if (f.count < 0 || f.count > kFillSetMax) return hipErrorInvalidValue;
  if (f.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_set, dim3(64), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_cigar_compact(int64_t npairs, const uint32_t *src, const int64_t *src_off,
                                const int32_t *len, const int64_t *dst_off, uint32_t *dst,
                                hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_cigar_compact, dim3(blocks_for(npairs, 16)), dim3(256), 0, st, npairs, src,
                     src_off, len, dst_off, dst);
  return hipGetLastError();
}

hipError_t launch_score2_inter(const Score2InterArgs &a, hipStream_t st) {
  if (!a.ntasks) return hipSuccess;
  hipLaunchKernelGGL(k_score2_inter, dim3(blocks_for(a.ntasks, 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_score2_plain(int64_t p, const int32_t *maxcol, int64_t lr, const int32_t *score1,
                               const int64_t *rbeg, const int64_t *rend, int32_t mask_len,
                               const int32_t *qlen, int32_t *score2, int64_t *rend2,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_score2_plain, dim3(1), dim3(256), 0, st, p, maxcol, lr, score1, rbeg, rend,
                     mask_len, qlen, score2, rend2);
  return hipGetLastError();
}

hipError_t launch_records(int64_t npairs, const int32_t *score1, const int32_t *score2,
                          const int32_t *qbeg, const int32_t *qend, const int64_t *rbeg,
                          const int64_t *rend, const int64_t *rend2, const int64_t *cig_off,
                          const int32_t *cig_len, const uint8_t *lane_bits, uint32_t flags,
                          swx_rec_dev *recs, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_records, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, score1,
                     score2, qbeg, qend, rbeg, rend, rend2, cig_off, cig_len, lane_bits, flags,
                     recs);
  return hipGetLastError();
}

// ---- the suboptimal alignment (the one behind score2) -------------------------
// Step 1: a window of the reference ending at ref_end2 that holds every
// positive-scoring path into that column (no such path spans more than
// W = Lq + (smax*Lq - o)/e + 1 columns; with e = 0 the whole prefix), so the
// forward recurrence started there is exact at the window's last column.
__global__ void k_sub_window(int64_t npairs, const int64_t *rstart, const int32_t *qlen,
                             const int32_t *score2, const int64_t *rend2, int32_t smax, int32_t o,
                             int32_t e, int64_t *wrstart, int64_t *wrlen, uint8_t *flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const bool ok = score2[p] > 0 && rend2[p] >= 0;
  int64_t lo = 0;
  if (ok && e > 0) {
    const int64_t lq = qlen[p];
    const int64_t span = lq + ((int64_t)smax * lq - o) / e + 1;
    lo = rend2[p] - span + 1;
    if (lo < 0) lo = 0;
  }
  wrstart[p] = rstart[p] + (ok ? lo : 0);
  wrlen[p] = ok ? rend2[p] - lo + 1 : 0;
  flag[p] = ok ? 1 : 0;
}

// Step 2: the anchored reversed pass from (end row, ref_end2): reversed
// prefixes, target anchor + score2; pairs whose window pass did not reproduce
// score2 at its last column are flagged as inconsistent.
__global__ void k_sub_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                                const int32_t *qlen, const int32_t *score2, const int64_t *rend2,
                                const int32_t *wscore, const int32_t *wqend, uint32_t anchor,
                                int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                                int32_t *target, uint8_t *flag, uint8_t *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  bool ok = score2[p] > 0 && rend2[p] >= 0;
  if (ok && (wscore[p] != score2[p] || wqend[p] < 0 || wqend[p] >= qlen[p])) {
    err[p] = 1;
    ok = false;
  }
  rqstart[p] = qstart[p];
  rrstart[p] = rstart[p];
  rqlen[p] = ok ? wqend[p] + 1 : 0;
  rrlen[p] = ok ? rend2[p] + 1 : 0;
  target[p] = ok ? (int32_t)(anchor + (uint32_t)score2[p]) : 0;
  flag[p] = ok ? 1 : 0;
}

// Step 3: begin = end - reversed end; the suboptimal record's arrays.
__global__ void k_sub_begins(int64_t npairs, const int32_t *score2, const int64_t *rend2,
                             const int32_t *wqend, const uint8_t *flag, const int32_t *target,
                             const int32_t *rscore, const int32_t *rqend, const int64_t *rrend,
                             int32_t *sscore, int32_t *sqbeg, int32_t *sqend, int64_t *srbeg,
                             int64_t *srend, uint8_t *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const bool ok = flag[p] != 0;
  if (ok && rscore[p] != target[p]) err[p] = 1;
  sscore[p] = ok ? score2[p] : 0;
  sqend[p] = ok ? wqend[p] : -1;
  srend[p] = ok ? rend2[p] : -1;
  sqbeg[p] = ok ? wqend[p] - rqend[p] : -1;
  srbeg[p] = ok ? rend2[p] - rrend[p] : -1;
}

// records' CIGAR offsets counted from the arena's start
__global__ void k_shift_cigar_offsets(int64_t npairs, int64_t base, swx_rec_dev *recs) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  if (recs[p].cigar_len > 0) recs[p].cigar_off += base;
}

hipError_t launch_sub_window(int64_t npairs, const int64_t *rstart, const int32_t *qlen,
                             const int32_t *score2, const int64_t *rend2, int32_t smax, int32_t o,
                             int32_t e, int64_t *wrstart, int64_t *wrlen, uint8_t *flag,
                             hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_sub_window, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, rstart,
                     qlen, score2, rend2, smax, o, e, wrstart, wrlen, flag);
  return hipGetLastError();
}

hipError_t launch_sub_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                                const int32_t *qlen, const int32_t *score2, const int64_t *rend2,
                                const int32_t *wscore, const int32_t *wqend, uint32_t anchor,
                                int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                                int32_t *target, uint8_t *flag, uint8_t *err, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_sub_rev_views, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs,
                     qstart, rstart, qlen, score2, rend2, wscore, wqend, anchor, rqstart, rqlen,
                     rrstart, rrlen, target, flag, err);
  return hipGetLastError();
}

hipError_t launch_sub_begins(int64_t npairs, const int32_t *score2, const int64_t *rend2,
                             const int32_t *wqend, const uint8_t *flag, const int32_t *target,
                             const int32_t *rscore, const int32_t *rqend, const int64_t *rrend,
                             int32_t *sscore, int32_t *sqbeg, int32_t *sqend, int64_t *srbeg,
                             int64_t *srend, uint8_t *err, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_sub_begins, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, score2,
                     rend2, wqend, flag, target, rscore, rqend, rrend, sscore, sqbeg, sqend, srbeg,
                     srend, err);
  return hipGetLastError();
}

hipError_t shift_cigar_offsets(int64_t npairs, int64_t base, swx_rec_dev *recs, hipStream_t st) {
  if (!npairs || !base) return hipSuccess;
  hipLaunchKernelGGL(k_shift_cigar_offsets, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs,
                     base, recs);
  return hipGetLastError();
}

hipError_t launch_begins(int64_t npairs, const int32_t *score1, const int32_t *qend,
                         const int64_t *rend, const int32_t *rscore, const int32_t *rqend,
                         const int64_t *rrend, int32_t *qbeg, int64_t *rbeg, uint8_t *err,
                         hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_begins, dim3(blocks_for(npairs, 256)), dim3(256), 0, st, npairs, score1,
                     qend, rend, rscore, rqend, rrend, qbeg, rbeg, err);
  return hipGetLastError();
}

// ---- long/short split and small gathers for the intra-sequence path -------
__global__ void k_split_long(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t cells_thr,
                             int64_t rlen_thr, uint8_t *is_long, uint8_t *is_short) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const bool lg = (int64_t)qlen[p] * rlen[p] > cells_thr || rlen[p] > rlen_thr;
  is_long[p] = lg ? 1 : 0;
  is_short[p] = lg ? 0 : 1;
}

// out[6k + f]: qlen, rlen, score, qend, rend, band of pair ids[k] (0 for null arrays)
__global__ void k_gather_pairs(int64_t n, const int64_t *ids, const int32_t *qlen,
                               const int64_t *rlen, const int32_t *score, const int32_t *qend,
                               const int64_t *rend, const int32_t *band, int64_t *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t p = ids[k];
  out[6 * k + 0] = qlen ? qlen[p] : 0;
  out[6 * k + 1] = rlen ? rlen[p] : 0;
  out[6 * k + 2] = score ? score[p] : 0;
  out[6 * k + 3] = qend ? qend[p] : 0;
  out[6 * k + 4] = rend ? rend[p] : 0;
  out[6 * k + 5] = band ? band[p] : 0;
}

__global__ void k_clear_flags(int64_t n, const int64_t *ids, uint8_t *f1, uint8_t *f2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  f1[ids[k]] = 0;
  f2[ids[k]] = 0;
}

hipError_t split_long(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t cells_thr,
                      int64_t rlen_thr, uint8_t *is_long, uint8_t *is_short, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_split_long, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, qlen, rlen,
                     cells_thr, rlen_thr, is_long, is_short);
  return hipGetLastError();
}

hipError_t gather_pairs(int64_t n, const int64_t *ids, const int32_t *qlen, const int64_t *rlen,
                        const int32_t *score, const int32_t *qend, const int64_t *rend,
                        const int32_t *band, int64_t *out, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_gather_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, ids, qlen,
                     rlen, score, qend, rend, band, out);
  return hipGetLastError();
}

hipError_t clear_flags(int64_t n, const int64_t *ids, uint8_t *f1, uint8_t *f2, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_clear_flags, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, ids, f1, f2);
  return hipGetLastError();
}

}  // namespace swx
