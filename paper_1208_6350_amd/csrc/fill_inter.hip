// fill_inter.hip -- inter-sequence Smith-Waterman-Gotoh fill.
//
// Computes, for many pairs at once, the local-alignment matrix
//   H(i,j) = max(0, H(i-1,j-1) + S(q_i,r_j), E(i,j), F(i,j))
//   E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o),  F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)
// (paper, Introduction and method section "Algorithm and implementation"),
// the per-column max array of the method section, and the end cell of the
// best alignment under rule T1 (smallest column, then smallest row).
//
// Layout: one wave per task of up to 128 pairs (16-bit lanes, two pairs per
// lane) or 64 pairs (32-bit lanes).  Pairs of a task are padded to common
// dimensions (qp rows, rp columns).  Forward passes pad at the top and left:
// padding rows/columns score <= 0 against everything, so they compute H = 0
// and leave the real cells untouched.  Reversed passes pad at the bottom and
// right instead so that all pairs share the start corner and the band.
//
// Each lane walks the matrix in strips of R rows.  For each column of a strip
// the lane keeps H and E of its R rows in registers and receives H and F of
// the row above from the boundary planes written by the previous strip; the
// whole cell update is 11 saturating 16-bit-pair instructions plus two for
// the column max with the row code (value * 32 + code, so that a max over the
// strip also names the first row reaching it).
//
// Scores live in a biased domain: the substitution term arrives as
// S + bias >= 0 (bias = -min S), E and F are kept as E + bias and F + bias
// floored at 0 by saturating subtraction, and H is recovered with one
// saturating subtraction of the bias, which also applies the zero floor.
#include <hip/hip_runtime.h>

#include "lanes.h"
#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

constexpr int64_t kNoReach = INT64_MAX / 4;

__device__ __forceinline__ int64_t wave_max64(int64_t v) {
  for (int off = 32; off >= 1; off >>= 1) {
    int64_t o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

template <class V, int R, uint32_t MODE>
__device__ __forceinline__ void load_scores(const InterArgs &a, const InterTask &tk, int s, int lane,
                                            const uint32_t *s_lut, uint32_t symA, uint32_t symB,
                                            uint32_t (&X)[R / 4][2]) {
  using T = VT<V>;
  if constexpr (MODE == kQSel) {
    // column LUTs: the same dword pair serves every row
    X[0][0] = s_lut[symA];
    X[0][1] = (T::kHalves == 2) ? s_lut[symB] : 0u;
  } else {
    const int np1 = a.n + 1;
    const uint8_t *base = a.prof + tk.qdata_off;
    const int64_t strip = (int64_t)s * np1 * T::kHalves * 64 * R;
    const uint4 *pA = (const uint4 *)(base + strip + (((int64_t)symA * T::kHalves + 0) * 64 + lane) * R);
#pragma unroll
    for (int k = 0; k < R / 16; ++k) {
      uint4 v = pA[k];
      X[4 * k + 0][0] = v.x; X[4 * k + 1][0] = v.y; X[4 * k + 2][0] = v.z; X[4 * k + 3][0] = v.w;
    }
    if constexpr (T::kHalves == 2) {
      const uint4 *pB = (const uint4 *)(base + strip + (((int64_t)symB * 2 + 1) * 64 + lane) * R);
#pragma unroll
      for (int k = 0; k < R / 16; ++k) {
        uint4 v = pB[k];
        X[4 * k + 0][1] = v.x; X[4 * k + 1][1] = v.y; X[4 * k + 2][1] = v.z; X[4 * k + 3][1] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < R / 4; ++k) X[k][1] = 0u;
    }
  }
}

template <class V, int R, uint32_t MODE>
__global__ __launch_bounds__(256) void k_inter_fill(InterArgs a) {
  using T = VT<V>;
  constexpr int NH = T::kHalves;
  __shared__ uint32_t s_lut[8];
  if (threadIdx.x < 8) s_lut[threadIdx.x] = a.lut[threadIdx.x];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int64_t tid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tid >= a.ntasks) return;
  const InterTask tk = a.tasks[tid];
  const bool rev = a.rev != 0;
  const int nstrips = tk.qp / R;
  const int64_t rp = tk.rp;

  // slots of this lane
  int64_t pid[NH];
  int32_t padq[NH];
  int64_t padr[NH];
  int32_t tgt[NH];
  int64_t reach[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int s = lane + 64 * h;
    pid[h] = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
    if (pid[h] >= 0) {
      const int32_t lq = a.view.qlen[pid[h]];
      const int64_t lr = a.view.rlen[pid[h]];
      padq[h] = rev ? 0 : tk.qp - lq;
      padr[h] = rev ? 0 : rp - lr;
      tgt[h] = rev ? a.target[pid[h]] : 0;
      reach[h] = (rev && tgt[h] <= 0) ? -1 : kNoReach;
    } else {
      padq[h] = 0; padr[h] = 0; tgt[h] = 0; reach[h] = -1;
    }
  }
  int32_t bval[NH], brow[NH];
  int64_t bcol[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) { bval[h] = 0; brow[h] = -1; bcol[h] = -1; }

  uint32_t *bH = a.bnd + tk.bnd_off;
  uint32_t *bF = bH + rp * 64;
  uint32_t *bC = bF + rp * 64;
  const uint4 *sym = a.rsym + tk.sym_off;
  const V vbias = T::splat((uint32_t)a.bias);
  const V vo = T::splat((uint32_t)a.o);
  const V ve = T::splat((uint32_t)a.e);

  int64_t plo = 0, phi = 0;  // column window of the previous strip
  for (int s = 0; s < nstrips; ++s) {
    const int sR = s * R;
    int64_t clo = 0, chi = rp;
    if (rev) {
      if (tk.band >= 0) {
        clo = sR - tk.band; if (clo < 0) clo = 0;
        const int64_t c2 = (int64_t)sR + R + tk.band;
        if (c2 < chi) chi = c2;
      }
      int64_t bound = -1;
#pragma unroll
      for (int h = 0; h < NH; ++h) bound = bound > reach[h] ? bound : reach[h];
      bound = wave_max64(bound);
      if (bound < kNoReach && bound + 1 < chi) chi = bound + 1;
      if (clo >= chi) break;   // later strips have even later windows
    }

    uint32_t sel[R];
    if constexpr (MODE == kQSel) {
#pragma unroll
      for (int r = 0; r < R; ++r) sel[r] = a.qsel[tk.qdata_off + (int64_t)(sR + r) * 64 + lane];
    }

    V H[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = T::zero(); E[r] = T::zero(); }
    V hdtop = T::zero();
    if (s > 0 && clo >= 1 && clo - 1 >= plo && clo - 1 < phi)
      hdtop = T::from(bH[(clo - 1) * 64 + lane]);
    uint32_t sb[NH];
    int64_t sbcol[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) { sb[h] = 0u; sbcol[h] = -1; }
    const bool last = (s == nstrips - 1);

    for (int64_t c = clo; c < chi; ++c) {
      const bool inprev = (s > 0) && (c >= plo) && (c < phi);
      const int64_t bi = c * 64 + lane;
      V hup = inprev ? T::from(bH[bi]) : T::zero();
      V F = inprev ? T::from(bF[bi]) : T::zero();
      V cmin = (!rev && s > 0) ? T::from(bC[bi]) : T::zero();

      const uint4 sy = sym[(c >> 3) * 64 + lane];
      const int sh = (int)(c & 3) * 8;
      const uint32_t wA = (c & 4) ? sy.y : sy.x;
      const uint32_t wB = (c & 4) ? sy.w : sy.z;
      const uint32_t symA = (wA >> sh) & 0xFFu;
      const uint32_t symB = (wB >> sh) & 0xFFu;
      uint32_t X[R / 4][2];
      load_scores<V, R, MODE>(a, tk, s, lane, s_lut, symA, symB, X);

      V hdiag = hdtop;
      hdtop = hup;
      V cm = T::zero();
      V ho = T::zero();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t sraw;
        if constexpr (MODE == kQSel) sraw = perm(X[0][1], X[0][0], sel[r]);
        else sraw = perm(X[r >> 2][1], X[r >> 2][0], T::sel_const(r & 3));
        const V t = T::add(hdiag, T::from(sraw));
        hdiag = H[r];
        const V hb = T::max(T::max(t, E[r]), F);
        const V hn = T::subs(hb, vbias);
        H[r] = hn;
        cm = T::max(cm, T::enc(hn, T::code_splat((uint32_t)(R - 1 - r))));
        ho = T::subs(hb, vo);
        E[r] = T::max(T::subs(E[r], ve), ho);
        F = T::max(T::subs(F, ve), ho);   // F of the next row
      }
      if (!last || rev) {
        bH[bi] = T::bits(H[R - 1]);
        bF[bi] = T::bits(F);
      }
      if (!rev) bC[bi] = T::bits(T::max(cmin, T::shr5(cm)));
      // strip best: first column reaching the strip's largest value
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const uint32_t v = T::half(cm, h);
        if ((v | 31u) > (sb[h] | 31u)) { sb[h] = v; sbcol[h] = c; }
      }
    }
    // merge the strip best into the pair best (earlier strips win ties)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int32_t v = (int32_t)(sb[h] >> 5);
      if (v > 0) {
        const int32_t row = sR + (R - 1 - (int32_t)(sb[h] & 31u)) - padq[h];
        const int64_t col = sbcol[h] - padr[h];
        if (v > bval[h] || (v == bval[h] && col < bcol[h])) {
          bval[h] = v; brow[h] = row; bcol[h] = col;
        }
        if (rev && v >= tgt[h] && sbcol[h] < reach[h]) reach[h] = sbcol[h];
      }
    }
    plo = clo;
    phi = chi;
  }

  constexpr int32_t limit = (NH == 2) ? kInter16Limit : (1 << 26) - 1;
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    if (pid[h] < 0) continue;
    const int64_t p = pid[h];
    a.out.score[p] = bval[h];
    a.out.qend[p] = bval[h] > 0 ? brow[h] : -1;
    a.out.rend[p] = bval[h] > 0 ? bcol[h] : -1;
    a.out.overflow[p] = (bval[h] >= limit) ? 1 : 0;
  }
}

// ---- packing: reference symbols, QSEL row selectors, QGEN profiles ------
// Reference symbols of a task: uint4 per (8 columns, lane): bytes 0-7 hold
// the low-half pair's symbols, bytes 8-15 the high-half pair's.  Padding
// columns carry the pad symbol `pad`.


__device__ __forceinline__ int32_t ref_sym(const PackArgs &a, int64_t p, int64_t c, int64_t rp) {
  if (p < 0) return -1;
  const int64_t lr = a.view.rlen[p];
  int64_t j = a.rev ? c : c - (rp - lr);
  if (j < 0 || j >= lr) return -1;
  const int64_t idx = a.view.reversed ? a.view.rstart[p] + lr - 1 - j : a.view.rstart[p] + j;
  return a.view.rcat[idx];
}

__device__ __forceinline__ int32_t qry_sym(const PackArgs &a, int64_t p, int64_t ip, int32_t qp) {
  if (p < 0) return -1;
  const int32_t lq = a.view.qlen[p];
  int64_t i = a.rev ? ip : ip - (qp - lq);
  if (i < 0 || i >= lq) return -1;
  const int64_t idx = a.view.reversed ? a.view.qstart[p] + lq - 1 - i : a.view.qstart[p] + i;
  return a.view.qcat[idx];
}

__global__ __launch_bounds__(256) void k_inter_pack(PackArgs a) {
  const int64_t t = blockIdx.x;
  if (t >= a.ntasks) return;
  const InterTask tk = a.tasks[t];
  const int pad = a.n;   // pad symbol code
  // reference symbols
  const int64_t nblk = tk.rp / 8;
  for (int64_t k = threadIdx.x; k < nblk * 64; k += blockDim.x) {
    const int lane = (int)(k & 63);
    const int64_t blk = k >> 6;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int h = 0; h < a.halves; ++h) {
      const int s = lane + 64 * h;
      const int64_t p = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
      for (int cc = 0; cc < 8; ++cc) {
        int32_t v = ref_sym(a, p, blk * 8 + cc, tk.rp);
        uint32_t b = (uint32_t)(v < 0 ? pad : v) & 0xFFu;
        w[2 * h + (cc >> 2)] |= b << ((cc & 3) * 8);
      }
    }
    a.rsym[tk.sym_off + k] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  if (a.mode == (int)kQSel) {
    for (int64_t k = threadIdx.x; k < (int64_t)tk.qp * 64; k += blockDim.x) {
      const int lane = (int)(k & 63);
      const int64_t ip = k >> 6;
      uint32_t sel = 0x0C0C0C0Cu;
      for (int h = 0; h < a.halves; ++h) {
        const int s = lane + 64 * h;
        const int64_t p = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
        const int32_t v = qry_sym(a, p, ip, tk.qp);
        const uint32_t b = (v < 0) ? 0x0Cu : (uint32_t)v + 4u * h;
        sel = (sel & ~(0xFFu << (16 * h))) | (b << (16 * h));
      }
      a.qsel[tk.qdata_off + k] = sel;
    }
  } else {
    const int R = a.strip_rows;
    const int np1 = a.n + 1;
    const int64_t total = (int64_t)tk.qp * np1 * a.halves * 64;
    for (int64_t k = threadIdx.x; k < total; k += blockDim.x) {
      // k enumerates (strip, symbol, half, lane, row-in-strip) with the row fastest
      const int r = (int)(k % R);
      int64_t rest = k / R;
      const int lane = (int)(rest % 64); rest /= 64;
      const int h = (int)(rest % a.halves); rest /= a.halves;
      const int sy = (int)(rest % np1);
      const int64_t strip = rest / np1;
      const int s = lane + 64 * h;
      const int64_t p = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
      const int32_t qv = qry_sym(a, p, strip * R + r, tk.qp);
      uint8_t b = 0;
      if (qv >= 0 && sy < a.n) b = (uint8_t)(a.matrix[qv * a.n + sy] + a.bias);
      a.prof[tk.qdata_off + k] = b;
    }
  }
}

// ---- host-side launchers ------------------------------------------------
template <class V, int R, uint32_t MODE>
static hipError_t launch_fill(const InterArgs &a, hipStream_t st) {
  const int waves_per_block = 4;
  const int64_t blocks = (a.ntasks + waves_per_block - 1) / waves_per_block;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_inter_fill<V, R, MODE>), dim3((unsigned)blocks), dim3(64 * waves_per_block),
                     0, st, a);
  return hipGetLastError();
}

hipError_t inter_fill(const InterArgs &a, int lane_bits, int R, hipStream_t st) {
  const uint32_t mode = a.qsel ? kQSel : kQGen;
  if (lane_bits == 16) {
    if (R == 32) return mode == kQSel ? launch_fill<u16x2, 32, kQSel>(a, st)
                                      : launch_fill<u16x2, 32, kQGen>(a, st);
    if (R == 16) return mode == kQSel ? launch_fill<u16x2, 16, kQSel>(a, st)
                                      : launch_fill<u16x2, 16, kQGen>(a, st);
  } else {
    if (R == 32) return mode == kQSel ? launch_fill<uint32_t, 32, kQSel>(a, st)
                                      : launch_fill<uint32_t, 32, kQGen>(a, st);
    if (R == 16) return mode == kQSel ? launch_fill<uint32_t, 16, kQSel>(a, st)
                                      : launch_fill<uint32_t, 16, kQGen>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t inter_pack(const PackArgs &a, hipStream_t st) {
  if (a.ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inter_pack, dim3((unsigned)a.ntasks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace swx
