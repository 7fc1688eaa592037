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
// cell update is 9 saturating 16-bit-pair instructions plus two for the
// column max with the row code (value * 32 + code, so that a max over the
// strip also names the first row reaching it; one and a half when rows go in
// pairs, see kColPair), one fewer when the bias is the gap open penalty.
// Boundary planes and the reference symbols (packed per task by k_inter_rsym,
// padding included) move in groups of 4 columns: one 16-byte word per lane
// and plane.
//
// Scores live in a biased domain: the substitution term arrives as
// S + bias >= 0 (bias >= -min S), E and F are kept as E + bias and F + bias
// floored at 0 by saturating subtraction, and H is recovered with one
// saturating subtraction of the bias, which also applies the zero floor.
// When the bias equals o, that same subtraction is the H - o that opens a
// gap (a candidate below zero is raised to zero, i.e. to -bias: gap values
// at or below zero never decide a cell, whose H is at least zero).
#include <hip/hip_runtime.h>

#include <type_traits>

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

// A sequence as seen by one lane-half: padded index i maps to symbol
// base[i - pad] (forward) or base[len - 1 - (i - pad)] (reversed view).
// base is always readable at index 0 (a dummy buffer for empty slots), so
// every access below is a plain load from a clamped index.
struct SeqRef {
  const int8_t *base;
  int64_t len;
  int64_t pad;
  bool rev;
};

__device__ __forceinline__ SeqRef make_seq(const int8_t *base, int64_t len, int64_t pad, bool rev,
                                           const int8_t *dummy) {
  return SeqRef{len > 0 ? base : dummy, len, pad, rev};
}

__device__ __forceinline__ int32_t seq_at(const SeqRef &s, int64_t i) {
  const int64_t j = i - s.pad;
  const bool ok = (uint64_t)j < (uint64_t)s.len;
  const int64_t idx = ok ? (s.rev ? s.len - 1 - j : j) : 0;
  const int32_t v = s.base[idx];
  return ok ? v : -1;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int k) {
  return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// Register budget: 256 VGPRs per lane (two waves per SIMD) for 32-row strips,
// 168 (three waves) for shorter strips.
template <int R> constexpr int fill_waves() { return R >= 32 ? 2 : 3; }

// Shared state of a cooperative task: the four waves of a workgroup take the
// strips of one task round robin, strip s starting on a column group once
// strip s - 1 has stored that group of the boundary planes (in place: every
// strip reads a group before it writes it, in strip order).
struct CoopShared {
  int32_t prog[kCoopMaxStrips];            // strip s stored groups [0, prog & ~bit31); bit 31: done
  int64_t reach[kSlots16];                 // reversed pass: earliest column reaching the target
  int32_t mval[kCoopWaves][kSlots16];      // per-wave partial results, merged at the end
  int32_t mrow[kCoopWaves][kSlots16];
  int64_t mcol[kCoopWaves][kSlots16];
  int64_t task;                            // queued scheduling: the workgroup's task
};
constexpr int32_t kStripDone = (int32_t)0x80000000u;
constexpr int64_t kCoopSpinLimit = int64_t(1) << 26;

// How a 16-bit fill keeps a column's maximum (value * 32 + row code): one
// max per row, the same after clamping the value to the field's top (scores
// of the launch may pass it), or one packed three-way maximum per two rows
// (every encoded value of the launch below 0x7C00).  32-bit lanes use the
// first.
enum : int { kColPlain = 0, kColClamp = 1, kColPair = 2 };
// Form of a fill kernel: the column maximum's form, plus kFormHo when the
// launch's bias equals o (H and H - o are then one value).
constexpr int kFormHo = 4;

// One task (up to 64 or 128 pairs) on one wave: every strip, column group by
// column group.  tid is uniform across the wave, so the task and everything
// derived from it (bounds, plane addresses) live in SGPRs.
template <class V, int R, uint32_t MODE, int FORM, bool REV, bool COOP>
__device__ __forceinline__ void inter_task(const InterArgs &a, const int64_t tid,
                                           const uint32_t *s_lut, CoopShared *cs, int wave) {
  using T = VT<V>;
  constexpr int NH = T::kHalves;
  constexpr int COL = FORM & 3;
  constexpr bool HO = (FORM & kFormHo) != 0;
  const int lane = threadIdx.x & 63;
  const InterTask tk = a.tasks[tid];
  if (tk.nslots == 0) return;   // an empty task of a fixed-capacity plan (uniform per workgroup)
  constexpr bool rev = REV;
  const int nstrips = (tk.qp + R - 1) / R;
  // cooperative task: this wave's strips are s_first, s_first + s_step, ...
  constexpr bool coop = COOP;
  const bool sync = coop && nstrips <= kCoopMaxStrips;
  int s_first = 0, s_step = 1, s_end = nstrips;
  if (sync) {
    s_first = wave;
    s_step = kCoopWaves;
  } else if (coop && wave != 0) {
    s_end = 0;   // too many strips to pipeline: wave 0 takes the whole task
  }
  bool spin_fail = false;
  // forward passes only: the last strip has R / 2 rows (a reversed pass,
  // padded at the bottom, runs its last strip full: the extra rows are padding)
  const bool half_tail = !REV && (tk.qp % R) != 0;
  const int64_t rp = tk.rp;

  // slots of this lane
  int64_t pid[NH];
  SeqRef qs[NH];
  int64_t rpad[NH];
  int32_t tgt[NH];
  int64_t reach[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int s = lane + 64 * h;
    pid[h] = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
    if (pid[h] >= 0) {
      const int64_t p = pid[h];
      const int32_t lq = a.view.qlen[p];
      qs[h] = make_seq(a.view.qcat + a.view.qstart[p], lq, rev ? 0 : tk.qp - lq,
                       a.view.reversed != 0, a.dummy);
      rpad[h] = rev ? 0 : rp - a.view.rlen[p];
      tgt[h] = rev ? a.target[p] : 0;
      reach[h] = (rev && tgt[h] <= 0) ? -1 : kNoReach;
    } else {
      qs[h] = SeqRef{a.dummy, 0, 0, false};
      rpad[h] = 0;
      tgt[h] = 0;
      reach[h] = -1;
    }
  }
  int32_t bval[NH], brow[NH];
  int64_t bcol[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) { bval[h] = 0; brow[h] = -1; bcol[h] = -1; }

  // boundary planes: [rp/4][64] 16-byte words each
  uint4 *bH = reinterpret_cast<uint4 *>(a.bnd + tk.bnd_off);
  uint4 *bF = bH + rp * 16;
  uint4 *bC = bF + rp * 16;
  const uint2 *rsym = a.rsym + rsym_offset(tk.bnd_off);
  const V vbias = T::splat((uint32_t)a.bias);
  const uint32_t code_top = (uint32_t)a.code_top;   // R - 1, opaque to the compiler
  // the row-code multiplier (32 in each half) in a VGPR the compiler cannot
  // see through, so value * 32 + code stays one v_pk_mad_u16
  uint32_t mul32;
  asm volatile("v_mov_b32 %0, %1" : "=v"(mul32) : "s"(0x00200020u));
  const V vtop = T::splat((uint32_t)kInter16Limit);   // the value field's top (16-bit lanes)
  const V vo = T::splat((uint32_t)a.o);
  const V ve = T::splat((uint32_t)a.e);
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);

  int64_t plo = 0, phi = 0;  // column window of the previous strip (multiples of 4)
  for (int s = s_first; s < s_end; s += s_step) {
    const int sR = s * R;
    // cooperative: progress of strip s - 1 (groups known stored; done)
    int32_t avail = 0;
    bool pdone = (s == 0);
    auto wait_prev = [&](int64_t g) {
      if (!sync || pdone || g < avail) return;
      int64_t spins = 0;
      for (;;) {
        const int32_t v = __hip_atomic_load(&cs->prog[s - 1], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
        avail = v & ~kStripDone;
        pdone = (v & kStripDone) != 0;
        if (pdone || g < avail) break;
        if (++spins > kCoopSpinLimit) {   // never expected: fail the task's pairs, go on
          spin_fail = true;
          pdone = true;
          avail = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    auto publish = [&](int64_t groups, bool fin) {
      if (!sync) return;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0)
        __hip_atomic_store(&cs->prog[s], (int32_t)groups | (fin ? kStripDone : 0),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    int64_t clo = 0, chi = rp;
    if (rev) {
      if (sync) {   // earliest columns reached by strips above, as far as known now
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int64_t r = __hip_atomic_load(&cs->reach[lane + 64 * h], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
          if (r < reach[h]) reach[h] = r;
        }
        // the previous strip's window start (its end comes with its progress)
        plo = 0;
        if (s > 0 && tk.band >= 0) {
          plo = (int64_t)(s - 1) * R - tk.band_q;
          if (plo < 0) plo = 0;
          plo &= ~(int64_t)3;
        }
      }
      if (tk.band >= 0) {
        clo = sR - tk.band_q; if (clo < 0) clo = 0;
        const int64_t c2 = (int64_t)sR + R + tk.band;
        if (c2 < chi) chi = c2;
      }
      int64_t bound = -1;
#pragma unroll
      for (int h = 0; h < NH; ++h) bound = bound > reach[h] ? bound : reach[h];
      bound = wave_max64(bound);
      if (bound < kNoReach && bound + 1 < chi) chi = bound + 1;
      // whole column groups: a wider window only adds cells whose values are
      // lower bounds of the true ones (an exact band stays exact)
      clo &= ~(int64_t)3;
      chi = (chi + 3) & ~(int64_t)3;
      if (chi > rp) chi = rp;
      if (clo >= chi) {   // later strips have even later windows
        if (!sync) break;
        publish(0, true);   // nothing stored: the strip below reads zeros
        continue;
      }
    }

    // per-row byte selectors (QSEL): query symbol of each half, 0x0C = pad
    uint32_t sel[R];
    if constexpr (MODE == kQSel) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t w = 0x0C0C0C0Cu;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int32_t qv = seq_at(qs[h], sR + r);
          const uint32_t b = (qv < 0 || qv >= a.n) ? 0x0Cu : (uint32_t)qv + 4u * h;
          w = (w & ~(0xFFu << (16 * h))) | (b << (16 * h));
        }
        sel[r] = w;
      }
    }

    V H[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = T::zero(); E[r] = T::zero(); }
    V hdtop = T::zero();
    if (sync && s > 0 && clo >= 1) {
      wait_prev((clo - 1) >> 2);
      if (clo - 1 >= plo && ((clo - 1) >> 2) < avail)
        hdtop = T::from(reinterpret_cast<const uint32_t *>(bH)[bnd_index(clo - 1, lane)]);
    } else if (s > 0 && clo >= 1 && clo - 1 >= plo && clo - 1 < phi) {
      hdtop = T::from(reinterpret_cast<const uint32_t *>(bH)[bnd_index(clo - 1, lane)]);
    }
    // anchored reversed pass: the corner before the first cell holds
    // `anchor` and the row above the first row the gap run that leaves it;
    // every other border starts from zero, far below, so only alignments that
    // leave the corner (forward: end in the anchor cell, possibly with a
    // deletion run) reach anchor + target
    if (REV && NH == 1 && s == 0 && a.anchor) hdtop = T::splat(a.anchor);
    uint32_t sb[NH];      // encoded strip best (value * 32 + row code)
    uint32_t sbk[NH];     // sb | 31: its value part, for the strict comparison
    int32_t sbcol[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) { sb[h] = 0u; sbk[h] = 31u; sbcol[h] = -1; }
    const bool last = (s == nstrips - 1);
    const bool half = last && half_tail;

    // Column groups of 4.  The boundary words and reference symbols of group
    // g+1 are requested before group g is computed, so the loads overlap four
    // columns of arithmetic.
    int64_t cdone = chi;   // one past the last column this strip computes
    const int64_t g0 = clo >> 2, g1 = chi >> 2;
    uint4 nh, nf, nc;
    uint2 nsy;
    auto fetch_group = [&](int64_t g) {
      // forward strips all span every column, so only the first strip lacks a
      // row above; reversed strips use column windows.  Cooperative: wait
      // until the strip above has stored the group (or finished short of it).
      bool inprev;
      if (sync) {
        wait_prev(g);
        inprev = (s > 0) && (!rev || 4 * g >= plo) && (g < avail);
      } else {
        inprev = rev ? ((s > 0) && (4 * g >= plo) && (4 * g < phi)) : (s > 0);
      }
      const int64_t gi = g * 64 + lane;
      nsy = rsym[gi];
      nh = inprev ? bH[gi] : zero4;
      nf = inprev ? bF[gi] : zero4;
      nc = (!rev && s > 0) ? bC[gi] : zero4;
    };
    // QGEN: profile words of the next column, one column ahead
    uint32_t nX[R / 4][2];
    // a batch whose pairs share one query reads the query's profile, built
    // once: forward rows sR .. sR + R - 1 of a symbol are contiguous; a
    // reversed pass needs rows from qlen - lq + sR on (lq: the reversed
    // view's height), taken from the copy of the table shifted so that they
    // start on a 16-byte boundary
    int64_t qoffA = 0, qoffB = 0;
    if (a.qprof) {
      if constexpr (REV) {
        const int64_t kA = (int64_t)a.qprof_qlen - qs[0].len + sR;
        qoffA = (kA & 15) * a.qprof_copy + (kA & ~(int64_t)15);
        if constexpr (NH == 2) {
          const int64_t kB = (int64_t)a.qprof_qlen - qs[1].len + sR;
          qoffB = (kB & 15) * a.qprof_copy + (kB & ~(int64_t)15);
        }
      } else {
        qoffA = qoffB = sR;
      }
    }
    auto fetch_prof = [&](uint32_t symA, uint32_t symB) {
      const int np1 = a.n + 1;
      const uint8_t *base = a.prof + tk.qdata_off + (int64_t)s * np1 * NH * 64 * R;
      const uint4 *pA = a.qprof ? (const uint4 *)(a.qprof + symA * a.qprof_row + qoffA)
                                : (const uint4 *)(base + (((int64_t)symA * NH + 0) * 64 + lane) * R);
#pragma unroll
      for (int k = 0; k < R / 16; ++k) {
        const uint4 v = pA[k];
        nX[4 * k + 0][0] = v.x; nX[4 * k + 1][0] = v.y; nX[4 * k + 2][0] = v.z; nX[4 * k + 3][0] = v.w;
      }
      if constexpr (NH == 2) {
        const uint4 *pB = a.qprof ? (const uint4 *)(a.qprof + symB * a.qprof_row + qoffB)
                                  : (const uint4 *)(base + (((int64_t)symB * 2 + 1) * 64 + lane) * R);
#pragma unroll
        for (int k = 0; k < R / 16; ++k) {
          const uint4 v = pB[k];
          nX[4 * k + 0][1] = v.x; nX[4 * k + 1][1] = v.y; nX[4 * k + 2][1] = v.z; nX[4 * k + 3][1] = v.w;
        }
      } else {
#pragma unroll
        for (int k = 0; k < R / 4; ++k) nX[k][1] = 0u;
      }
    };
    fetch_group(g0);
    if constexpr (MODE == kQGen) fetch_prof(nsy.x & 0xFFu, nsy.y & 0xFFu);

    // Forward pass: a group's boundary words are stored one group late,
    // right after the wait for the next group's operands, so that the memory
    // counter never waits for a store issued moments earlier (loads and
    // stores in flight together make every wait a wait for all).  Before the
    // first group the pending words are the first group's own (a write of
    // what was read).  The reversed pass, short of registers, stores at once.
    constexpr bool kDelay = !REV;
    uint4 ph = nh, pf = nf, pc = nc;
    int64_t pgi = g0 * 64 + lane, pghf = pgi;
    auto flush = [&]() {
      bH[pghf] = ph;
      bF[pghf] = pf;
      if (!rev) bC[pgi] = pc;
    };

    // the column groups, computing NR rows per column: R, or R / 2 in a
    // half strip (a second copy of the loop, chosen once per strip)
    auto run_groups = [&](auto nr) {
      constexpr int NR = decltype(nr)::value;
  #pragma unroll 1
      for (int64_t g = g0; g < g1; ++g) {
        // groups before g - 1 are stored (their stores precede the loads of
        // group g, which the release below waits for)
        if (sync && g > g0) publish(g - 1, false);
        const uint4 ch = nh, cf = nf, cc = nc;
        const uint2 sy = nsy;
        if constexpr (kDelay) flush();
        if (g + 1 < g1) fetch_group(g + 1);
        uint32_t lx[4][2];   // QSEL: LUT words of the group's 4 columns
        if constexpr (MODE == kQSel) {
  #pragma unroll
          for (int k = 0; k < 4; ++k) {
            lx[k][0] = s_lut[__builtin_amdgcn_ubfe(sy.x, 8 * k, 8)];
            lx[k][1] = (NH == 2) ? s_lut[__builtin_amdgcn_ubfe(sy.y, 8 * k, 8)] : 0u;
          }
        }
        uint32_t oh[4], of[4], oc[4];
  #pragma unroll
        for (int k = 0; k < 4; ++k) {
          // keep the scheduler from hoisting later columns' score operands
          // (independent of the recurrence) into this one: they would take
          // R registers per column
          __builtin_amdgcn_sched_barrier(0);
          const int64_t c = 4 * g + k;
          uint32_t X[R / 4][2];
          if constexpr (MODE == kQGen) {
  #pragma unroll
            for (int i = 0; i < R / 4; ++i) { X[i][0] = nX[i][0]; X[i][1] = nX[i][1]; }
            if (k < 3) {
              fetch_prof(__builtin_amdgcn_ubfe(sy.x, 8 * (k + 1), 8),
                         __builtin_amdgcn_ubfe(sy.y, 8 * (k + 1), 8));
            } else if (g + 1 < g1) {
              fetch_prof(nsy.x & 0xFFu, nsy.y & 0xFFu);
            }
          } else {
            X[0][0] = lx[k][0];
            X[0][1] = lx[k][1];
          }
          V hup = T::from(word_of(ch, k));
          // anchored reversed pass: the row above the first row is the run of
          // gap symbols that may follow the anchor cell's alignment (a forward
          // alignment may end in a deletion run: its end cell is then in the
          // gap state), H = anchor - o - c*e at column c
          if constexpr (REV && NH == 1) {   // anchored passes run on 32-bit lanes only
            if (s == 0 && a.anchor) {
              const uint32_t gap = (uint32_t)a.o + (uint32_t)c * (uint32_t)a.e;
              hup = T::splat(a.anchor > gap ? a.anchor - gap : 0u);
            }
          }
          const V hdiag_in = hdtop;
          V F = T::from(word_of(cf, k));
          const V cmin = T::from(word_of(cc, k));

          // rows: the part of each cell that does not depend on the F chain
          // (diagonal + substitution) is computed one row ahead
          hdtop = hup;
          V cm = T::zero();
          V enc0 = T::zero();   // paired column maximum: the pair's first row
          V ho = T::zero();
          auto score_of = [&](int r) -> V {
            uint32_t sraw;
            if constexpr (MODE == kQSel) sraw = perm(X[0][1], X[0][0], sel[r]);
            else sraw = perm(X[r >> 2][1], X[r >> 2][0], T::sel_const(r & 3));
            return T::from(sraw);
          };
          V u_next = T::add(hdiag_in, score_of(0));
          static_assert(NR % 2 == 0, "rows come in pairs");
  #pragma unroll
          for (int r = 0; r < NR; ++r) {
            const V u = u_next;
            if (r + 1 < NR) u_next = T::add(H[r], score_of(r + 1));
            // every lane value stays below 0x7C00 unless the pair has passed
            // the 11-bit value field (then it is flagged and re-run wider)
            const V hb = T::max3(u, E[r], F);
            const V hn = T::subs(hb, vbias);
            H[r] = hn;
            const uint32_t code = code_top - (uint32_t)r;
            // scores past the 11-bit value field enter the code as the field's
            // top (the pass is then flagged and re-run wider)
            // (32-bit lanes hold any score beside the code)
            const V enc = T::enc_nosat((COL == kColClamp && NH == 2) ? T::min(hn, vtop) : hn, code, mul32);
            if constexpr (COL == kColPair && NH == 2) {
              // rows in pairs, one packed three-way maximum per pair: every
              // encoded value is below 0x7C00 here (scores of the launch are
              // at most kInter16PairLimit), where it is the unsigned maximum
              if (r & 1) cm = T::max3(cm, enc0, enc);
              else enc0 = enc;
            } else {
              cm = T::max(cm, enc);
            }
            ho = HO ? hn : T::subs(hb, vo);
            E[r] = T::max(T::subs(E[r], ve), ho);
            F = T::max(T::subs(F, ve), ho);   // F of the next row
          }
          oh[k] = T::bits(H[NR - 1]);
          of[k] = T::bits(F);
          oc[k] = T::bits(T::max(cmin, T::shr5(cm)));
          // strip best: first column reaching the strip's largest value
  #pragma unroll
          for (int h = 0; h < NH; ++h) {
            const uint32_t v = T::half(cm, h);
            const uint32_t vk = v | 31u;
            // lastcol (32-bit lanes): only the pair's last column (padded
            // column rp - 1) counts
            const bool imp = vk > sbk[h] && (REV || NH == 2 || !a.lastcol || c == rp - 1);
            sb[h] = imp ? v : sb[h];
            sbk[h] = imp ? vk : sbk[h];
            sbcol[h] = imp ? (int32_t)c : sbcol[h];
          }
        }
        const int64_t gi = g * 64 + lane;
        // the last forward strip has no reader for H and F: it overwrites the
        // first group's words instead (they stay in L2).  A store that is
        // skipped instead costs registers: the compiler splits the loop.
        const int64_t ghf = (last && !rev) ? (int64_t)lane : gi;
        ph = make_uint4(oh[0], oh[1], oh[2], oh[3]);
        pf = make_uint4(of[0], of[1], of[2], of[3]);
        pc = make_uint4(oc[0], oc[1], oc[2], oc[3]);
        pgi = gi;
        pghf = ghf;
        if constexpr (!kDelay) flush();
        if (rev && (g & 1)) {
          // leave the strip once every pair has reached its target at or before
          // the group's last column: later columns can neither give an earlier
          // column nor a smaller row
          int64_t need = -1;
  #pragma unroll
          for (int h = 0; h < NH; ++h) {
            int64_t rr = reach[h];
            if (rr >= 0 && (int32_t)(sb[h] >> 5) >= tgt[h] && sbcol[h] < rr) rr = sbcol[h];
            need = rr > need ? rr : need;
          }
          if (wave_max64(need) <= 4 * g + 4) { cdone = 4 * g + 4; break; }
        }
      }
    };
    if constexpr (MODE == kQSel && !REV) {
      if (half) run_groups(std::integral_constant<int, R / 2>{});
      else run_groups(std::integral_constant<int, R>{});
    } else {
      run_groups(std::integral_constant<int, R>{});
    }
    if constexpr (kDelay) flush();   // the strip's last group, before the next strip reads it
    publish(cdone >> 2, true);
    // merge the strip best into the pair best (earlier strips win ties)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int32_t v = (int32_t)(sb[h] >> 5);
      if (v > 0) {
        const int32_t row = sR + (R - 1 - (int32_t)(sb[h] & 31u)) - (int32_t)qs[h].pad;
        const int64_t col = (int64_t)sbcol[h] - rpad[h];
        if (v > bval[h] || (v == bval[h] && col < bcol[h])) {
          bval[h] = v; brow[h] = row; bcol[h] = col;
        }
        if (rev && v >= tgt[h] && sbcol[h] < reach[h]) {
          reach[h] = sbcol[h];
          if (sync)
            __hip_atomic_fetch_min(&cs->reach[lane + 64 * h], (int64_t)sbcol[h], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    plo = clo;
    phi = cdone;
  }

  if constexpr (coop) {
    // merge the waves' partial results: largest value, then smallest column,
    // then smallest row (the order a single wave's strip-by-strip merge gives)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      cs->mval[wave][lane + 64 * h] = bval[h];
      cs->mrow[wave][lane + 64 * h] = brow[h];
      cs->mcol[wave][lane + 64 * h] = bcol[h];
    }
    if (spin_fail) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
        if (pid[h] >= 0 && a.out.err) a.out.err[pid[h]] = 1;
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        for (int w = 1; w < kCoopWaves; ++w) {
          const int32_t v = cs->mval[w][lane + 64 * h];
          const int32_t r = cs->mrow[w][lane + 64 * h];
          const int64_t c = cs->mcol[w][lane + 64 * h];
          if (v > bval[h] || (v == bval[h] && v > 0 && (c < bcol[h] || (c == bcol[h] && r < brow[h])))) {
            bval[h] = v; brow[h] = r; bcol[h] = c;
          }
        }
      }
    }
    __syncthreads();   // the shared state is reused by the workgroup's next task
    if (wave != 0) return;
  } else if (spin_fail) {
#pragma unroll
    for (int h = 0; h < NH; ++h)
      if (pid[h] >= 0 && a.out.err) a.out.err[pid[h]] = 1;
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

// Task order: tasks are sorted by (band, strips, columns) ascending, so the
// largest come last, or (order) listed by ascending area.  sched 0 runs
// them in that order, 1 largest first, 2 keeps a grid of resident waves that
// take tasks largest first from a device counter (a work queue: one 64-bit
// atomic per task) until it runs past the last task.
template <class V, int R, uint32_t MODE, int FORM, bool REV, bool COOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fill_waves<R>()))) void k_inter_fill(
    InterArgs a) {
  struct NoShared {};
  __shared__ uint32_t s_lut[8];
  __shared__ std::conditional_t<COOP, CoopShared, NoShared> s_coop;
  CoopShared *csp = nullptr;
  if constexpr (COOP) csp = &s_coop;
  if (threadIdx.x < 8) s_lut[threadIdx.x] = a.lut[threadIdx.x];
  __syncthreads();
  const bool queued = a.sched == 2;
  constexpr bool coop = COOP;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // one task per wave, or (cooperative) one task per workgroup
  int64_t k = coop ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  for (;;) {   // one pass unless queued (a single call site keeps one copy of the body)
    if constexpr (coop) {
      if (queued && threadIdx.x == 0) s_coop.task = (int64_t)atomicAdd(a.queue, 1ull);
      for (int i = threadIdx.x; i < kCoopMaxStrips; i += blockDim.x) s_coop.prog[i] = 0;
      for (int i = threadIdx.x; i < kSlots16; i += blockDim.x) s_coop.reach[i] = kNoReach;
      __syncthreads();
      if (queued) k = s_coop.task;
    } else if (queued) {
      unsigned long long t = 0;
      if ((threadIdx.x & 63) == 0) t = atomicAdd(a.queue, 1ull);
      const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t);
      const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(t >> 32));
      k = (int64_t)(((uint64_t)hi << 32) | lo);
    }
    if (k >= a.ntasks) return;   // uniform per workgroup in the cooperative mode
    const int64_t tix = a.sched == 0 ? k : a.ntasks - 1 - k;
    inter_task<V, R, MODE, FORM, REV, COOP>(a, a.order ? a.order[tix] : tix, s_lut, csp, wave);
    if (!queued) return;
  }
}

__global__ void k_area_keys(const InterTask *tasks, int64_t ntasks, int32_t R, uint64_t *keys,
                            int64_t *vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const InterTask tk = tasks[t];
  // a banded (reversed) task's strips sweep windows of R + band_q + band columns
  uint64_t w = (uint32_t)tk.rp;
  if (tk.band >= 0) {
    const uint64_t win = (uint64_t)R + (uint32_t)tk.band_q + (uint32_t)tk.band + 4;
    w = win < w ? win : w;
  }
  // in units of 256 cells, clamped to 24 bits (tasks above 2^32 cells share
  // the top key: only the order of their launch depends on it)
  const uint64_t k = ((uint64_t)(uint32_t)tk.qp * w) >> 8;
  keys[t] = k < 0xFFFFFFull ? k : 0xFFFFFFull;
  vals[t] = t;
}

__global__ void k_zero_queue(unsigned long long *q) {
  if (threadIdx.x == 0) *q = 0ull;
}

// ---- packed reference symbols: per task, column group, lane -------------
// One block per task.  The reference bytes of a chunk of 256 columns are read
// pair by pair (consecutive threads read consecutive bytes of one sequence,
// so the reads coalesce) into an LDS tile [slot][column], then written out
// transposed as the [group][lane] words the fill reads.  The tile row stride
// of 260 bytes keeps the transposed dword reads free of bank conflicts.
constexpr int kRsymChunk = 256;
constexpr int kRsymStride = kRsymChunk + 4;

__global__ __launch_bounds__(256) void k_inter_rsym(PackArgs a) {
  __shared__ uint8_t tile[kSlots16 * kRsymStride];
  __shared__ const int8_t *s_base[kSlots16];
  __shared__ int64_t s_len[kSlots16], s_pad[kSlots16];
  const int64_t t = blockIdx.x;
  if (t >= a.ntasks) return;
  const InterTask tk = a.tasks[t];
  const int nslots = a.halves * 64;
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    const int64_t p = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
    if (p >= 0) {
      const int64_t lr = a.view.rlen[p];
      s_base[s] = a.view.rcat + a.view.rstart[p];
      s_len[s] = lr;
      s_pad[s] = a.rev ? 0 : tk.rp - lr;
    } else {
      s_base[s] = nullptr;
      s_len[s] = 0;
      s_pad[s] = 0;
    }
  }
  __syncthreads();
  const bool reversed = a.view.reversed != 0;
  const uint8_t pad_sym = (uint8_t)a.n;
  uint2 *dst = a.rsym + rsym_offset(tk.bnd_off);
  for (int64_t c0 = 0; c0 < tk.rp; c0 += kRsymChunk) {
    const int64_t c = c0 + threadIdx.x;
    // slots in groups of 64: the group's loads are all in flight before the
    // first byte is written to the tile (one memory wait per 64 slots)
    for (int s0 = 0; s0 < nslots; s0 += 64) {
      int8_t raw[64];
#pragma unroll
      for (int u = 0; u < 64; ++u) {
        const int s = s0 + u;
        const int64_t j = c - s_pad[s];
        const int64_t len = s_len[s];
        const bool in = j >= 0 && j < len;
        raw[u] = in ? s_base[s][reversed ? len - 1 - j : j] : (int8_t)-1;
      }
#pragma unroll
      for (int u = 0; u < 64; ++u) {
        const int8_t x = raw[u];
        tile[(s0 + u) * kRsymStride + threadIdx.x] =
            (x >= 0 && x < a.n) ? (uint8_t)x : pad_sym;   // a bad code never indexes a table
      }
    }
    __syncthreads();
    int64_t ng = (tk.rp - c0) / 4;
    if (ng > kRsymChunk / 4) ng = kRsymChunk / 4;
    for (int u = threadIdx.x; u < ng * 64; u += blockDim.x) {
      const int g = u >> 6, lane = u & 63;
      const uint32_t x = *reinterpret_cast<const uint32_t *>(&tile[lane * kRsymStride + 4 * g]);
      const uint32_t y = (a.halves == 2)
          ? *reinterpret_cast<const uint32_t *>(&tile[(lane + 64) * kRsymStride + 4 * g])
          : (uint32_t)pad_sym * 0x01010101u;
      dst[(c0 / 4 + g) * 64 + lane] = make_uint2(x, y);
    }
    __syncthreads();
  }
}

// ---- QGEN profile: per task, strip, symbol, half, lane: R biased bytes ----
__global__ __launch_bounds__(256) void k_inter_prof(PackArgs a) {
  const int64_t t = blockIdx.x;
  if (t >= a.ntasks) return;
  const InterTask tk = a.tasks[t];
  const int R = a.strip_rows;
  const int np1 = a.n + 1;
  const int64_t nstrips = tk.qp / R;
  const int64_t units = nstrips * np1 * a.halves * 64;
  for (int64_t u = threadIdx.x; u < units; u += blockDim.x) {
    const int lane = (int)(u & 63);
    int64_t rest = u >> 6;
    const int h = (int)(rest % a.halves); rest /= a.halves;
    const int sy = (int)(rest % np1);
    const int64_t strip = rest / np1;
    const int s = lane + 64 * h;
    const int64_t p = (s < tk.nslots) ? a.slot_pair[tk.slot_base + s] : -1;
    uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // up to R = 32 bytes
    if (p >= 0 && sy < a.n) {
      const int32_t lq = a.view.qlen[p];
      const SeqRef q = make_seq(a.view.qcat + a.view.qstart[p], lq, a.rev ? 0 : tk.qp - lq,
                                a.view.reversed != 0, a.matrix);
      for (int r = 0; r < R; ++r) {
        const int32_t qv = seq_at(q, strip * R + r);
        const uint32_t b = (qv < 0 || qv >= a.n) ? 0u : (uint32_t)(uint8_t)(a.matrix[qv * a.n + sy] + a.bias);
        w[r >> 2] |= b << (8 * (r & 3));
      }
    }
    uint4 *dst = (uint4 *)(a.prof + tk.qdata_off + u * R);
    for (int k = 0; k < R / 16; ++k)
      dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
  }
}

// ---- host-side launchers ------------------------------------------------
template <class V, int R, uint32_t MODE, int FORM>
static void launch_form(const InterArgs &a, dim3 g, dim3 b, hipStream_t st) {
  const bool coop = a.coop > 1;
  if (a.rev) {
    if (coop) hipLaunchKernelGGL((k_inter_fill<V, R, MODE, FORM, true, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_inter_fill<V, R, MODE, FORM, true, false>), g, b, 0, st, a);
  } else {
    if (coop) hipLaunchKernelGGL((k_inter_fill<V, R, MODE, FORM, false, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_inter_fill<V, R, MODE, FORM, false, false>), g, b, 0, st, a);
  }
}

template <class V, int R, uint32_t MODE>
static hipError_t launch_fill(const InterArgs &a, hipStream_t st) {
  // forward passes: one wave per workgroup, so that each wave slot takes the
  // next task as soon as its own task ends (with four, a workgroup's slots
  // wait for its longest task: measured 11.35 -> 10.95 ms on the benchmark
  // workload); reversed passes (short tasks, early exits) measured faster in
  // workgroups of four
  const int waves_per_block = (a.coop > 1 || a.rev) ? 4 : 1;
  if (a.coop != 1 && a.coop != kCoopWaves) return hipErrorInvalidValue;
  int64_t blocks = a.coop > 1 ? a.ntasks : (a.ntasks + waves_per_block - 1) / waves_per_block;
  if (blocks == 0) return hipSuccess;
  if (a.sched == 2) {
    if (!a.queue || a.cus < 1) return hipErrorInvalidValue;
    // resident blocks: waves per SIMD x 4 SIMDs per CU / waves per block
    const int64_t resident = (int64_t)a.cus * fill_waves<R>() * (4 / waves_per_block);
    if (blocks > resident) blocks = resident;
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, a.queue);
  }
  const dim3 g((unsigned)blocks), b(64 * waves_per_block);
  // 32-bit lanes: one form (their values hold any score beside the code);
  // 16-bit strips other than 32 rows (tuning choices): no pairs, no merged H - o
  if constexpr (VT<V>::kHalves == 1) {
    launch_form<V, R, MODE, kColPlain>(a, g, b, st);
  } else if constexpr (R != 32) {
    if (a.clamp) launch_form<V, R, MODE, kColClamp>(a, g, b, st);
    else launch_form<V, R, MODE, kColPlain>(a, g, b, st);
  } else {
    const int col = a.clamp ? kColClamp : (a.pair3 ? kColPair : kColPlain);
    switch (col | (a.bias == a.o ? kFormHo : 0)) {
      case kColPlain: launch_form<V, R, MODE, kColPlain>(a, g, b, st); break;
      case kColClamp: launch_form<V, R, MODE, kColClamp>(a, g, b, st); break;
      case kColPair: launch_form<V, R, MODE, kColPair>(a, g, b, st); break;
      case kColPlain | kFormHo: launch_form<V, R, MODE, kColPlain | kFormHo>(a, g, b, st); break;
      case kColClamp | kFormHo: launch_form<V, R, MODE, kColClamp | kFormHo>(a, g, b, st); break;
      default: launch_form<V, R, MODE, kColPair | kFormHo>(a, g, b, st); break;
    }
  }
  return hipGetLastError();
}

hipError_t inter_fill(const InterArgs &a, int lane_bits, int R, hipStream_t st) {
  const bool qsel = (a.prof == nullptr && a.qprof == nullptr);
  if (lane_bits == 16) {
    if (R == 32) return qsel ? launch_fill<u16x2, 32, kQSel>(a, st) : launch_fill<u16x2, 32, kQGen>(a, st);
    if (R == 24 && qsel) return launch_fill<u16x2, 24, kQSel>(a, st);
    if (R == 16) return qsel ? launch_fill<u16x2, 16, kQSel>(a, st) : launch_fill<u16x2, 16, kQGen>(a, st);
  } else {
    if (R == 32) return qsel ? launch_fill<uint32_t, 32, kQSel>(a, st) : launch_fill<uint32_t, 32, kQGen>(a, st);
    if (R == 24 && qsel) return launch_fill<uint32_t, 24, kQSel>(a, st);
    if (R == 16) return qsel ? launch_fill<uint32_t, 16, kQSel>(a, st) : launch_fill<uint32_t, 16, kQGen>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t inter_area_keys(const InterTask *tasks, int64_t ntasks, int32_t R, uint64_t *keys,
                           int64_t *vals, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_area_keys, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0, st, tasks,
                     ntasks, R, keys, vals);
  return hipGetLastError();
}

hipError_t inter_pack_ref(const PackArgs &a, hipStream_t st) {
  if (a.ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inter_rsym, dim3((unsigned)a.ntasks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t inter_pack(const PackArgs &a, hipStream_t st) {
  if (a.ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inter_prof, dim3((unsigned)a.ntasks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace swx
