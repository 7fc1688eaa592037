// fill_intra.hip -- intra-sequence Smith-Waterman-Gotoh fill for long pairs.
//
// Same recurrences as the inter-sequence fill (paper, Introduction and method
// section "Algorithm and implementation"), but one pair is spread over the
// 64 lanes of a wave: lane k owns RL consecutive query rows of a strip of
// 64*RL rows and computes column c - k at step c.  Per step a lane receives
// from the lane above, through a one-lane DPP shift, the H leaving that lane's
// last row, the F entering its own first row, the running column max and the
// reference symbol; lane 0 receives them from the previous strip's hand-over
// row (or zeros) and from a 64-column buffer refilled every 64 steps.  The
// column max leaves lane 63 and is collected, 64 columns at a time, into a
// register for one coalesced store.
//
// Forward pass: the max array of the method section, as one word per column,
// value << kbits | (2^kbits - 1 - padded row), so that the max over rows and
// strips also names the first row reaching the value.  The end (rule T1)
// comes from a reduction over the max array (k_intra_end).
// Reversed pass: stops at the first reversed column whose max reaches the
// target score and reports the smallest row there (the begin, rule T2).
//
// All lanes are 32-bit, biased like the inter-sequence kernel: scores arrive
// as S + bias >= 0, E and F are kept biased and floored at 0, and one
// saturating subtraction of the bias yields H with its zero floor (and, when
// the bias is the gap open penalty, also the H - o that opens a gap).
#include <hip/hip_runtime.h>

#include "lanes.h"
#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

typedef u16x2 V16;

constexpr int kDppWaveShr1 = 0x138;   // DPP control: lane k reads lane k - 1

// value of src from the lane above; lane 0 takes `top`
__device__ __forceinline__ uint32_t from_above(uint32_t src, uint32_t top) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)top, (int)src, kDppWaveShr1, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t lane_value(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// vec with lane `at` of the wave replaced by the (uniform) v
__device__ __forceinline__ uint32_t set_lane(uint32_t vec, int at, uint32_t v) {
  return ((int)(threadIdx.x & 63) == at) ? v : vec;
}

constexpr int kDppWaveShl1 = 0x130;   // DPP control: lane k reads lane k + 1

// vec moved one lane down (lane k takes lane k + 1) with lane 63 taking its
// own v: a queue of lane 63's values, the newest at lane 63
__device__ __forceinline__ uint32_t shift_in(uint32_t vec, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)vec, kDppWaveShl1, 0xF, 0xF, false);
}

// RL bytes (RL a multiple of 4) of the LDS profile as RL/4 words
template <int RL>
__device__ __forceinline__ void lds_load_words(const uint8_t *src, uint32_t (&w)[RL / 4]) {
  if constexpr (RL % 16 == 0) {
#pragma unroll
    for (int k = 0; k < RL / 16; ++k) {
      const uint4 v = reinterpret_cast<const uint4 *>(src)[k];
      w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
    }
  } else if constexpr (RL == 8) {
    const uint2 v = *reinterpret_cast<const uint2 *>(src);
    w[0] = v.x; w[1] = v.y;
  } else {
    w[0] = *reinterpret_cast<const uint32_t *>(src);
  }
}

template <int RL>
__device__ __forceinline__ void lds_store_words(uint8_t *dst, const uint32_t (&w)[RL / 4]) {
  if constexpr (RL % 16 == 0) {
#pragma unroll
    for (int k = 0; k < RL / 16; ++k)
      reinterpret_cast<uint4 *>(dst)[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
  } else if constexpr (RL == 8) {
    *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
  } else {
    *reinterpret_cast<uint32_t *>(dst) = w[0];
  }
}

// Strips of one job run on the waves of one workgroup: wave w takes strips
// w, w + NW, w + 2*NW, ...  Strip s reads the hand-over row of strip s - 1
// (global memory, one row per boundary) only after strip s - 1 has published,
// through a progress counter in LDS, that those columns are written.  Every
// strip depends only on the one above, the waves of a workgroup are resident
// together, and no strip ever waits on a later one, so the waits always end;
// a spin limit still bounds them (exceeding it flags the pair as failed).
//
// Spread jobs (SPREAD): the strips of one job run on the waves of `segs`
// workgroups (global wave g = segment * NW + wave takes strips g, g + segs*NW,
// ...), with the progress counters, the reversed pass's hits and a completion
// count in global memory (IntraSync, agent-scope release and acquire).  The
// host launches a spread grid only when every workgroup of it fits on the
// device at once (at most one per compute unit), so a strip's producer is
// always running; the same spin limit bounds the waits.
constexpr int kMaxStrips = kIntraMaxStrips;
constexpr int kMaxWaves = 8;
constexpr int64_t kSpinLimit = int64_t(1) << 26;

__device__ __forceinline__ void lds_wave_sync() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

template <int RL, bool REV, bool SPREAD, bool HO>
__global__ __launch_bounds__(64 * kMaxWaves) void k_intra_fill(IntraArgs a) {
  extern __shared__ uint4 s_dyn[];            // per wave: [(n + 1) symbols][64 lanes][RL bytes]
  __shared__ int8_t s_mat[32 * 32];
  __shared__ int32_t l_prog[SPREAD ? 1 : kMaxStrips];      // columns published by strip s (from its window start)
  __shared__ int32_t l_done[SPREAD ? 1 : kMaxStrips];      // strip s finished (its progress is final)
  __shared__ int64_t l_rcol[SPREAD ? 1 : kMaxStrips];      // reversed pass: first column of strip s reaching the target
  __shared__ int32_t l_rrow[SPREAD ? 1 : kMaxStrips];
  __shared__ unsigned long long l_best;       // reversed pass: smallest such column so far (~0: none)
  constexpr int SH = 64 * RL;
  constexpr int SCOPE = SPREAD ? __HIP_MEMORY_SCOPE_AGENT : __HIP_MEMORY_SCOPE_WORKGROUP;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  // spread grids: workgroups go to the 8 XCDs round robin by block id, so
  // block 8 * slot + x (slot = (j / 8) * G + segment) puts every segment of
  // job j on XCD j % 8, where the hand-over rows stay in one L2; the grid is
  // 8 * G * ceil(njobs / 8) blocks and those past the last job leave at once
  const int G = SPREAD ? a.segs : 1;
  int64_t jix = blockIdx.x, seg = 0;
  if constexpr (SPREAD) {
    const int64_t slot = blockIdx.x / 8;
    jix = (slot / G) * 8 + blockIdx.x % 8;
    seg = slot % G;
    if (jix >= a.njobs) return;
  }
  IntraSync *gs = SPREAD ? a.sync + jix : nullptr;
  int32_t *s_prog = SPREAD ? gs->prog : l_prog;
  int32_t *s_done = SPREAD ? gs->done : l_done;
  int64_t *s_rcol = SPREAD ? gs->rcol : l_rcol;
  int32_t *s_rrow = SPREAD ? gs->rrow : l_rrow;
  unsigned long long *s_best = SPREAD ? &gs->best : &l_best;
  const IntraJob jb = a.jobs[jix];
  if (!REV && jb.c1 <= jb.cw) return;   // an empty column chunk
  const int64_t p = jb.pair;
  const int32_t Lq = a.view.qlen[p];
  const int64_t Lr = a.view.rlen[p];
  const int8_t *qs = a.view.qcat + a.view.qstart[p];
  const int8_t *rs = a.view.rcat + a.view.rstart[p];
  const bool rv = a.view.reversed != 0;
  const int n = a.n;
  const int64_t qp = ((int64_t)Lq + SH - 1) / SH * SH;
  const int nstrips = (int)(qp / SH);
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) s_mat[i] = a.matrix[i];
  if constexpr (!SPREAD) {   // spread jobs: set by intra_sync_init before the launch
    for (int i = threadIdx.x; i < nstrips && i < kMaxStrips; i += blockDim.x) {
      s_prog[i] = 0;
      s_done[i] = 0;
      s_rcol[i] = -1;
      s_rrow[i] = -1;
    }
    if (threadIdx.x == 0) *s_best = ~0ull;
  }
  __syncthreads();

  const int64_t qpad = REV ? 0 : qp - Lq;   // forward: padding rows on top
  const int kb = jb.kbits;
  const uint32_t M = (1u << kb) - 1u;
  const int32_t tgt = REV ? a.target[p] : 0;
  const int64_t width = jb.c1 - jb.cw;
  uint32_t *mc = a.maxcol + jb.mc_off;
  const uint32_t vbias = (uint32_t)a.bias, vo = (uint32_t)a.o, ve = (uint32_t)a.e;
  uint8_t *s_prof = reinterpret_cast<uint8_t *>(s_dyn) + (size_t)wave * (n + 1) * 64 * RL;
  using T = VT<uint32_t>;

  // column window of strip s (the reversed pass bands it)
  auto window = [&](int s, int64_t &clo, int64_t &chi) {
    clo = jb.cw;
    chi = jb.c1;
    if (REV && jb.band >= 0) {
      const int64_t l = (int64_t)s * SH - jb.band;
      if (l > clo) clo = l;
      const int64_t h = (int64_t)s * SH + SH + jb.band;
      if (h < chi) chi = h;
    }
    if (chi < clo) chi = clo;
  };

  auto fence_rel = [] {
    if constexpr (SPREAD) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  };
  auto fence_acq = [] {
    if constexpr (SPREAD) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };

  for (int s = (int)seg * NW + wave; s < nstrips; s += G * NW) {
    int64_t clo, chi, plo = 0, phi = 0;
    window(s, clo, chi);
    if (s > 0) window(s - 1, plo, phi);
    uint32_t *bndH = a.bnd + jb.bnd_off + 2 * width * (int64_t)s;   // this strip's hand-over row
    uint32_t *bndF = bndH + width;
    uint32_t *inH = bndH - 2 * width;                              // the row of strip s - 1
    uint32_t *inF = inH + width;
    const bool hand_over = (s + 1 < nstrips);
    int32_t published = 0;
    auto publish = [&](int32_t ncols, bool fin) {
      fence_rel();
      if (lane == 0) {
        __hip_atomic_store(&s_prog[s], ncols, __ATOMIC_RELAXED, SCOPE);
        if (fin) __hip_atomic_store(&s_done[s], 1, __ATOMIC_RELAXED, SCOPE);
      }
    };
    // the reversed pass skips a strip that cannot hold an earlier column
    if (REV && __hip_atomic_load(s_best, __ATOMIC_RELAXED, SCOPE) <= (unsigned long long)clo) {
      publish(0, true);
      continue;
    }

    // strip profile: biased scores of this lane's RL rows against every symbol
    {
      int32_t qv[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int64_t i = (int64_t)s * SH + lane * RL + r - qpad;
        qv[r] = (i >= 0 && i < Lq) ? (int32_t)qs[rv ? Lq - 1 - i : i] : -1;
      }
      for (int sy = 0; sy <= n; ++sy) {
        uint32_t w[RL / 4];
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) w[k] = 0u;
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const uint32_t b = (qv[r] >= 0 && sy < n) ? (uint32_t)(uint8_t)(s_mat[qv[r] * n + sy] + a.bias) : 0u;
          w[r >> 2] |= b << (8 * (r & 3));
        }
        lds_store_words<RL>(s_prof + ((int64_t)sy * 64 + lane) * RL, w);
      }
    }
    lds_wave_sync();

    // code offset of this lane's rows: code = M - padded row
    const uint32_t DL = M - (uint32_t)((int64_t)s * SH + lane * RL + RL - 1);
    // wait until strip s - 1 has published `need` columns (or finished);
    // returns the columns available
    int32_t avail = 0;
    bool spin_fail = false;
    auto wait_for = [&](int32_t need) {
      if (s == 0) return;
      int64_t spins = 0;
      for (;;) {
        const int32_t done = __hip_atomic_load(&s_done[s - 1], __ATOMIC_RELAXED, SCOPE);
        avail = __hip_atomic_load(&s_prog[s - 1], __ATOMIC_RELAXED, SCOPE);
        if (done || avail >= need) break;
        if (++spins > kSpinLimit) { spin_fail = true; break; }
        __builtin_amdgcn_s_sleep(2);
      }
      fence_acq();
    };

    uint32_t H[RL], E[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) { H[r] = 0u; E[r] = 0u; }
    uint32_t hup_prev = 0u;
    if (s > 0 && clo >= 1 && clo - 1 >= plo && clo - 1 < phi) {
      wait_for((int32_t)(clo - plo));
      if (lane == 0 && clo - 1 < plo + avail)
        hup_prev = __hip_atomic_load(&inH[clo - 1 - jb.cw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t hout = 0u, fout = 0u, cmout = 0u;
    uint32_t hbuf = 0u, fbuf = 0u;
    uint32_t obH = 0u, obF = 0u, obC = 0u;
    const int64_t nsteps = (chi - clo) + 63;
    int64_t cdone = chi;
    // reference symbols of columns [c0, c0 + 64) at lane c - c0 (n past the window)
    auto symbols = [&](int64_t c0) -> uint32_t {
      const int64_t c = c0 + lane;
      return c < chi ? (uint32_t)(uint8_t)rs[rv ? Lr - 1 - c : c] : (uint32_t)n;
    };
    // the symbols of this 64-step chunk and of the next one; the profile row
    // of a step is read one step ahead (its symbol is the one the lane above
    // holds now), so the LDS latency hides behind a step's arithmetic
    uint32_t symbuf = symbols(clo), symnext = symbols(clo + 64);
    uint32_t sym = from_above((uint32_t)n, lane_value(symbuf, 0));
    uint32_t X[RL / 4];
    lds_load_words<RL>(s_prof + ((int64_t)sym * 64 + lane) * RL, X);

    // store the outputs of columns [col - j, col], held by lanes 63 - j .. 63
    auto flush = [&](int64_t col, int j) {
      if (lane >= 63 - j) {
        const int64_t c = col - 63 + lane;
        if (hand_over) {
          bndH[c - jb.cw] = obH;
          bndF[c - jb.cw] = obF;
        }
        if (!REV && c >= jb.c0 && c < jb.c1) atomicMax(&mc[c], obC);
      }
      if (hand_over) publish((int32_t)(col + 1 - clo), false);
    };

    // Steps go in blocks of 64: the block's start reads the symbols and the
    // row above for its 64 columns, its step 62 completes the output queues
    // of 64 columns (flushed there from the second block on), and step 63
    // takes its next symbol from the next block's lanes; so the steps in
    // between carry no per-step tests beyond the reversed pass's target.
    bool stop = false;
#pragma unroll 1
    for (int64_t t0 = 0; t0 < nsteps; t0 += 64) {
      if (REV && t0 >= 63 &&
          (unsigned long long)(clo + t0 - 63) >= __hip_atomic_load(s_best, __ATOMIC_RELAXED, SCOPE)) {
        cdone = clo + t0 - 63;   // an earlier strip already reached the target at or before here
        break;
      }
      if (t0 > 0) {
        symbuf = symnext;
        symnext = symbols(clo + t0 + 64);
      }
      {   // inputs of lane 0 for the next 64 steps
        const int64_t cend = (clo + t0 + 64 < phi) ? clo + t0 + 64 : phi;
        if (s > 0 && cend > plo) wait_for((int32_t)(cend - plo));
        const int64_t c = clo + t0 + lane;
        const bool prev = c < chi && s > 0 && c >= plo && c < plo + avail && c < phi;
        // read past the CU's L1 (another wave wrote them)
        hbuf = prev ? __hip_atomic_load(&inH[c - jb.cw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        fbuf = prev ? __hip_atomic_load(&inF[c - jb.cw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      }
      // step t0 + tm; the next step's symbol is lane `nl` of `nsym`.  Returns
      // true when the reversed pass has reached its target (outputs flushed).
      auto step = [&](int tm, uint32_t nsym, int nl) -> bool {
        const uint32_t hup = from_above(hout, lane_value(hbuf, tm));
        uint32_t F = from_above(fout, lane_value(fbuf, tm));
        const uint32_t cmin = from_above(cmout, 0u);
        // next step's symbol and profile row
        const uint32_t symn = from_above(sym, lane_value(nsym, nl));
        uint32_t Xn[RL / 4];
        lds_load_words<RL>(s_prof + ((int64_t)symn * 64 + lane) * RL, Xn);

        uint32_t cm = 0u;
        uint32_t u_next = T::max(hup_prev + __builtin_amdgcn_ubfe(X[0], 0, 8), E[0]);
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const uint32_t u = u_next;
          if (r + 1 < RL)
            u_next = T::max(H[r] + __builtin_amdgcn_ubfe(X[(r + 1) >> 2], 8 * ((r + 1) & 3), 8), E[r + 1]);
          const uint32_t hb = T::max(u, F);
          const uint32_t hn = T::subs(hb, vbias);
          H[r] = hn;
          const uint32_t enc = (hn << kb) + (uint32_t)(RL - 1 - r);
          cm = cm > enc ? cm : enc;
          const uint32_t ho = HO ? hn : T::subs(hb, vo);   // HO: bias == o
          E[r] = T::max(T::subs(E[r], ve), ho);
          F = T::max(T::subs(F, ve), ho);
        }
        hup_prev = hup;
        hout = H[RL - 1];
        fout = F;
        const uint32_t cml = cm + DL;
        cmout = cmin > cml ? cmin : cml;
        sym = symn;
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) X[k] = Xn[k];

        // lane 63's outputs enter at lane 63 while the collected ones move one
        // lane down: after 64 steps lane k holds the k-th column of the chunk
        obH = shift_in(obH, hout);
        obF = shift_in(obF, fout);
        obC = shift_in(obC, cmout);
        if constexpr (REV) {
          const int64_t t = t0 + tm;
          if (t >= 63) {
            const uint32_t oc = lane_value(cmout, 63);
            if (tgt > 0 && (int32_t)(oc >> kb) >= tgt) {
              const int64_t col = clo + t - 63;
              flush(col, (int)((t - 63) & 63));
              cdone = col + 1;
              if (lane == 0) {
                s_rcol[s] = col;
                s_rrow[s] = (int32_t)(M - (oc & M));
                atomicMin(s_best, (unsigned long long)col);
              }
              return true;
            }
          }
        }
        return false;
      };
      const int tn = (int)(nsteps - t0 < 64 ? nsteps - t0 : 64);
      const int ta = tn < 62 ? tn : 62;
#pragma unroll 1
      for (int tm = 0; tm < ta; ++tm)
        if (step(tm, symbuf, tm + 1)) { stop = true; break; }
      if (stop) break;
      if (tn > 62) {
        if (step(62, symbuf, 63)) break;
        if (t0 >= 64) flush(clo + t0 - 1, 63);   // step t0 + 62 ends columns ..t0 - 1 + clo
      }
      if (tn > 63 && step(63, symnext, 0)) break;
      if (t0 + tn == nsteps) {   // the strip's last step: the rest of its outputs
        const int64_t t = nsteps - 1;
        const int j = (int)((t - 63) & 63);
        if (t >= 63 && j != 63) flush(clo + t - 63, j);
      }
    }
    publish((int32_t)(cdone - clo), true);
    if (spin_fail && lane == 0) a.err[p] = 1;   // reported as an internal failure
  }
  if constexpr (SPREAD) {
    if constexpr (!REV) return;
    // the last segment of the job to finish reduces the strips' hits
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __shared__ int32_t s_last;
    if (threadIdx.x == 0) s_last = atomicAdd(&gs->fin, 1) == G - 1;
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  } else {
    __syncthreads();
  }

  if (REV && threadIdx.x == 0) {
    // first column reaching the target; on a tie the earlier strip (smaller row)
    int64_t bc = -1;
    int32_t br = -1;
    for (int s = 0; s < nstrips && s < kMaxStrips; ++s) {
      if (s_rcol[s] >= 0 && (bc < 0 || s_rcol[s] < bc)) { bc = s_rcol[s]; br = s_rrow[s]; }
    }
    const bool hit = bc >= 0;
    a.out.score[p] = hit ? tgt : 0;
    a.out.qend[p] = hit ? br : -1;
    a.out.rend[p] = hit ? bc : -1;
    a.out.overflow[p] = 0;
  }
}

// ---- packed 16-bit lanes: two column streams per wave ---------------------
// The forward pass on 2 x 16-bit lanes.  Two jobs with the same strip layout
// (jobs[2b] in the low halves, jobs[2b + 1] in the high halves) share a wave:
// lane k holds rows [k*RL, (k+1)*RL) of both, so one packed instruction
// updates a cell of each.  Both jobs' scores must stay below 2^15 (checked
// before launch: a score can reach smax * min(qlen, rlen)).  The column max
// leaves a lane per job as one 32-bit word value << 16 | (65535 - padded
// row), built from the packed H with v_perm, so the max array has the same
// layout as the 32-bit pass with kbits = 16.  Hand-over rows hold the 16-bit
// values in 32-bit words, one row per job as in the 32-bit pass.
// M3: every lane value of the launch stays below 0x7C00 (score bound plus
// bias), so H is taken with one packed three-way maximum.
template <int RL, bool M3, bool HO>
__global__ __launch_bounds__(64 * kMaxWaves) void k_intra_fill16(IntraArgs a) {
  extern __shared__ uint4 s_dyn[];            // per wave and job: [(n + 1) symbols][64 lanes][RL bytes]
  __shared__ int8_t s_mat[32 * 32];
  __shared__ int32_t s_prog[kMaxStrips];
  __shared__ int32_t s_done[kMaxStrips];
  constexpr int SH = 64 * RL;
  using T = VT<u16x2>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int n = a.n;
  const IntraJob jA = a.jobs[2 * (int64_t)blockIdx.x];
  const IntraJob jB = a.jobs[2 * (int64_t)blockIdx.x + 1];
  const bool hasB = jB.pair >= 0;
  const int64_t pA = jA.pair, pB = hasB ? jB.pair : jA.pair;
  const int32_t LqA = a.view.qlen[pA], LqB = a.view.qlen[pB];
  const int64_t LrA = a.view.rlen[pA], LrB = a.view.rlen[pB];
  const int8_t *qsA = a.view.qcat + a.view.qstart[pA], *qsB = a.view.qcat + a.view.qstart[pB];
  const int8_t *rsA = a.view.rcat + a.view.rstart[pA], *rsB = a.view.rcat + a.view.rstart[pB];
  // both jobs have the same padded height (the host pairs them so)
  const int64_t qp = ((int64_t)LqA + SH - 1) / SH * SH;
  const int nstrips = (int)(qp / SH);
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) s_mat[i] = a.matrix[i];
  for (int i = threadIdx.x; i < nstrips && i < kMaxStrips; i += blockDim.x) {
    s_prog[i] = 0;
    s_done[i] = 0;
  }
  __syncthreads();
  const int64_t qpadA = qp - LqA, qpadB = qp - LqB;
  const int64_t widthA = jA.c1 - jA.cw, widthB = hasB ? jB.c1 - jB.cw : 0;
  const int64_t width = widthA > widthB ? widthA : widthB;   // steps of the wave, both jobs
  uint32_t *mcA = a.maxcol + jA.mc_off, *mcB = a.maxcol + (hasB ? jB.mc_off : jA.mc_off);
  const V16 vbias = T::splat((uint32_t)a.bias), vo = T::splat((uint32_t)a.o), ve = T::splat((uint32_t)a.e);
  const size_t tbl = (size_t)(n + 1) * 64 * RL;
  uint8_t *s_profA = reinterpret_cast<uint8_t *>(s_dyn) + (size_t)wave * 2 * tbl;
  uint8_t *s_profB = s_profA + tbl;
  // v_perm selectors: the low (A) or high (B) 16-bit half of H above a 16-bit code
  const uint32_t selA = 0x05040100u, selB = 0x07060100u;

  for (int s = wave; s < nstrips; s += NW) {
    uint32_t *bHA = a.bnd + jA.bnd_off + 2 * widthA * (int64_t)s;
    uint32_t *bFA = bHA + widthA;
    uint32_t *bHB = a.bnd + (hasB ? jB.bnd_off : jA.bnd_off) + 2 * widthB * (int64_t)s;
    uint32_t *bFB = bHB + widthB;
    uint32_t *iHA = bHA - 2 * widthA, *iFA = iHA + widthA;   // rows of strip s - 1
    uint32_t *iHB = bHB - 2 * widthB, *iFB = iHB + widthB;
    const bool hand_over = (s + 1 < nstrips);
    auto publish = [&](int32_t ncols, bool fin) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) {
        __hip_atomic_store(&s_prog[s], ncols, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (fin) __hip_atomic_store(&s_done[s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    };
    // strip profiles of both jobs
    {
      int32_t qa[RL], qb[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int64_t row = (int64_t)s * SH + lane * RL + r;
        const int64_t ia = row - qpadA, ib = row - qpadB;
        qa[r] = (ia >= 0 && ia < LqA) ? (int32_t)qsA[ia] : -1;
        qb[r] = (hasB && ib >= 0 && ib < LqB) ? (int32_t)qsB[ib] : -1;
      }
      for (int sy = 0; sy <= n; ++sy) {
        uint32_t wa[RL / 4], wb[RL / 4];
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) { wa[k] = 0u; wb[k] = 0u; }
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const uint32_t ba = (qa[r] >= 0 && sy < n) ? (uint32_t)(uint8_t)(s_mat[qa[r] * n + sy] + a.bias) : 0u;
          const uint32_t bb = (qb[r] >= 0 && sy < n) ? (uint32_t)(uint8_t)(s_mat[qb[r] * n + sy] + a.bias) : 0u;
          wa[r >> 2] |= ba << (8 * (r & 3));
          wb[r >> 2] |= bb << (8 * (r & 3));
        }
        lds_store_words<RL>(s_profA + ((int64_t)sy * 64 + lane) * RL, wa);
        lds_store_words<RL>(s_profB + ((int64_t)sy * 64 + lane) * RL, wb);
      }
    }
    lds_wave_sync();

    // code offset of this lane's rows: 65535 - padded row of row r is
    // (RL - 1 - r) + DL
    const uint32_t DL = 65535u - (uint32_t)((int64_t)s * SH + lane * RL + RL - 1);
    int32_t avail = 0;
    bool spin_fail = false;
    auto wait_for = [&](int32_t need) {
      if (s == 0) return;
      int64_t spins = 0;
      for (;;) {
        const int32_t done = __hip_atomic_load(&s_done[s - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        avail = __hip_atomic_load(&s_prog[s - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (done || avail >= need) break;
        if (++spins > kSpinLimit) { spin_fail = true; break; }
        __builtin_amdgcn_s_sleep(2);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };

    V16 H[RL], E[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) { H[r] = T::zero(); E[r] = T::zero(); }
    V16 hup_prev = T::zero();
    V16 hout = T::zero(), fout = T::zero();
    uint32_t cmoutA = 0u, cmoutB = 0u;
    uint32_t hbuf = 0u, fbuf = 0u;
    uint32_t obH = 0u, obF = 0u, obCA = 0u, obCB = 0u;
    const int64_t nsteps = width + 63;
    // both jobs' reference symbols of step offsets [o0, o0 + 64), A in the
    // low byte, B in the next; the profile rows of a step are read one step
    // ahead, as in the 32-bit pass
    auto symbols = [&](int64_t o0) -> uint32_t {
      const int64_t off = o0 + lane;
      const uint32_t sa = off < widthA ? (uint32_t)(uint8_t)rsA[jA.cw + off] : (uint32_t)n;
      const uint32_t sb = (hasB && off < widthB) ? (uint32_t)(uint8_t)rsB[jB.cw + off] : (uint32_t)n;
      return sa | (sb << 8);
    };
    uint32_t symbuf = symbols(0), symnext = symbols(64);
    uint32_t sym = from_above((uint32_t)n * 0x101u, lane_value(symbuf, 0));
    uint32_t XA[RL / 4], XB[RL / 4];
    lds_load_words<RL>(s_profA + ((int64_t)(sym & 0xFFu) * 64 + lane) * RL, XA);
    lds_load_words<RL>(s_profB + ((int64_t)((sym >> 8) & 0xFFu) * 64 + lane) * RL, XB);

    // store the outputs of step offsets [o - j, o], held by lanes 63 - j .. 63
    // (packed H and F: A in the low half, B in the high half)
    auto flush = [&](int64_t o, int j) {
      if (lane >= 63 - j) {
        const int64_t off = o - 63 + lane;
        if (off < widthA) {
          if (hand_over) { bHA[off] = obH & 0xFFFFu; bFA[off] = obF & 0xFFFFu; }
          const int64_t col = jA.cw + off;
          if (col >= jA.c0 && col < jA.c1) atomicMax(&mcA[col], obCA);
        }
        if (hasB && off < widthB) {
          if (hand_over) { bHB[off] = obH >> 16; bFB[off] = obF >> 16; }
          const int64_t col = jB.cw + off;
          if (col >= jB.c0 && col < jB.c1) atomicMax(&mcB[col], obCB);
        }
      }
      if (hand_over) publish((int32_t)(o + 1), false);
    };

    // steps in blocks of 64, as in the 32-bit pass
#pragma unroll 1
    for (int64_t t0 = 0; t0 < nsteps; t0 += 64) {
      if (t0 > 0) {
        symbuf = symnext;
        symnext = symbols(t0 + 64);
      }
      {   // inputs of lane 0 for the next 64 steps, both jobs
        const int64_t cend = (t0 + 64 < width) ? t0 + 64 : width;
        if (s > 0 && cend > 0) wait_for((int32_t)cend);
        const int64_t off = t0 + lane;
        const bool inA = off < widthA, inB = hasB && off < widthB;
        const bool prev = s > 0 && off < avail;
        const uint32_t ha = (prev && inA) ? __hip_atomic_load(&iHA[off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const uint32_t fa = (prev && inA) ? __hip_atomic_load(&iFA[off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const uint32_t hb = (prev && inB) ? __hip_atomic_load(&iHB[off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const uint32_t fb = (prev && inB) ? __hip_atomic_load(&iFB[off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        hbuf = perm(hb, ha, 0x05040100u);   // A in the low half, B in the high half
        fbuf = perm(fb, fa, 0x05040100u);
      }
      // step t0 + tm; the next step's symbols are lane `nl` of `nsym`
      auto step = [&](int tm, uint32_t nsym, int nl) {
        const V16 hup = T::from(from_above(T::bits(hout), lane_value(hbuf, tm)));
        V16 F = T::from(from_above(T::bits(fout), lane_value(fbuf, tm)));
        const uint32_t cminA = from_above(cmoutA, 0u), cminB = from_above(cmoutB, 0u);
        const uint32_t symn = from_above(sym, lane_value(nsym, nl));
        uint32_t XnA[RL / 4], XnB[RL / 4];
        lds_load_words<RL>(s_profA + ((int64_t)(symn & 0xFFu) * 64 + lane) * RL, XnA);
        lds_load_words<RL>(s_profB + ((int64_t)((symn >> 8) & 0xFFu) * 64 + lane) * RL, XnB);

        uint32_t cmA = 0u, cmB = 0u;
        auto score_of = [&](int r) -> V16 { return T::from(perm(XB[r >> 2], XA[r >> 2], T::sel_const(r & 3))); };
        V16 u_next = M3 ? T::add(hup_prev, score_of(0)) : T::max(T::add(hup_prev, score_of(0)), E[0]);
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const V16 u = u_next;
          if (r + 1 < RL) {
            u_next = T::add(H[r], score_of(r + 1));
            if constexpr (!M3) u_next = T::max(u_next, E[r + 1]);
          }
          V16 hb;
          if constexpr (M3) hb = T::max3(u, E[r], F);
          else hb = T::max(u, F);
          const V16 hn = T::subs(hb, vbias);
          H[r] = hn;
          const uint32_t kc = (uint32_t)(RL - 1 - r);
          const uint32_t wa = perm(T::bits(hn), kc, selA), wb = perm(T::bits(hn), kc, selB);
          cmA = cmA > wa ? cmA : wa;
          cmB = cmB > wb ? cmB : wb;
          const V16 ho = HO ? hn : T::subs(hb, vo);   // HO: bias == o
          E[r] = T::max(T::subs(E[r], ve), ho);
          F = T::max(T::subs(F, ve), ho);
        }
        hup_prev = hup;
        hout = H[RL - 1];
        fout = F;
        const uint32_t cmlA = cmA + DL, cmlB = cmB + DL;
        cmoutA = cminA > cmlA ? cminA : cmlA;
        cmoutB = cminB > cmlB ? cminB : cmlB;
        sym = symn;
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) { XA[k] = XnA[k]; XB[k] = XnB[k]; }

        obH = shift_in(obH, T::bits(hout));
        obF = shift_in(obF, T::bits(fout));
        obCA = shift_in(obCA, cmoutA);
        obCB = shift_in(obCB, cmoutB);
      };
      const int tn = (int)(nsteps - t0 < 64 ? nsteps - t0 : 64);
      const int ta = tn < 62 ? tn : 62;
#pragma unroll 1
      for (int tm = 0; tm < ta; ++tm) step(tm, symbuf, tm + 1);
      if (tn > 62) {
        step(62, symbuf, 63);
        if (t0 >= 64) flush(t0 - 1, 63);   // step t0 + 62 ends offsets ..t0 - 1
      }
      if (tn > 63) step(63, symnext, 0);
      if (t0 + tn == nsteps) {   // the last step: the rest of the outputs
        const int64_t t = nsteps - 1;
        const int j = (int)((t - 63) & 63);
        if (t >= 63 && j != 63) flush(t - 63, j);
      }
    }
    publish((int32_t)width, true);
    if (spin_fail && lane == 0) {
      a.err[pA] = 1;
      if (hasB) a.err[pB] = 1;
    }
  }
}

// ---- end of the best alignment and score2 from the max array --------------
// Two phases: blocks (slice, pair) reduce a slice of one pair's max array to
// its best (value, column) -- the largest value, then the smallest column --
// and one block per pair reduces the slices.  T1 takes every column; T4
// skips the masked columns around the primary alignment.
constexpr int kSlices = 64;

__device__ __forceinline__ void better(int32_t &bv, int64_t &bj, int32_t v, int64_t j) {
  if (v > bv || (v == bv && j < bj)) { bv = v; bj = j; }
}

__device__ void block_best(int32_t &bv, int64_t &bj) {
  __shared__ int32_t sv[256];
  __shared__ int64_t sj[256];
  sv[threadIdx.x] = bv;
  sj[threadIdx.x] = bj;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      int32_t v = sv[threadIdx.x];
      int64_t j = sj[threadIdx.x];
      better(v, j, sv[threadIdx.x + w], sj[threadIdx.x + w]);
      sv[threadIdx.x] = v;
      sj[threadIdx.x] = j;
    }
    __syncthreads();
  }
  bv = sv[0];
  bj = sj[0];
  __syncthreads();
}

// mode 0: T1 over all columns; mode 1: T4 outside the mask
__global__ __launch_bounds__(256) void k_intra_slices(IntraPairArgs a, int mode) {
  const IntraPair ip = a.pairs[blockIdx.y];
  const int64_t p = ip.pair;
  const int64_t Lr = a.rlen[p];
  const uint32_t *mc = a.maxcol + ip.mc_off;
  int64_t lo = 1, hi = 0;   // masked columns [lo, hi]
  bool skip = false;
  if (mode == 1) {
    skip = a.score[p] <= 0;
    int64_t m = a.mask_len;
    if (m < 0) { m = a.qlen[p] / 2; if (m < 15) m = 15; }
    lo = a.rbeg[p] - m;
    hi = a.rend[p] + m;
  }
  const int64_t per = (Lr + kSlices - 1) / kSlices;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = (j0 + per < Lr) ? j0 + per : Lr;
  int32_t bv = 0;
  int64_t bj = INT64_MAX;
  if (!skip) {
    for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      if (j >= lo && j <= hi) continue;
      const int32_t v = (int32_t)(mc[j] >> ip.kbits);
      if (v > bv) { bv = v; bj = j; }
    }
  }
  block_best(bv, bj);
  if (threadIdx.x == 0) {
    a.part_v[(int64_t)blockIdx.y * kSlices + blockIdx.x] = bv;
    a.part_j[(int64_t)blockIdx.y * kSlices + blockIdx.x] = bj;
  }
}

__global__ __launch_bounds__(64) void k_intra_finish(IntraPairArgs a, int mode) {
  const IntraPair ip = a.pairs[blockIdx.x];
  const int64_t p = ip.pair;
  if (threadIdx.x != 0) return;
  int32_t bv = 0;
  int64_t bj = INT64_MAX;
  for (int k = 0; k < kSlices; ++k)
    better(bv, bj, a.part_v[(int64_t)blockIdx.x * kSlices + k],
           a.part_j[(int64_t)blockIdx.x * kSlices + k]);
  if (mode == 0) {
    const uint32_t M = (1u << ip.kbits) - 1u;
    if (bv > 0) {
      const int64_t qp = ((int64_t)a.qlen[p] + ip.sh - 1) / ip.sh * ip.sh;
      const uint32_t w = a.maxcol[ip.mc_off + bj];
      a.score[p] = bv;
      a.qend[p] = (int32_t)((int64_t)(M - (w & M)) - (qp - a.qlen[p]));
      a.rend[p] = bj;
    } else {
      a.score[p] = 0;
      a.qend[p] = -1;
      a.rend[p] = -1;
    }
    a.overflow[p] = 0;
  } else {
    a.score2[p] = bv;
    a.rend2[p] = bv > 0 ? bj : -1;
  }
}

// ---- fixed-capacity (graph) jobs: fixed counts and strides -----------------
// Fixed-capacity jobs cut into nc column chunks of cw_ columns per pair: job
// k * nc + c owns columns [c * cw_, (c + 1) * cw_) of pair k and starts W =
// Lq + floor(max(smax * Lq - o, 0) / e) + 1 columns early (no positive-scoring
// path is wider, so its owned columns are exact); with e = 0 chunk 0 owns the
// whole reference.  Chunks past the reference are empty.
__global__ void k_intra_jobs_chunked(int64_t B, int32_t nc, int64_t cw_, const int32_t *qlen,
                                     const int64_t *rlen, int32_t smax, int32_t o, int32_t e,
                                     int32_t kbits, int32_t sh, int64_t mc_stride,
                                     int64_t bnd_stride, IntraJob *jobs, IntraPair *pairs) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= B * nc) return;
  const int64_t k = x / nc;
  const int32_t c = (int32_t)(x % nc);
  const int64_t Lr = rlen[k], Lq = qlen[k];
  int64_t c0 = (int64_t)c * cw_, c1 = c0 + cw_, W = Lr;
  if (e > 0) {
    const int64_t gain = (int64_t)smax * Lq - o;
    W = Lq + (gain > 0 ? gain : 0) / e + 1;
  } else {
    c0 = c == 0 ? 0 : Lr;
    c1 = c == 0 ? Lr : Lr;
  }
  if (c1 > Lr) c1 = Lr;
  if (c0 > Lr) c0 = Lr;
  IntraJob jb{};
  jb.pair = k;
  jb.c0 = c0;
  jb.c1 = c1;
  jb.cw = c0 >= c1 ? c1 : (c0 - W > 0 ? c0 - W : 0);
  jb.mc_off = k * mc_stride;
  jb.bnd_off = x * bnd_stride;
  jb.kbits = kbits;
  jb.band = -1;
  jobs[x] = jb;
  if (c == 0) pairs[k] = IntraPair{k, k * mc_stride, kbits, sh};
}

hipError_t intra_jobs_chunked(int64_t B, int32_t nc, int64_t cw, const int32_t *qlen,
                              const int64_t *rlen, int32_t smax, int32_t o, int32_t e,
                              int32_t kbits, int32_t sh, int64_t mc_stride, int64_t bnd_stride,
                              IntraJob *jobs, IntraPair *pairs, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const int64_t n = B * nc;
  hipLaunchKernelGGL(k_intra_jobs_chunked, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B,
                     nc, cw, qlen, rlen, smax, o, e, kbits, sh, mc_stride, bnd_stride, jobs, pairs);
  return hipGetLastError();
}

__global__ void k_intra_rev_jobs_fixed(int64_t B, const int32_t *score, const int64_t *rend,
                                       const int32_t *band, int32_t kbits, int64_t bnd_stride,
                                       IntraJob *jobs) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= B) return;
  IntraJob jb{};
  jb.pair = k;
  jb.cw = 0;
  jb.c0 = 0;
  jb.c1 = score[k] > 0 ? rend[k] + 1 : 0;
  jb.mc_off = 0;
  jb.bnd_off = k * bnd_stride;
  jb.kbits = kbits;
  jb.band = band[k];
  jobs[k] = jb;
}

hipError_t intra_rev_jobs_fixed(int64_t B, const int32_t *score, const int64_t *rend,
                                const int32_t *band, int32_t kbits, int64_t bnd_stride,
                                IntraJob *jobs, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_intra_rev_jobs_fixed, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, B,
                     score, rend, band, kbits, bnd_stride, jobs);
  return hipGetLastError();
}

// ---- launchers ----------------------------------------------------------------
size_t intra_lds_bytes(int n, int RL) { return (size_t)(n + 1) * 64 * RL; }

template <int RL, bool HO>
static void launch_rl_ho(const IntraArgs &a, int waves, bool rev, hipStream_t st) {
  const dim3 b(64 * waves);
  const size_t lds = intra_lds_bytes(a.n, RL) * waves;
  if (a.segs > 1) {
    const dim3 g((unsigned)(8 * a.segs * ((a.njobs + 7) / 8)));
    if (rev) hipLaunchKernelGGL((k_intra_fill<RL, true, true, HO>), g, b, lds, st, a);
    else hipLaunchKernelGGL((k_intra_fill<RL, false, true, HO>), g, b, lds, st, a);
    return;
  }
  const dim3 g((unsigned)a.njobs);
  if (rev) hipLaunchKernelGGL((k_intra_fill<RL, true, false, HO>), g, b, lds, st, a);
  else hipLaunchKernelGGL((k_intra_fill<RL, false, false, HO>), g, b, lds, st, a);
}

// the bias is the gap open penalty: H and H - o are one value
template <int RL>
static void launch_rl(const IntraArgs &a, int waves, bool rev, hipStream_t st) {
  if (a.bias == a.o) launch_rl_ho<RL, true>(a, waves, rev, st);
  else launch_rl_ho<RL, false>(a, waves, rev, st);
}

__global__ void k_intra_sync_init(IntraSync *sync, int64_t njobs) {
  const int64_t j = blockIdx.x;
  if (j >= njobs) return;
  IntraSync &y = sync[j];
  for (int i = threadIdx.x; i < kIntraMaxStrips; i += blockDim.x) {
    y.prog[i] = 0;
    y.done[i] = 0;
    y.rcol[i] = -1;
    y.rrow[i] = -1;
  }
  if (threadIdx.x == 0) {
    y.best = ~0ull;
    y.fin = 0;
    y.pad_ = 0;
  }
}

hipError_t intra_sync_init(IntraSync *sync, int64_t njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_intra_sync_init, dim3((unsigned)njobs), dim3(256), 0, st, sync, njobs);
  return hipGetLastError();
}

template <int RL>
static void launch_rl16(const IntraArgs &a, int waves, bool m3, hipStream_t st) {
  const dim3 g((unsigned)(a.njobs / 2)), b(64 * waves);
  const size_t lds = intra_lds_bytes16(a.n, RL) * waves;
  if (a.bias == a.o) {   // H and H - o are one value
    if (m3) hipLaunchKernelGGL((k_intra_fill16<RL, true, true>), g, b, lds, st, a);
    else hipLaunchKernelGGL((k_intra_fill16<RL, false, true>), g, b, lds, st, a);
  } else {
    if (m3) hipLaunchKernelGGL((k_intra_fill16<RL, true, false>), g, b, lds, st, a);
    else hipLaunchKernelGGL((k_intra_fill16<RL, false, false>), g, b, lds, st, a);
  }
}

hipError_t intra_fill16(const IntraArgs &a, int RL, int waves, bool m3, hipStream_t st) {
  if (a.njobs == 0) return hipSuccess;
  if (waves < 1 || waves > kMaxWaves || (a.njobs & 1)) return hipErrorInvalidValue;
  switch (RL) {
    case 4: launch_rl16<4>(a, waves, m3, st); break;
    case 8: launch_rl16<8>(a, waves, m3, st); break;
    case 16: launch_rl16<16>(a, waves, m3, st); break;
    case 32: launch_rl16<32>(a, waves, m3, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t intra_lds_bytes16(int n, int RL) { return 2 * (size_t)(n + 1) * 64 * RL; }

hipError_t intra_fill(const IntraArgs &a, int RL, int waves, bool rev, hipStream_t st) {
  if (a.njobs == 0) return hipSuccess;
  if (waves < 1 || waves > kMaxWaves || (a.segs > 1 && !a.sync))
    return hipErrorInvalidValue;
  switch (RL) {
    case 4: launch_rl<4>(a, waves, rev, st); break;
    case 8: launch_rl<8>(a, waves, rev, st); break;
    case 16: launch_rl<16>(a, waves, rev, st); break;
    case 32: launch_rl<32>(a, waves, rev, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int intra_max_strips() { return kMaxStrips; }
int intra_max_waves() { return kMaxWaves; }
size_t intra_static_lds() { return 32 * 32 + kMaxStrips * (4 + 4 + 8 + 4) + 8 + 4; }

int intra_slices() { return kSlices; }

static hipError_t reduce(const IntraPairArgs &a, int64_t npairs, int mode, hipStream_t st) {
  for (int64_t b0 = 0; b0 < npairs; b0 += 65535) {
    const int64_t nb = (npairs - b0 < 65535) ? npairs - b0 : 65535;
    IntraPairArgs s = a;
    s.pairs = a.pairs + b0;
    s.part_v = a.part_v + b0 * kSlices;
    s.part_j = a.part_j + b0 * kSlices;
    hipLaunchKernelGGL(k_intra_slices, dim3(kSlices, (unsigned)nb), dim3(256), 0, st, s, mode);
    hipLaunchKernelGGL(k_intra_finish, dim3((unsigned)nb), dim3(64), 0, st, s, mode);
  }
  return hipGetLastError();
}

hipError_t intra_end(const IntraPairArgs &a, int64_t npairs, hipStream_t st) {
  if (npairs == 0) return hipSuccess;
  return reduce(a, npairs, 0, st);
}

hipError_t intra_score2(const IntraPairArgs &a, int64_t npairs, hipStream_t st) {
  if (npairs == 0) return hipSuccess;
  return reduce(a, npairs, 1, st);
}

}  // namespace swx
