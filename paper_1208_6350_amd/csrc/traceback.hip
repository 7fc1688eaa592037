// traceback.hip -- the banded pass that produces the detailed alignment.
//
// Method section: "the banded SW (whose band is defined by the beginning and
// ending positions) generates the detailed alignment".  For each pair the
// global 3-state DP on q[qbeg..qend] x r[rbeg..rend] is filled inside the
// safe band (every path of score score1 has at most G gap symbols, so it stays
// within a fixed set of diagonals; inside any superset of that set the DP
// values on those paths are exact), a 4-bit choice code is stored per cell,
// and the path is traced back from the end cell with rule T3 (M, then D, then
// I; inside a gap "open" before "extend").
//
// Layout: one lane per pair, 64 pairs of similar band width per wave.  The
// band of a lane is BW diagonals starting at its own lowest diagonal; BW is
// the task's width class (8, 16, 32 or 64), a superset of the lane's band.
// The previous row of H and F lives in registers; cells left of column 0 hold
// -inf and cells right of the last column only feed cells right of it, so no
// per-cell masking is needed.  Choice codes of one row are packed 8 per dword
// (the first cell in the top nibble) and stored lane-interleaved (coalesced).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

constexpr int32_t kNeg = -(1 << 29);
constexpr int64_t kTbMaxStripsDecl = 256;   // strips of one wave-traceback pair (kTbMaxStrips)

// Choice code of a cell: bit 3 "H does not come from the diagonal"
// (diag < H), bit 2 "F rather than E" (E < F), bit 1 "E extends" (the
// opening H - o < the extension E - e), bit 0 "F extends".  Each bit is the
// sign of a difference (every value here lies in [-2^30, 2^26]), shifted into
// the accumulator from the right, so a word fills from its top nibble down.
// Ties give M before E before F and "open" before "extend" (rule T3).
constexpr uint32_t kCodeNotM = 8u, kCodeF = 4u, kCodeEExt = 2u, kCodeFExt = 1u;
__device__ __forceinline__ uint32_t push_code(uint32_t acc, int32_t diag, int32_t h, int32_t eij,
                                              int32_t fij, int32_t eo, int32_t ex, int32_t fo,
                                              int32_t fx) {
  acc = __builtin_amdgcn_alignbit(acc, (uint32_t)(diag - h), 31);
  acc = __builtin_amdgcn_alignbit(acc, (uint32_t)(eij - fij), 31);
  acc = __builtin_amdgcn_alignbit(acc, (uint32_t)(eo - ex), 31);
  return __builtin_amdgcn_alignbit(acc, (uint32_t)(fo - fx), 31);
}
// the source of H named by a code: 0 diagonal, 1 E, 2 F
__device__ __forceinline__ uint32_t code_src(uint32_t c) {
  return (c & kCodeNotM) ? ((c & kCodeF) ? 2u : 1u) : 0u;
}
// The walk's moves (rule T3) by state (0 H, 1 E, 2 F) and choice code:
// nibble c of walk_moves(state) = next state << 2 | row up << 1 | column
// left.  In H the code names H's source: the diagonal (M, up and left) or a
// gap state; in E a D move left, staying in E while E extends; in F an I move
// up, staying in F while F extends.
constexpr uint64_t walk_moves(int state) {
  uint64_t t = 0;
  for (uint32_t c = 0; c < 16; ++c) {
    uint32_t v = 0;
    if (state == 0) {
      const uint32_t src = (c & kCodeNotM) ? ((c & kCodeF) ? 2u : 1u) : 0u;
      v = src == 0 ? 3u : (src << 2);
    } else if (state == 1) {
      v = ((c & kCodeEExt) ? 1u : 0u) << 2 | 1u;
    } else {
      v = ((c & kCodeFExt) ? 2u : 0u) << 2 | 2u;
    }
    t |= (uint64_t)v << (4 * c);
  }
  return t;
}
constexpr uint64_t kMovesH = walk_moves(0), kMovesE = walk_moves(1), kMovesF = walk_moves(2);

// row 0 of the global DP: reached from the left by one deletion run
__device__ __forceinline__ uint32_t row0_code(int64_t j, int32_t o, int32_t e) {
  return (j == 0) ? 0u : (kCodeNotM | ((j == 1 || o <= e) ? 0u : kCodeEExt));
}

__device__ __forceinline__ bool tb_coords_ok(const TbArgs &a, int64_t p) {
  return a.qbeg[p] >= 0 && a.qbeg[p] <= a.qend[p] && a.qend[p] < a.qlen[p] && a.rbeg[p] >= 0 &&
         a.rbeg[p] <= a.rend[p] && a.rend[p] < a.rlen[p];
}

// per pair: band class (0: none, 1..4: BW 8/16/32/64, 5: wider), rows, key
__global__ void k_tb_classify(TbArgs a, int64_t npairs, uint8_t *cls, uint64_t *key,
                              int64_t *vals, int64_t *ccap) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  uint8_t c = 0;
  int64_t m = 0, w = 0, bw = 0, dlo = 0;
  if (a.score[p] > 0) {
    if (tb_coords_ok(a, p)) {
      m = a.qend[p] - a.qbeg[p] + 1;
      w = a.rend[p] - a.rbeg[p] + 1;
      safe_band(m, w, a.score[p], a.smax, a.o, a.e, &dlo, &bw);
      // bands wider than 32 go to the strip kernel (a 64-wide band in one
      // lane's registers spills and leaves too few waves); pairs of more
      // than wave_cells band cells to the wave-parallel kernel
      const bool wave_fits = m <= int64_t(64) * 16 * kTbMaxStripsDecl;   // the wave kernel's strip limit
      c = (m * bw > a.wave_cells && wave_fits) ? 6 : bw <= 8 ? 1 : bw <= 16 ? 2 : bw <= 32 ? 3 : 5;
    } else {
      a.err[p] = 1;
    }
  }
  cls[p] = c;
  // class, then rows (clamped: only the grouping of similar heights matters);
  // wide bands (16 pairs share a task's column window, the union of their
  // bands) by rows in steps of 16, then lowest and highest diagonal, so that
  // a task's pairs have similar bands
  uint64_t sub = (uint64_t)(m > 0xFFFFF ? 0xFFFFF : m);
  if (c == 5) {
    const int64_t mq = m / 16 > 63 ? 63 : m / 16;
    const int64_t lo = -dlo < 0 ? 0 : (-dlo > 127 ? 127 : -dlo);
    const int64_t hi = dlo + bw - 1 + 32;
    sub = (uint64_t)(mq << 14) | (uint64_t)(lo << 7) | (uint64_t)(hi < 0 ? 0 : (hi > 127 ? 127 : hi));
  }
  key[p] = ((uint64_t)c << (kTbKeyBits - 3)) | sub;
  vals[p] = p;
  ccap[p] = (c != 0) ? (m + w + 2) : 0;
}

__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// tasks over sorted[n0 .. n1); with range (device) the bounds are read there
// and every task slot up to ntasks_cap is written (empty past the range).
// One wave per task, one lane per slot.
__global__ void k_tb_tasks(int64_t n0, int64_t n1, const int64_t *range, int64_t ntasks_cap,
                           const int64_t *sorted, const TbArgs a, int32_t bw, TbTask *tasks,
                           int64_t *dir_words) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (range) { n0 = range[0]; n1 = range[1]; }
  const int64_t ntasks = (n1 - n0 + 63) / 64;
  if (t >= (range ? ntasks_cap : ntasks)) return;
  if (t >= ntasks) {
    if (lane == 0) {
      tasks[t] = TbTask{};
      dir_words[t] = 0;
    }
    return;
  }
  const int64_t s0 = n0 + t * 64;
  const int64_t s1 = (s0 + 64 < n1) ? s0 + 64 : n1;
  int64_t rows = 1;
  if (s0 + lane < s1) {
    const int64_t p = sorted[s0 + lane];
    rows = a.qend[p] - a.qbeg[p] + 1;
  }
  rows = wave_max_i64(rows);
  if (lane != 0) return;
  TbTask tk{};
  tk.nslots = (int32_t)(s1 - s0);
  tk.rows = (int32_t)rows;
  tk.bw = bw;
  tk.slot_base = s0;
  tasks[t] = tk;
  dir_words[t] = (rows + 1) * (bw / 8) * 64;
}

__global__ void k_tb_offsets(int64_t ntasks, TbTask *tasks, const int64_t *off) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntasks) tasks[t].dir_off = off[t];
}

template <int BW, bool LUT4>
__global__ __launch_bounds__(256) void k_tb_band(TbArgs a, const TbTask *tasks, int64_t ntasks,
                                                 const int64_t *sorted) {
  __shared__ int8_t s_mat[32 * 32];
  __shared__ uint32_t s_lut4[32];   // LUT4: scores of query symbol x against reference 0..3
  constexpr int kRunSlots = 16;     // CIGAR runs per thread kept in LDS during the walk
  __shared__ uint32_t s_runs[(kRunSlots + 1) * 256];
  for (int k = threadIdx.x; k < a.n * a.n; k += blockDim.x) s_mat[k] = a.matrix[k];
  if (LUT4 && (int)threadIdx.x < a.n) {
    uint32_t l = 0;
    for (int b = 0; b < a.n; ++b) l |= (uint32_t)(uint8_t)a.matrix[threadIdx.x * a.n + b] << (8 * b);
    s_lut4[threadIdx.x] = l;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // tasks are sorted by rows, ascending: the largest go first, so that the
  // launch does not end on its longest tasks
  const int64_t k_ = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k_ >= ntasks) return;
  const int64_t tid = ntasks - 1 - k_;
  const TbTask tk = tasks[tid];
  if (tk.nslots == 0) return;
  const bool live = lane < tk.nslots;
  const int64_t p = live ? sorted[tk.slot_base + lane] : -1;
  int64_t m = 1, w = 1, dlo = 0, bwl = 1;
  int32_t s1 = 0;
  const int8_t *q = a.qcat, *r = a.rcat;
  if (live) {
    s1 = a.score[p];
    m = a.qend[p] - a.qbeg[p] + 1;
    w = a.rend[p] - a.rbeg[p] + 1;
    safe_band(m, w, s1, a.smax, a.o, a.e, &dlo, &bwl);
    q = a.qcat + a.qstart[p] + a.qbeg[p];
    r = a.rcat + a.rstart[p] + a.rbeg[p];
  }
  const int32_t o = a.o, e = a.e;
  uint32_t *dir = a.dir + tk.dir_off;
  constexpr int ND = BW / 8;        // direction dwords per row
  constexpr int NW = BW / 4 + 2;    // reference window dwords

  const int8_t *qq = live ? q : (const int8_t *)a.matrix;   // readable bytes for empty lanes
  const int8_t *rr = live ? r : (const int8_t *)a.matrix;
  const int64_t mq = live ? m : 1, wr = live ? w : 1;
  // reference window: byte k of the window = symbol at local column
  // base + k (1-based columns j use symbol r[j-1]); row i covers j = i+dlo+k.
  // Its bytes are loaded all at once (indices clamped into the sequence) and
  // masked afterwards.
  uint32_t win[NW];
  {
    const int64_t j0 = 1 + dlo;   // row 1, k = 0
    int32_t raw[4 * NW];
#pragma unroll
    for (int x = 0; x < 4 * NW; ++x) {
      int64_t y = j0 + x - 1;
      y = y < 0 ? 0 : (y > wr - 1 ? wr - 1 : y);
      raw[x] = rr[y];
    }
#pragma unroll
    for (int d = 0; d < NW; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t j = j0 + 4 * d + b;
        const int32_t c = (live && j >= 1 && j <= w) ? raw[4 * d + b] : 0;
        const uint32_t sy = (c >= 0 && c < a.n) ? (uint32_t)c : 0u;   // a bad code never indexes a table
        v |= (LUT4 ? sy * 8u : sy) << (8 * b);
      }
      win[d] = v;
    }
  }
  int32_t H[BW], F[BW];
  // row 0: H(0,0) = 0, H(0,j) = E(0,j) = -(o + (j-1)e); F(0,.) = -inf
  {
    uint32_t dw[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) dw[d] = 0;
#pragma unroll
    for (int k = 0; k < BW; ++k) {
      const int64_t j = dlo + k;
      int32_t h = kNeg;
      uint32_t c = 0;
      if (j == 0) h = 0;
      else if (j > 0) {
        h = -(o + (int32_t)(j - 1) * e);
        c = row0_code(j, o, e);
      }
      H[k] = h;
      F[k] = kNeg;
      dw[k >> 3] |= c << (4 * (7 - (k & 7)));
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) dir[(int64_t)d * 64 + lane] = dw[d];
  }
  int32_t hend = kNeg;
  const int64_t kend = w - m - dlo;
  // Rows go in blocks of UB: the query symbols and the window's next
  // reference bytes of block b+1 are requested while block b is computed.
  // The loads are unconditional (indices clamped into the sequences), so
  // they land straight in their registers; values outside the pair are
  // masked when decoded.
  constexpr int UB = BW <= 16 ? 8 : (BW <= 32 ? 4 : 2);
  // row and column arithmetic in 32 bits (pairs of this path are far
  // shorter than 2^31), so that clamps are single instructions
  const int32_t mq32 = (int32_t)mq, wr32 = (int32_t)wr, dlo32 = (int32_t)dlo;
  const int32_t m32 = (int32_t)m, w32 = (int32_t)w, rows32 = (int32_t)tk.rows;
  auto load_block = [&](int32_t i0, int32_t (&qo)[UB], int32_t (&no)[UB]) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int32_t x = i0 + u - 1;                       // query index of row i0 + u
      x = x < 0 ? 0 : (x > mq32 - 1 ? mq32 - 1 : x);
      qo[u] = qq[x];
      int32_t y = i0 + u + dlo32 + 4 * NW - 1;   // reference index of the window's new column
      y = y < 0 ? 0 : (y > wr32 - 1 ? wr32 - 1 : y);
      no[u] = rr[y];
    }
  };
  int32_t qraw[UB], nraw[UB];
  load_block(1, qraw, nraw);
  for (int32_t i0 = 1; i0 <= rows32; i0 += UB) {
    uint32_t qb[UB], nbb[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int32_t i = i0 + u;
      const int32_t c = (live && i <= m32) ? qraw[u] : -1;
      qb[u] = (c >= 0 && c < a.n) ? (uint32_t)c : 0xFFu;
      const int32_t j = i + 1 + dlo32 + 4 * NW - 1;   // 1-based column entering the window
      const int32_t cr = (live && j >= 1 && j <= w32) ? nraw[u] : 0;
      const uint32_t v = (cr >= 0 && cr < a.n) ? (uint32_t)cr : 0u;   // a bad code never indexes a table
      nbb[u] = LUT4 ? v * 8u : v;
    }
    load_block(i0 + UB, qraw, nraw);
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int32_t i = i0 + u;
      if (i > rows32) break;
      int32_t lut = 0, qrow = 0;
      if (qb[u] != 0xFFu) {
        if (LUT4) lut = (int32_t)s_lut4[qb[u]];
        else qrow = (int32_t)qb[u] * a.n;
      }
      uint32_t dw[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) dw[d] = 0;
      int32_t ev = kNeg, hleft = kNeg;
#pragma unroll
      for (int k = 0; k < BW; ++k) {
        const uint32_t sym = __builtin_amdgcn_ubfe(win[k >> 2], 8 * (k & 3), 8);
        const int32_t sc = LUT4 ? __builtin_amdgcn_sbfe(lut, sym, 8) : (int32_t)s_mat[qrow + sym];
        const int32_t hup = (k + 1 < BW) ? H[k + 1] : kNeg;
        const int32_t fup = (k + 1 < BW) ? F[k + 1] : kNeg;
        const int32_t diag = H[k] + sc;
        const int32_t fo = hup - o, fx = fup - e;
        const int32_t fij = fo > fx ? fo : fx;
        const int32_t eo = hleft - o, ex = ev - e;
        const int32_t eij = eo > ex ? eo : ex;
        int32_t h = diag > eij ? diag : eij;
        h = h > fij ? h : fij;
        dw[k >> 3] = push_code(dw[k >> 3], diag, h, eij, fij, eo, ex, fo, fx);
        H[k] = h;
        F[k] = fij;
        ev = eij;
        hleft = h;
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) dir[(i * ND + d) * 64 + lane] = dw[d];
      if (live && i == m32) {
#pragma unroll
        for (int k = 0; k < BW; ++k)
          if (k == kend) hend = H[k];
      }
      // slide the reference window one column to the right
#pragma unroll
      for (int d = 0; d < NW - 1; ++d) win[d] = __builtin_amdgcn_alignbyte(win[d + 1], win[d], 1);
      win[NW - 1] = (win[NW - 1] >> 8) | (nbb[u] << 24);
    }
  }
  if (!live) return;
  if (s1 <= 0) { a.cig_len[p] = 0; return; }
  if (hend != s1 || kend < 0 || kend >= BW) a.err[p] = 1;
  // Walk from (m, w) in state H.  D moves stay in their row and every other
  // move goes up exactly one row, so a lane handles row m - t at its t-th row
  // step: the lanes step through rows together, and each lane's row codes
  // stream in kWP rows ahead, loaded at the same point of every step.  The
  // walk itself issues no global store (a store between a load and its use
  // would make the wait for that load a wait for everything): runs go to
  // this thread's LDS slots, and are written out, in CIGAR order, after the
  // walk.  A lane whose runs outgrow its slots finishes on a plain walk.
  uint32_t *out = a.cig + a.cig_off[p];
  int32_t nruns = 0;
  int32_t i = m32, j = w32;   // 32-bit walk state
  int state = 0;
  uint32_t cur_op = 3, cur_len = 0;   // 3: no run yet
  // flags as 0/1 integers: lane booleans that live across the walk loop
  // would be kept as lane masks, merged with scalar instructions per move
  uint32_t walking = 1, bad = 0, full = 0;
  uint32_t pend = 0;
  // (a masked OR rather than a select chain, which the compiler would turn
  // into an indexed load from a private copy of the ring)
  auto code_at = [&](const uint32_t (&rc)[ND], int32_t k) -> uint32_t {
    const uint32_t idx = (uint32_t)(k >> 3);
    uint32_t word = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) word |= rc[d] & (0u - (uint32_t)(idx == (uint32_t)d));
    return (word >> (4 * (7 - (k & 7)))) & 0xFu;
  };
  // one move of the state machine from code c; returns the op (0xFF: none)
  auto move = [&](uint32_t c, bool &up) -> uint32_t {
    uint32_t op = 0xFF;
    up = false;
    if (state == 0) {
      const uint32_t src = code_src(c);
      if (src == 0 && i > 0 && j > 0) { op = 0; --i; --j; up = true; }
      else if (src == 1) state = 1;
      else state = 2;
    } else if (state == 1) {
      op = 2;
      state = (c & kCodeEExt) ? 1 : 0;
      --j;
    } else {
      op = 1;
      state = (c & kCodeFExt) ? 2 : 0;
      --i;
      up = true;
    }
    return op;
  };
  constexpr int kWP = 8;
  uint32_t ring[kWP][ND];
  // rows above row 0 are never walked: their slots load row 0, so that every
  // load lands straight in its ring registers
  auto load_row = [&](int32_t row, uint32_t (&dst)[ND]) {
    const int32_t rr = row >= 0 ? row : 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) dst[d] = dir[(rr * ND + d) * 64 + lane];
  };
#pragma unroll
  for (int u = 0; u < kWP; ++u) load_row(m - u, ring[u]);
  for (int32_t t0 = 0; t0 <= m32 && walking; t0 += kWP) {
#pragma unroll
    for (int u = 0; u < kWP; ++u) {   // no early exit: every step issues the same loads
      const int32_t row = m32 - (t0 + u);
      // the moves inside this row: D moves, then one M or I out of it.  One
      // move per iteration, in lane arithmetic rather than branches (the lanes
      // of a wave sit in different states): the move comes from walk_moves, the
      // run bookkeeping from 0/1 integers, and the finished run is stored
      // unconditionally into the next free slot (slot kRunSlots takes the
      // stores that end no run).
      for (int g = 0; g < 2 * BW + 4 && row >= 0 && walking; ++g) {
        const int32_t k = j - i - dlo32;
        const uint32_t ok = (uint32_t)(((k | (BW - 1 - k)) >= 0) & (i == row));
        const uint32_t c = code_at(ring[u], k);   // k out of range matches no word
        const uint64_t moves = state == 0 ? kMovesH : (state == 1 ? kMovesE : kMovesF);
        const uint32_t r = (uint32_t)(moves >> (4 * c)) & 15u;
        const uint32_t step = (r & 3u) * ok;          // 2 * (row up) + (column left)
        const uint32_t op = 3u - step;                // M 0, I 1, D 2; 3: no move
        const uint32_t moved = step != 0u;
        const uint32_t same = op == cur_op;
        const uint32_t ends = moved & (same ^ 1u) & (cur_len != 0u);
        const uint32_t run = (cur_len << 4) | cur_op;
        s_runs[nruns * 256 + threadIdx.x] = run;
        const uint32_t room = nruns < kRunSlots;
        nruns += ends & room;
        const uint32_t spill = ends & (room ^ 1u);   // no slot left: finish on the plain walk
        pend = spill ? run : pend;
        full |= spill;
        cur_len = moved ? (same ? cur_len + 1 : 1u) : cur_len;
        cur_op = moved ? op : cur_op;
        i -= (int32_t)(step >> 1);
        j -= (int32_t)(step & 1u);
        state = ok ? (int)(r >> 2) : state;
        bad |= ok ^ 1u;
        const uint32_t stop = (ok ^ 1u) | (uint32_t)((i | j) == 0) | full;
        walking &= stop ^ 1u;
        if (stop | (step >> 1)) break;   // the move went up a row
      }
      load_row(row - kWP, ring[u]);   // the slot is free again: kWP rows up
    }
  }
  if (full) {
    // the runs so far, the one that found no slot, then the rest of the walk
    for (int32_t x = 0; x < nruns; ++x) out[x] = s_runs[x * 256 + threadIdx.x];
    out[nruns++] = pend;
    int64_t guard = 2 * (m + w) + 4;
    while ((i > 0 || j > 0) && guard-- > 0) {
      const int32_t k = j - i - dlo32;
      if (k < 0 || k >= BW) { bad = true; break; }
      const uint32_t word = dir[(i * ND + (k >> 3)) * 64 + lane];
      bool up;
      const uint32_t op = move((word >> (4 * (7 - (k & 7)))) & 0xFu, up);
      if (op != 0xFF) {
        if (op == cur_op) ++cur_len;
        else {
          if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
          cur_op = op;
          cur_len = 1;
        }
      }
    }
  }
  if (bad || i != 0 || j != 0) a.err[p] = 1;
  if (full) {
    if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
    for (int32_t x = 0, y = nruns - 1; x < y; ++x, --y) {
      const uint32_t t = out[x]; out[x] = out[y]; out[y] = t;
    }
  } else {
    // runs were found end -> begin: write them reversed
    const int32_t total = nruns + (cur_len ? 1 : 0);
    if (cur_len) out[0] = (cur_len << 4) | cur_op;
    for (int32_t x = 0; x < nruns; ++x) out[total - 1 - x] = s_runs[x * 256 + threadIdx.x];
    nruns = total;
  }
  a.cig_len[p] = nruns;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t tb_classify(const TbArgs &a, int64_t npairs, uint8_t *cls, uint64_t *key, int64_t *vals,
                       int64_t *ccap, hipStream_t st) {
  if (!npairs) return hipSuccess;
  hipLaunchKernelGGL(k_tb_classify, dim3(nblk(npairs, 256)), dim3(256), 0, st, a, npairs, cls, key,
                     vals, ccap);
  return hipGetLastError();
}

hipError_t tb_tasks(int64_t n0, int64_t n1, const int64_t *sorted, const TbArgs &a, int32_t bw,
                    TbTask *tasks, int64_t *dir_words, hipStream_t st) {
  const int64_t nt = (n1 - n0 + 63) / 64;
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tb_tasks, dim3(nblk(nt, 4)), dim3(256), 0, st, n0, n1,
                     (const int64_t *)nullptr, (int64_t)0, sorted, a, bw, tasks, dir_words);
  return hipGetLastError();
}

hipError_t tb_tasks_range(const int64_t *range, int64_t ntasks_cap, const int64_t *sorted,
                          const TbArgs &a, int32_t bw, TbTask *tasks, int64_t *dir_words,
                          hipStream_t st) {
  if (ntasks_cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tb_tasks, dim3(nblk(ntasks_cap, 4)), dim3(256), 0, st, (int64_t)0,
                     (int64_t)0, range, ntasks_cap, sorted, a, bw, tasks, dir_words);
  return hipGetLastError();
}

hipError_t tb_offsets(int64_t ntasks, TbTask *tasks, const int64_t *off, hipStream_t st) {
  if (!ntasks) return hipSuccess;
  hipLaunchKernelGGL(k_tb_offsets, dim3(nblk(ntasks, 128)), dim3(128), 0, st, ntasks, tasks, off);
  return hipGetLastError();
}

template <int BW>
static hipError_t launch_band(const TbArgs &a, const TbTask *tasks, int64_t ntasks,
                              const int64_t *sorted, bool lut4, hipStream_t st) {
  const unsigned blocks = nblk(ntasks, 4);
  if (lut4)
    hipLaunchKernelGGL((k_tb_band<BW, true>), dim3(blocks), dim3(256), 0, st, a, tasks, ntasks, sorted);
  else
    hipLaunchKernelGGL((k_tb_band<BW, false>), dim3(blocks), dim3(256), 0, st, a, tasks, ntasks, sorted);
  return hipGetLastError();
}

hipError_t tb_band(const TbArgs &a, const TbTask *tasks, int64_t ntasks, const int64_t *sorted,
                   int32_t bw, hipStream_t st) {
  if (!ntasks) return hipSuccess;
  const bool lut4 = a.n <= 4;
  switch (bw) {
    case 8: return launch_band<8>(a, tasks, ntasks, sorted, lut4, st);
    case 16: return launch_band<16>(a, tasks, ntasks, sorted, lut4, st);
    case 32: return launch_band<32>(a, tasks, ntasks, sorted, lut4, st);
    default: return hipErrorInvalidValue;
  }
}


// ---- wide bands: row strips over four lanes, columns swept left to right ---
// A task holds kTbwSlots pairs; four consecutive lanes share one pair.  The
// task's strip s covers rows sR+1 .. sR+R (R = 16, 1-based, row 0 is the
// virtual row before the begin) and columns [clo(s), chi(s)): the unclipped
// window starts at c0(s) = sR + 1 + dlo_min and is W = R + (width of the union
// of the task's bands) columns wide, clipped to [0, wmax], so every pair
// computes a superset of its own safe band.  Lane g of a pair holds rows
// sR+4g+1 .. sR+4g+4 and at step t computes column clo + t - g: the H and F of
// its last row reach lane g+1 through a one-lane DPP shift, one step later,
// as the row above.  H and F of a strip's last row are handed to the next
// strip through global memory.  Lane g's four choice codes of step t (16 bits)
// are stored as half t & 1 of dword [s][t >> 1][g][slot], so that each store
// covers the whole wave with one 256-byte write.
namespace {
constexpr int kStripR = 16;                     // rows per strip
constexpr int kStripLP = 4;                     // lanes per pair
constexpr int kStripRL = kStripR / kStripLP;    // rows per lane
static_assert(kTbwSlots * kStripLP == 64, "one task per wave");

// columns of strip s and the code dwords a strip holds per (lane, slot)
__device__ __forceinline__ void strip_window(int64_t s, const TbwTask &tk, int64_t *clo,
                                             int64_t *chi) {
  const int64_t cstart = s * kStripR + 1 + tk.dlo;
  int64_t lo = cstart > 0 ? cstart : 0;
  int64_t hi = cstart + tk.width;
  if (hi > tk.wmax + 1) hi = tk.wmax + 1;
  *clo = lo;
  *chi = hi > lo ? hi : lo;
}
// lane k of each quad of lanes, to the whole quad (k a constant after unrolling)
__device__ __forceinline__ int32_t quad_bcast(int32_t x, int k) {
  switch (k) {
    // every source lane exists: no old value to keep
    case 0: return __builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, true);
    case 1: return __builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, true);
    case 2: return __builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, true);
    default: return __builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, true);
  }
}
__host__ __device__ __forceinline__ int64_t strip_dwords(int64_t width) {
  return (width + kStripLP) / 2;   // steps: at most width + kStripLP - 1
}
}  // namespace

__global__ void k_tbw_tasks(int64_t n0, int64_t n1, const int64_t *range, int64_t ntasks_cap,
                            const int64_t *sorted, const TbArgs a, TbwTask *tasks,
                            int64_t *dir_words, int64_t *bnd_words) {
  // one wave per task, one lane per slot
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (range) { n0 = range[0]; n1 = range[1]; }
  const int64_t ntasks = (n1 - n0 + kTbwSlots - 1) / kTbwSlots;
  if (t >= (range ? ntasks_cap : ntasks)) return;
  if (t >= ntasks) {
    if (lane == 0) {
      tasks[t] = TbwTask{};
      dir_words[t] = 0;
      bnd_words[t] = 0;
    }
    return;
  }
  const int64_t s0 = n0 + t * kTbwSlots;
  const int64_t s1 = (s0 + kTbwSlots < n1) ? s0 + kTbwSlots : n1;
  int64_t rows = 1, wmax = 1, ndlo_max = 0, dhi_max = 0;   // ndlo: -dlo, so all four are maxima
  if (lane < kTbwSlots && s0 + lane < s1) {
    const int64_t p = sorted[s0 + lane];
    const int64_t m = a.qend[p] - a.qbeg[p] + 1, w = a.rend[p] - a.rbeg[p] + 1;
    int64_t dlo, bw;
    safe_band(m, w, a.score[p], a.smax, a.o, a.e, &dlo, &bw);
    rows = m > rows ? m : rows;
    wmax = w > wmax ? w : wmax;
    ndlo_max = -dlo > ndlo_max ? -dlo : ndlo_max;
    dhi_max = (dlo + bw - 1) > dhi_max ? (dlo + bw - 1) : dhi_max;
  }
  rows = wave_max_i64(rows);
  wmax = wave_max_i64(wmax);
  const int64_t dlo_min = -wave_max_i64(ndlo_max);
  dhi_max = wave_max_i64(dhi_max);
  if (lane != 0) return;
  TbwTask tk{};
  tk.nslots = (int32_t)(s1 - s0);
  tk.rows = rows;
  tk.wmax = wmax;
  tk.dlo = dlo_min;
  tk.width = kStripR + (dhi_max - dlo_min + 1);
  tk.slot_base = s0;
  tasks[t] = tk;
  const int64_t nstrips = (rows + kStripR - 1) / kStripR;
  dir_words[t] = nstrips * strip_dwords(tk.width) * 64;
  bnd_words[t] = 2 * (wmax + 1) * kTbwSlots;
}

__global__ void k_tbw_offsets(int64_t ntasks, TbwTask *tasks, const int64_t *doff,
                              const int64_t *boff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntasks) { tasks[t].dir_off = doff[t]; tasks[t].bnd_off = boff[t]; }
}

template <bool LUT4>
__global__ __launch_bounds__(256) void k_tb_strip(TbArgs a, const TbwTask *tasks, int64_t ntasks,
                                                  const int64_t *sorted, int32_t *bndbuf) {
  constexpr int LP = kStripLP, RL = kStripRL, NS = kTbwSlots;
  constexpr int kCU = 16;   // walk cache: code dwords (32 steps) per lane
  __shared__ int8_t s_mat[32 * 32];
  __shared__ uint32_t s_walk[4 * 64 * kCU];
  for (int k = threadIdx.x; k < a.n * a.n; k += blockDim.x) s_mat[k] = a.matrix[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int g = lane & (LP - 1);        // row group of this lane
  const int slot = lane / LP;           // pair slot of the task
  // tasks are sorted by rows and band, ascending: the largest go first
  const int64_t k_ = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k_ >= ntasks) return;
  const int64_t tid = ntasks - 1 - k_;
  const TbwTask tk = tasks[tid];
  if (tk.nslots == 0) return;
  const bool live = slot < tk.nslots;
  const int64_t p = live ? sorted[tk.slot_base + slot] : -1;
  int64_t m = 1, w = 1, dlo = 0, bwl = 1;
  int32_t s1 = 0;
  const int8_t *q = a.qcat, *r = a.rcat;
  if (live) {
    s1 = a.score[p];
    m = a.qend[p] - a.qbeg[p] + 1;
    w = a.rend[p] - a.rbeg[p] + 1;
    safe_band(m, w, s1, a.smax, a.o, a.e, &dlo, &bwl);
    q = a.qcat + a.qstart[p] + a.qbeg[p];
    r = a.rcat + a.rstart[p] + a.rbeg[p];
  }
  const int32_t o = a.o, e = a.e;
  uint32_t *dir = a.dir + tk.dir_off;
  int32_t *bH = bndbuf + tk.bnd_off;
  int32_t *bF = bH + (tk.wmax + 1) * NS;
  const int64_t SW = strip_dwords(tk.width);
  // row 0 (virtual): H(0,0) = 0, H(0,j) = -(o + (j-1)e), F = -inf; the walk
  // decodes row 0 itself, so it has no stored codes
  for (int64_t j = g; j <= tk.wmax; j += LP) {
    bH[j * NS + slot] = (j == 0) ? 0 : -(o + (int32_t)(j - 1) * e);
    bF[j * NS + slot] = kNeg;
  }
  const int64_t nstrips = (tk.rows + kStripR - 1) / kStripR;
  int32_t plo = 0, phi = (int32_t)tk.wmax + 1;   // columns of row sR that hold valid values
  const int8_t *rr = live ? r : (const int8_t *)a.matrix;   // readable bytes for empty slots
  const int8_t *qq = live ? q : (const int8_t *)a.matrix;
  const int64_t mq = live ? m : 1;
  for (int64_t s = 0; s < nstrips; ++s) {
    const int64_t sR = s * kStripR;
    int64_t clo64, chi64;
    strip_window(s, tk, &clo64, &chi64);
    // 32-bit column and step arithmetic (a strip task spans well under 2^31
    // code dwords), so that the block's addresses stay in few registers
    const int32_t clo = (int32_t)clo64, chi = (int32_t)chi64;
    const int32_t ncol = chi - clo;
    const int32_t nsteps = ncol + LP - 1;
    const int32_t wmax = (int32_t)tk.wmax, wl = (int32_t)w;
    uint32_t *sdir = dir + s * SW * 64;
    // this lane's rows: score tables
    int32_t lut[RL], qn[RL], qraw[RL];
#pragma unroll
    for (int k = 0; k < RL; ++k) {   // all loads first (clamped), then decode
      int64_t x = sR + g * RL + k;
      x = x > mq - 1 ? mq - 1 : x;
      qraw[k] = qq[x];
    }
#pragma unroll
    for (int k = 0; k < RL; ++k) {
      const int64_t i = sR + g * RL + 1 + k;
      lut[k] = 0;
      qn[k] = 0;
      const int32_t qs = (live && i <= m) ? qraw[k] : -1;
      if (qs >= 0 && qs < a.n) {   // a bad code never indexes a table
        if (LUT4) {
          uint32_t l = 0;
          for (int b = 0; b < a.n; ++b) l |= (uint32_t)(uint8_t)s_mat[qs * a.n + b] << (8 * b);
          lut[k] = (int32_t)l;
        } else {
          qn[k] = qs * a.n;
        }
      }
    }
    int32_t H[RL], E[RL], HO[RL];   // HO = H - o: the E opening of the next column
#pragma unroll
    for (int k = 0; k < RL; ++k) { H[k] = kNeg; E[k] = kNeg; HO[k] = kNeg - o; }
    // H of the row above at the previous column (lane 0: row sR at clo - 1)
    int32_t hdiag0 = kNeg;
    if (g == 0 && clo >= 1 && clo - 1 >= plo && clo - 1 < phi) hdiag0 = bH[(clo - 1) * NS + slot];
    int32_t xh = kNeg, xf = kNeg;   // last row's H, F of the previous step
    uint32_t xs = 0;                // reference symbol of the previous step
    // Steps go in blocks of kPB.  Lane 0 of a pair consumes the row above and
    // the reference symbol of its column; the pair's four lanes load them, a
    // quarter each, and hand them over by a DPP broadcast inside the lane
    // quad (the other lanes take theirs from the lane before).  The strip's
    // last row goes the other way: lane 3 broadcasts it and the lanes keep
    // a quarter each for the boundary stores.  At the top of a block the wave
    // waits for the block's operands (requested one block earlier), then
    // stores the previous block's codes and boundary values and requests the
    // next block's operands, and only then computes.
    constexpr int kPB = 4;   // (8 leaves three waves per SIMD, 4 leaves four)
    constexpr int kPV = kPB / LP;   // columns per lane and block
    int32_t n_h[kPV], n_f[kPV], n_c[kPV];
    // lane g loads columns clo + t0 + g + LP * v of the block
    auto fetch_block = [&](int32_t t0) {
#pragma unroll
      for (int v = 0; v < kPV; ++v) {
        int32_t j = clo + t0 + g + LP * v;
        j = j < 0 ? 0 : (j > wmax ? wmax : j);
        n_h[v] = bH[j * NS + slot];
        n_f[v] = bF[j * NS + slot];
        int32_t x = clo + t0 + g + LP * v - 1;
        x = x < 0 ? 0 : (x > wl - 1 ? wl - 1 : x);
        n_c[v] = (int32_t)rr[x];
      }
    };
    uint32_t p_code[kPB / 2];
    int32_t p_h[kPV], p_f[kPV];   // last row of step g + LP * v of the pending block
    int32_t p_t0 = -1;   // first step of the pending block (-1: none)
    auto flush = [&]() {
      if (p_t0 < 0) return;
#pragma unroll
      for (int u = 0; u < kPB / 2; ++u)
        if (p_t0 + 2 * u < nsteps) sdir[((p_t0 >> 1) + u) * 64 + lane] = p_code[u];
#pragma unroll
      for (int v = 0; v < kPV; ++v) {
        const int32_t t = p_t0 + g + LP * v, j = clo + t - (LP - 1);
        if (t >= LP - 1 && t < nsteps) {
          bH[j * NS + slot] = p_h[v];
          bF[j * NS + slot] = p_f[v];
        }
      }
    };
    fetch_block(0);
    for (int32_t t0 = 0; t0 < nsteps; t0 += kPB) {
      int32_t c_h[kPV], c_f[kPV];
      int32_t c_sy[kPV];
#pragma unroll
      for (int v = 0; v < kPV; ++v) {
        const int32_t j = clo + t0 + g + LP * v;
        const bool inprev = j >= plo && j < phi;
        c_h[v] = inprev ? n_h[v] : kNeg;
        c_f[v] = inprev ? n_f[v] : kNeg;
        const int32_t c = (live && j >= 1 && j <= wl) ? n_c[v] : -1;
        c_sy[v] = (c >= 0 && c < a.n) ? c : 0;
      }
      // the operands are consumed (waited for) before any store is issued
      __builtin_amdgcn_sched_barrier(0);
      flush();
      fetch_block(t0 + kPB);   // past the window too: clamped, and never used
      uint32_t acc = 0;
#pragma unroll
      for (int u = 0; u < kPB; ++u) {
        const int32_t t = t0 + u;
        // lane 0's operands: from lane u % 4 of the quad
        const int32_t bh = quad_bcast(c_h[u / LP], u & (LP - 1));
        const int32_t bf = quad_bcast(c_f[u / LP], u & (LP - 1));
        const int32_t bs = quad_bcast(c_sy[u / LP], u & (LP - 1));
        // the other lanes': from the lane before (its last row, one step earlier)
        // (lane 0 of each row of 16 has no source and reads 0; it is a
        // pair's lane 0, which takes the loaded operands instead)
        const int32_t dh = __builtin_amdgcn_mov_dpp(xh, 0x111, 0xF, 0xF, true);
        const int32_t df = __builtin_amdgcn_mov_dpp(xf, 0x111, 0xF, 0xF, true);
        const int32_t ds = __builtin_amdgcn_mov_dpp((int32_t)xs, 0x111, 0xF, 0xF, true);
        const int32_t hup0 = g == 0 ? bh : dh;
        const int32_t fup0 = g == 0 ? bf : df;
        const uint32_t sym = (uint32_t)(g == 0 ? bs : ds);
        uint32_t code = 0;
        if (t >= g && t < g + ncol) {
          const uint32_t sym8 = LUT4 ? sym * 8u : sym;
          int32_t hdiag = hdiag0;
          hdiag0 = hup0;
          int32_t hupo = hup0 - o, fup = fup0;   // hupo: H of the row above, minus o
#pragma unroll
          for (int k = 0; k < RL; ++k) {
            const int32_t sc = LUT4 ? __builtin_amdgcn_sbfe(lut[k], sym8, 8) : (int32_t)s_mat[qn[k] + sym];
            const int32_t diag = hdiag + sc;
            const int32_t fo = hupo, fx = fup - e;
            const int32_t fij = fo > fx ? fo : fx;
            const int32_t eo = HO[k], ex = E[k] - e;      // row k at column j-1
            const int32_t eij = eo > ex ? eo : ex;
            int32_t h = diag > eij ? diag : eij;
            h = h > fij ? h : fij;
            code = push_code(code, diag, h, eij, fij, eo, ex, fo, fx);   // row k: bits 4(RL-1-k)
            hdiag = H[k];
            H[k] = h;
            E[k] = eij;
            hupo = h - o;
            HO[k] = hupo;
            fup = fij;
          }
          const int32_t hup = H[RL - 1];
          xh = hup;
          xf = fup;
        }
        xs = sym;
        // lane 3's last row, kept by lane u % 4
        const int32_t lh = quad_bcast(xh, LP - 1);
        const int32_t lf = quad_bcast(xf, LP - 1);
        if (g == (u & (LP - 1))) {
          p_h[u / LP] = lh;
          p_f[u / LP] = lf;
        }
        acc |= code << (16 * (u & 1));
        if (u & 1) {
          p_code[u >> 1] = acc;
          acc = 0;
        }
      }
      p_t0 = t0;
    }
    flush();   // the strip's last block, before the next strip reads it
    plo = clo;
    phi = chi;
  }
  if (!live) return;
  if (s1 <= 0) {
    if (g == 0) a.cig_len[p] = 0;
    return;
  }
  // Traceback from (m, w) in state H.  The four lanes of a pair walk it
  // together.  Each lane keeps kCU code dwords of its own row group of the
  // current strip in the pair's LDS slots (a window of columns ending at the
  // column where it was filled; the walk only moves up and left).  On entering
  // a strip the lanes also request the strip above, ending at the current
  // column, into registers: when the walk gets there, the window is written
  // to LDS from those registers without waiting for memory.  Only a walk
  // that leaves a window sideways waits for a load.
  uint32_t *out = a.cig + a.cig_off[p];
  int32_t nruns = 0;
  // (32-bit walk state: a strip task spans well under 2^31 code dwords)
  int32_t i = (int32_t)m, j = (int32_t)w;
  int state = 0;
  uint32_t cur_op = 3, cur_len = 0;   // 3: no run yet
  int64_t guard = 2 * (m + w) + 4;
  uint32_t *cache = s_walk + ((threadIdx.x >> 6) * 64 + slot * LP) * kCU;   // [g][kCU]
  int32_t cache_s = -1, cache_j = -1;
  uint32_t pfx[kCU];              // the strip above, in flight
  int32_t pf_s = -1, pf_j = -1;
  const int32_t SW32 = (int32_t)SW, dlo32 = (int32_t)tk.dlo, width32 = (int32_t)tk.width;
  const int32_t wmax32 = (int32_t)tk.wmax;
  auto window32 = [&](int32_t s, int32_t &clo, int32_t &chi) {   // strip_window in 32 bits
    const int32_t cstart = s * kStripR + 1 + dlo32;
    clo = cstart > 0 ? cstart : 0;
    int32_t hi = cstart + width32;
    hi = hi > wmax32 + 1 ? wmax32 + 1 : hi;
    chi = hi > clo ? hi : clo;
  };
  auto fetch_window = [&](int32_t s, int32_t jj, uint32_t (&dst)[kCU]) {
    int32_t clo, chi;
    window32(s, clo, chi);
    const int32_t mytop = (jj - clo + g) >> 1;
#pragma unroll
    for (int x = 0; x < kCU; ++x) {
      int32_t uu = mytop - x;
      uu = uu < 0 ? 0 : (uu > SW32 - 1 ? SW32 - 1 : uu);   // clamped: never read outside the strip
      dst[x] = dir[(s * SW32 + uu) * 64 + slot * LP + g];
    }
  };
  bool bad = false;
  while ((i > 0 || j > 0) && guard-- > 0) {
    uint32_t c;
    if (i == 0) {
      c = row0_code(j, o, e);
    } else {
      const int32_t s = (i - 1) / kStripR, k = (i - 1) % kStripR;
      const int32_t gk = k / RL;
      int32_t clo, chi;
      window32(s, clo, chi);
      if (j < clo || j >= chi) { bad = true; break; }
      const int32_t t = j - clo + gk;
      // cached: dwords (cache_j - clo + g) / 2 - kCU + 1 .. (cache_j - clo + g) / 2 of row group g
      const int32_t top = (cache_j - clo + gk) >> 1;
      if (s != cache_s || (t >> 1) > top || (t >> 1) <= top - kCU) {
        const int32_t ptop = (pf_j - clo + gk) >> 1;
        const bool use_pf = s == pf_s && (t >> 1) <= ptop && (t >> 1) > ptop - kCU;
        if (use_pf) {
#pragma unroll
          for (int x = 0; x < kCU; ++x) cache[g * kCU + x] = pfx[x];
          cache_j = pf_j;
        } else {
          uint32_t now[kCU];
          fetch_window(s, j, now);
#pragma unroll
          for (int x = 0; x < kCU; ++x) cache[g * kCU + x] = now[x];
          cache_j = j;
        }
        if (s != cache_s && s > 0) {   // a new strip: request the one above
          fetch_window(s - 1, j, pfx);
          pf_s = s - 1;
          pf_j = j;
        }
        cache_s = s;
      }
      const int32_t top2 = (cache_j - clo + gk) >> 1;
      const uint32_t dwv = cache[gk * kCU + (top2 - (t >> 1))];
      c = (dwv >> (16 * (t & 1) + 4 * (RL - 1 - k % RL))) & 0xFu;
    }
    // the move from the per-state table (M 0, I 1, D 2; 3: a change of state)
    const uint64_t moves = state == 0 ? kMovesH : (state == 1 ? kMovesE : kMovesF);
    const uint32_t r = (uint32_t)(moves >> (4 * c)) & 15u;
    const uint32_t step = r & 3u, op = 3u - step;
    i -= (int32_t)(step >> 1);
    j -= (int32_t)(step & 1u);
    state = (int)(r >> 2);
    if (step) {
      if (op == cur_op) ++cur_len;
      else {
        if (cur_len && g == 0) out[nruns] = (cur_len << 4) | cur_op;
        if (cur_len) ++nruns;
        cur_op = op;
        cur_len = 1;
      }
    }
  }
  if (g != 0) return;
  if (bad || i != 0 || j != 0) a.err[p] = 1;
  if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
  for (int32_t x = 0, y = nruns - 1; x < y; ++x, --y) {
    const uint32_t t = out[x]; out[x] = out[y]; out[y] = t;
  }
  a.cig_len[p] = nruns;
}

// ---- wave-parallel traceback (long pairs with wide bands) -------------------
// One pair per workgroup.  Lane k holds rows [k*RL+1, (k+1)*RL] of a strip of
// 64*RL rows and computes column c - k at step c; the H and F leaving a lane's
// last row move one lane down per step through a DPP shift, as in the
// intra-sequence fill.  Each step stores the lane's RL choice codes (same
// 4-bit code as the per-lane kernels, RL/2 bytes) at [step][lane], so a
// strip's codes are written with coalesced stores.  The walk then runs on the
// whole wave with uniform state, copying the codes of up to 32 KiB of steps
// at a time (a contiguous range: steps [t - TS + 1, t] of the current strip)
// into LDS with 16-byte loads: the walk only moves to smaller steps and lanes
// inside a strip, so each copy serves many moves.  RL is chosen per pair on
// the host: short lanes shorten the chain of strips and the work per step,
// tall ones hold longer queries within the strip limit.
__device__ __forceinline__ int32_t tb_from_above(int32_t src, int32_t top) {
  return __builtin_amdgcn_update_dpp(top, src, 0x138, 0xF, 0xF, false);   // wave_shr:1
}

constexpr int kTbMaxStrips = (int)kTbMaxStripsDecl;
constexpr int kTbMaxWaves = 8;
constexpr int64_t kTbSpinLimit = int64_t(1) << 26;
constexpr int kTbTileBytes = 32768;

// RL score bytes of the LDS profile as RL/4 words
template <int RL>
__device__ __forceinline__ void tb_prof_load(const int8_t *src, uint32_t (&w)[RL / 4]) {
  if constexpr (RL == 16) {
    const uint4 v = *reinterpret_cast<const uint4 *>(src);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  } else if constexpr (RL == 8) {
    const uint2 v = *reinterpret_cast<const uint2 *>(src);
    w[0] = v.x; w[1] = v.y;
  } else {
    w[0] = *reinterpret_cast<const uint32_t *>(src);
  }
}

// The walk back along the path (rule T3) over one pair's stored codes, by
// one wave (uniform state); defined below.
template <int RL>
__device__ void tb_wave_walk(const TbArgs &a, const TbWaveJob &jb, const uint8_t *dir,
                             uint4 *s_tile, int lane);

// SPREAD: the pair's strips on the waves of `segs` workgroups (progress
// records in global memory, agent scope, as in the intra-sequence fill; the
// grid fits on the device at once), and the walk left to k_tb_walk.
template <int RL, bool SPREAD>
__global__ __launch_bounds__(64 * kTbMaxWaves) void k_tb_wave(TbArgs a, const TbWaveJob *jobs,
                                                              int64_t njobs, int segs,
                                                              IntraSync *sync, uint8_t *dirw,
                                                              int32_t *bndbuf) {
  constexpr int64_t SH = 64 * RL;
  constexpr int WB = RL / 2;                      // code bytes per lane and step
  extern __shared__ uint4 s_dyn[];                // per wave: profile [(n+1)][64][RL] score bytes
  __shared__ uint4 s_tile[SPREAD ? 1 : kTbTileBytes / 16];
  __shared__ int8_t s_mat[32 * 32];
  __shared__ int32_t l_prog[SPREAD ? 1 : kTbMaxStrips];   // columns of strip s's last row published
  __shared__ int32_t l_done[SPREAD ? 1 : kTbMaxStrips];
  constexpr int SCOPE = SPREAD ? __HIP_MEMORY_SCOPE_AGENT : __HIP_MEMORY_SCOPE_WORKGROUP;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  // spread grids: block 8 * slot + x (slot = (j / 8) * G + segment) puts the
  // segments of job j on XCD j % 8; blocks past the last job leave at once
  const int G = SPREAD ? segs : 1;
  int64_t jix = blockIdx.x, seg = 0;
  if constexpr (SPREAD) {
    const int64_t slot = blockIdx.x / 8;
    jix = (slot / G) * 8 + blockIdx.x % 8;
    seg = slot % G;
    if (jix >= njobs) return;
  }
  int32_t *s_prog = SPREAD ? sync[jix].prog : l_prog;
  int32_t *s_done = SPREAD ? sync[jix].done : l_done;
  const TbWaveJob jb = jobs[jix];
  if (jb.m <= 0) return;   // a job without an alignment (one-pair graphs plan it on the device)
  const int64_t p = jb.pair, m = jb.m, w = jb.w;
  const int n = a.n;
  const int32_t o = a.o, e = a.e;
  const int64_t nstrips = (m + SH - 1) / SH;
  uint8_t *dir = dirw + jb.dir_off;
  for (int k = threadIdx.x; k < n * n; k += blockDim.x) s_mat[k] = a.matrix[k];
  if constexpr (!SPREAD) {   // spread jobs: set by intra_sync_init before the launch
    for (int k = threadIdx.x; k < nstrips && k < kTbMaxStrips; k += blockDim.x) {
      s_prog[k] = 0;
      s_done[k] = 0;
    }
  }
  const int8_t *q = a.qcat + a.qstart[p] + a.qbeg[p];
  const int8_t *r = a.rcat + a.rstart[p] + a.rbeg[p];
  // hand-over rows: row 0 is the virtual top row H(0,0) = 0,
  // H(0,j) = -(o + (j-1)e), F(0,j) = -inf; row s + 1 is strip s's last row
  int32_t *bnd0 = bndbuf + jb.bnd_off;
  if (seg == 0) {   // strip 0 (segment 0, wave 0) reads it after the barrier below
    for (int64_t j = threadIdx.x; j <= w; j += blockDim.x) {
      bnd0[j] = (j == 0) ? 0 : -(o + (int32_t)(j - 1) * e);
      bnd0[(w + 1) + j] = kNeg;
    }
  }
  __threadfence_block();
  __syncthreads();
  int8_t *s_prof = reinterpret_cast<int8_t *>(s_dyn) + (size_t)wave * (n + 1) * 64 * RL;
  bool spin_fail = false;

  // choice codes of strip s start this many bytes after those of strip 0
  auto strip_base = [&](int64_t s) {
    int64_t off = 0;
    for (int64_t k = 0; k < s; ++k) {
      int64_t lo, hi;
      tbw_window(k, SH, jb.dlo, jb.bw, w, &lo, &hi);
      off += ((hi - lo) + 63) * 64 * WB;
    }
    return off;
  };

  for (int64_t s = seg * NW + wave; s < nstrips; s += (int64_t)G * NW) {
    int64_t clo, chi, plo = 0, phi = w + 1;
    tbw_window(s, SH, jb.dlo, jb.bw, w, &clo, &chi);
    if (s > 0) tbw_window(s - 1, SH, jb.dlo, jb.bw, w, &plo, &phi);
    const int32_t *inH = bnd0 + 2 * (w + 1) * s;    // the row above this strip
    const int32_t *inF = inH + (w + 1);
    int32_t *outH = bnd0 + 2 * (w + 1) * (s + 1);   // this strip's last row
    int32_t *outF = outH + (w + 1);
    const bool hand_over = (s + 1 < nstrips);
    uint8_t *dstrip = dir + strip_base(s);
    auto publish = [&](int32_t ncols, bool fin) {
      if constexpr (SPREAD) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) {
        __hip_atomic_store(&s_prog[s], ncols, __ATOMIC_RELAXED, SCOPE);
        if (fin) __hip_atomic_store(&s_done[s], 1, __ATOMIC_RELAXED, SCOPE);
      }
    };
    int32_t avail = (s == 0) ? (int32_t)(w + 1) : 0;
    auto wait_for = [&](int32_t need) {
      if (s == 0) return;
      int64_t spins = 0;
      for (;;) {
        const int32_t done = __hip_atomic_load(&s_done[s - 1], __ATOMIC_RELAXED, SCOPE);
        avail = __hip_atomic_load(&s_prog[s - 1], __ATOMIC_RELAXED, SCOPE);
        if (done || avail >= need) break;
        if (++spins > kTbSpinLimit) { spin_fail = true; break; }
        __builtin_amdgcn_s_sleep(2);
      }
      if constexpr (SPREAD) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    auto rd = [](const int32_t *ptr) {   // past the L1: another wave wrote it
      return __hip_atomic_load(ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // profile of this lane's rows (signed scores; padding rows score 0)
    {
      int32_t qv[RL];
#pragma unroll
      for (int k = 0; k < RL; ++k) {
        const int64_t i = s * SH + lane * RL + k + 1;
        qv[k] = (i <= m) ? (int32_t)q[i - 1] : -1;
      }
      for (int sy = 0; sy <= n; ++sy) {
        uint32_t wv[RL / 4];
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) wv[k] = 0u;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const uint32_t b = (qv[k] >= 0 && sy < n) ? (uint32_t)(uint8_t)s_mat[qv[k] * n + sy] : 0u;
          wv[k >> 2] |= b << (8 * (k & 3));
        }
        uint32_t *dst = reinterpret_cast<uint32_t *>(s_prof + ((int64_t)sy * 64 + lane) * RL);
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) dst[k] = wv[k];
      }
    }
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
    int32_t H[RL], E[RL];
#pragma unroll
    for (int k = 0; k < RL; ++k) { H[k] = kNeg; E[k] = kNeg; }
    int32_t hup_prev = kNeg;
    if (clo >= 1 && clo - 1 >= plo && clo - 1 < phi) {
      wait_for((int32_t)(clo - plo));
      if (lane == 0 && clo - 1 < plo + avail) hup_prev = rd(&inH[clo - 1]);
    }
    int32_t hout = kNeg, fout = kNeg;
    int32_t hbuf = kNeg, fbuf = kNeg;
    int32_t obH = 0, obF = 0;
    const int64_t nsteps = (chi - clo) + 63;
    // reference symbols of columns [c0, c0 + 64) at lane c - c0; the profile
    // row of a step is read one step ahead (its symbol is the one the lane
    // above holds now)
    auto symbols = [&](int64_t c0) -> int32_t {
      const int64_t c = c0 + lane;
      return (c < chi && c >= 1) ? (int32_t)(uint8_t)r[c - 1] : n;
    };
    int32_t symbuf = symbols(clo), symnext = symbols(clo + 64);
    uint32_t sym = (uint32_t)tb_from_above(n, __builtin_amdgcn_readlane(symbuf, 0));
    uint32_t X[RL / 4];
    tb_prof_load<RL>(s_prof + ((int64_t)sym * 64 + lane) * RL, X);
    // Steps in blocks of 64: the block's start reads the symbols and the row
    // above for its 64 columns; step t gathers lane 63's H and F of column
    // clo + t - 63 into lane (t - 63) mod 64 (from step 63 on), and step 62
    // of every block after the first completes 64 such columns.
#pragma unroll 1
    for (int64_t t0 = 0; t0 < nsteps; t0 += 64) {
      if (t0 > 0) {
        symbuf = symnext;
        symnext = symbols(clo + t0 + 64);
      }
      {
        const int64_t cend = (clo + t0 + 64 < phi) ? clo + t0 + 64 : phi;
        if (cend > plo) wait_for((int32_t)(cend - plo));
        const int64_t c = clo + t0 + lane;
        const bool prev = c < chi && c >= plo && c < phi && c < plo + avail;
        hbuf = prev ? rd(&inH[c]) : kNeg;
        fbuf = prev ? rd(&inF[c]) : kNeg;
      }
      // step t0 + tm; the next step's symbol is lane `nl` of `nsym`; gather:
      // the step has a column to hand over (t >= 63)
      auto step = [&](int tm, int32_t nsym, int nl, bool gather) {
        const int64_t t = t0 + tm;
        const int32_t hup = tb_from_above(hout, __builtin_amdgcn_readlane(hbuf, tm));
        int32_t fup = tb_from_above(fout, __builtin_amdgcn_readlane(fbuf, tm));
        const uint32_t symn = (uint32_t)tb_from_above((int32_t)sym, __builtin_amdgcn_readlane(nsym, nl));
        uint32_t Xn[RL / 4];
        tb_prof_load<RL>(s_prof + ((int64_t)symn * 64 + lane) * RL, Xn);
        int32_t hdiag = hup_prev;
        int32_t hcur = hup;
        uint32_t dw[(RL + 7) / 8];
#pragma unroll
        for (int k = 0; k < (RL + 7) / 8; ++k) dw[k] = 0u;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int32_t sc = __builtin_amdgcn_sbfe((int32_t)X[k >> 2], 8 * (k & 3), 8);
          const int32_t diag = hdiag + sc;
          const int32_t fo = hcur - o, fx = fup - e;
          const int32_t fij = fo > fx ? fo : fx;
          const int32_t eo = H[k] - o, ex = E[k] - e;
          const int32_t eij = eo > ex ? eo : ex;
          int32_t h = diag > eij ? diag : eij;
          h = h > fij ? h : fij;
          // row k: nibble 7 - k % 8 of dword k / 8 (the first row on top)
          dw[k >> 3] = push_code(dw[k >> 3], diag, h, eij, fij, eo, ex, fo, fx);
          hdiag = H[k];
          H[k] = h;
          E[k] = eij;
          hcur = h;
          fup = fij;
        }
        hup_prev = hup;
        hout = H[RL - 1];
        fout = fup;
        sym = symn;
#pragma unroll
        for (int k = 0; k < RL / 4; ++k) X[k] = Xn[k];
        if constexpr (RL == 16) reinterpret_cast<uint2 *>(dstrip)[t * 64 + lane] = make_uint2(dw[0], dw[1]);
        else if constexpr (RL == 8) reinterpret_cast<uint32_t *>(dstrip)[t * 64 + lane] = dw[0];
        else reinterpret_cast<uint16_t *>(dstrip)[t * 64 + lane] = (uint16_t)dw[0];
        if (hand_over && gather) {
          const int jj = (tm + 1) & 63;   // (t - 63) mod 64
          const int32_t vh = __builtin_amdgcn_readlane(hout, 63);
          const int32_t vf = __builtin_amdgcn_readlane(fout, 63);
          obH = (lane == jj) ? vh : obH;
          obF = (lane == jj) ? vf : obF;
        }
      };
      // columns [cb, cb + jj] are complete: store and publish them
      auto hand = [&](int64_t cb, int jj) {
        if (lane <= jj) { outH[cb + lane] = obH; outF[cb + lane] = obF; }
        publish((int32_t)(cb + jj + 1 - clo), false);
      };
      const bool later = t0 >= 64;
      const int tn = (int)(nsteps - t0 < 64 ? nsteps - t0 : 64);
      const int ta = tn < 62 ? tn : 62;
#pragma unroll 1
      for (int tm = 0; tm < ta; ++tm) step(tm, symbuf, tm + 1, later);
      if (tn > 62) {
        step(62, symbuf, 63, later);
        if (hand_over && later) hand(clo + t0 - 64, 63);
      }
      if (tn > 63) step(63, symnext, 0, true);
      if (hand_over && t0 + tn == nsteps) {   // the strip's last step
        const int64_t t = nsteps - 1;
        const int jj = (int)((t - 63) & 63);
        if (t >= 63 && jj != 63) hand(clo + (t - 63) - jj, jj);
      }
    }
    publish((int32_t)(chi - clo), true);
  }
  if (spin_fail && lane == 0) a.err[p] = 1;   // reported as an internal failure
  if constexpr (!SPREAD) {
    // the walk reads every wave's codes: the barrier makes the workgroup's
    // stores visible to it (they pass through this compute unit's caches)
    __syncthreads();
    if (wave == 0) tb_wave_walk<RL>(a, jb, dir, s_tile, lane);
  }
}

// The walk of spread pairs, one wave per pair, after their fill kernel.
template <int RL>
__global__ __launch_bounds__(64) void k_tb_walk(TbArgs a, const TbWaveJob *jobs, uint8_t *dirw) {
  __shared__ uint4 s_tile[kTbTileBytes / 16];
  const TbWaveJob jb = jobs[blockIdx.x];
  if (jb.m <= 0) return;
  tb_wave_walk<RL>(a, jb, dirw + jb.dir_off, s_tile, (int)(threadIdx.x & 63));
}

template <int RL>
__device__ void tb_wave_walk(const TbArgs &a, const TbWaveJob &jb, const uint8_t *dir,
                             uint4 *s_tile, int lane) {
  constexpr int64_t SH = 64 * RL;
  constexpr int WB = RL / 2;
  constexpr int TS = kTbTileBytes / (64 * WB);
  const int64_t p = jb.pair, m = jb.m, w = jb.w;
  const int32_t o = a.o, e = a.e;
  const int64_t nstrips = (m + SH - 1) / SH;
  auto strip_base = [&](int64_t s) {
    int64_t off = 0;
    for (int64_t k = 0; k < s; ++k) {
      int64_t lo, hi;
      tbw_window(k, SH, jb.dlo, jb.bw, w, &lo, &hi);
      off += ((hi - lo) + 63) * 64 * WB;
    }
    return off;
  };

  // ---- walk back from (m, w) in state H (rule T3), uniform on the wave ------
  // Each iteration places the walk in a strip and a tile of its codes and
  // follows one run of the path (below).
  uint32_t *out = a.cig + a.cig_off[p];
  int32_t nruns = 0;
  int64_t i = m, j = w;
  int state = 0;
  uint32_t cur_op = 0xFF, cur_len = 0;
  int64_t guard = 2 * (m + w) + 4;
  int64_t ws = nstrips;          // strip whose codes start at wbase
  int64_t wbase = strip_base(nstrips), wclo = 0, wchi = 0;
  int64_t tile_s = -1, tile_lo = 0, tile_hi = -1;
  const uint8_t *tile = reinterpret_cast<const uint8_t *>(s_tile);
  bool bad = false;
  auto emit_run = [&](uint32_t op, uint32_t len) {
    if (op == cur_op) {
      cur_len += len;
    } else {
      if (cur_len && lane == 0) out[nruns] = (cur_len << 4) | cur_op;
      if (cur_len) ++nruns;
      cur_op = op;
      cur_len = len;
    }
  };
  while ((i > 0 || j > 0) && guard > 0) {
    if (i == 0) {   // row 0: reached from the left by one deletion run
      const uint32_t c = row0_code(j, o, e);
      --guard;
      if (state == 0) {
        state = code_src(c) == 1 ? 1 : 2;
      } else if (state == 1) {
        emit_run(2u, 1u);
        state = (c & kCodeEExt) ? 1 : 0;
        --j;
      } else {
        bad = true;   // no cell above row 0
        break;
      }
      continue;
    }
    const int64_t s = (i - 1) / SH;
    while (ws > s) {   // step the strip cursor up (the walk only moves up)
      --ws;
      tbw_window(ws, SH, jb.dlo, jb.bw, w, &wclo, &wchi);
      wbase -= ((wchi - wclo) + 63) * 64 * WB;
    }
    if (j < wclo || j >= wchi) { bad = true; break; }
    const int64_t x = (i - 1) - s * SH;
    int L = (int)(x / RL), rr = (int)(x % RL);
    const int64_t t = (j - wclo) + L;
    if (s != tile_s || t < tile_lo || t > tile_hi) {
      tile_s = s;
      tile_hi = t;
      tile_lo = t >= TS - 1 ? t - (TS - 1) : 0;
      // steps [tile_lo, tile_hi] are contiguous: 16 bytes per lane and load
      const uint4 *src = reinterpret_cast<const uint4 *>(dir + wbase + tile_lo * 64 * WB);
      const int nv = (int)((tile_hi - tile_lo + 1) * 64 * WB / 16);
      __builtin_amdgcn_wave_barrier();
      for (int v = lane; v < nv; v += 64) s_tile[v] = src[v];
      __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_wave_barrier();
    }
    // One run per iteration, on the whole wave: lane k reads the code of the
    // k-th cell along the run's direction (diagonal for M, left for D, up for
    // I; invalid past the strip's top, the window's left edge or the tile),
    // and a ballot finds where the run ends.  In state H the diagonal run
    // continues while a cell's code names the diagonal; a cell that names E
    // or F takes that gap step at once (same code); a gap run continues while
    // a cell's code extends the gap, the cell that does not still taking its
    // step.  A run cut short by an unreadable cell resumes in the next
    // iteration, after the strip cursor and the tile have moved.
    const int jw = (int)(j - wclo);    // the current column in the window
    const int xi = (int)x;             // the current row in the strip
    const int tlo = (int)tile_lo;
    auto lane_code = [&](int drow, int dcol, bool &valid) -> uint32_t {
      const int xr = xi - lane * drow, jc = jw - lane * dcol;
      const int xq = xr < 0 ? 0 : xr;
      const int Lk = xq / RL, rk = xq % RL;
      const int tk = jc + Lk - tlo;
      valid = xr >= 0 && jc >= 0 && tk >= 0;
      const uint8_t *wp = tile + (((valid ? tk : 0) * 64 + Lk) * WB);
      if constexpr (RL == 4) {
        return ((uint32_t)*reinterpret_cast<const uint16_t *>(wp) >> (4 * (3 - rk))) & 0xFu;
      } else {
        const uint32_t dv = reinterpret_cast<const uint32_t *>(wp)[rk >> 3];
        return (dv >> (4 * (7 - (rk & 7)))) & 0xFu;
      }
    };
    auto first_false = [](bool pred) -> int {
      const unsigned long long bm = __ballot(pred);
      return bm == ~0ull ? 64 : __builtin_ctzll(~bm);
    };
    if (state == 0) {
      bool v;
      const uint32_t ck = lane_code(1, 1, v);
      const int K = first_false(v && (ck & kCodeNotM) == 0 && j - lane > 0);
      if (K > 0) {
        emit_run(0u, (uint32_t)K);
        i -= K;
        j -= K;
        guard -= K;
        continue;
      }
      // the current cell (lane 0, always readable here) leaves the diagonal:
      // its code names E or F (at column 0 the path can only go up)
      const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)ck);
      const uint32_t src = code_src(c0);
      state = src == 0 ? 2 : (int)src;
    }
    const bool left = state == 1;
    bool v;
    const uint32_t ck = left ? lane_code(0, 1, v) : lane_code(1, 0, v);
    const bool ext = v && (ck & (left ? kCodeEExt : kCodeFExt)) != 0 && (!left || j - lane > 0);
    const int stop = first_false(ext);
    // the cell that ends the run takes its step too, when it was readable
    const bool ends = stop < 64 && ((__ballot(v) >> stop) & 1ull);
    const int moves = ends ? stop + 1 : stop;
    if (moves == 0) { bad = true; break; }
    if (ends) state = 0;
    emit_run(left ? 2u : 1u, (uint32_t)moves);
    if (left) j -= moves;
    else i -= moves;
    guard -= moves;
  }
  if (lane != 0) return;
  if (bad || i != 0 || j != 0) a.err[p] = 1;
  if (cur_len) out[nruns++] = (cur_len << 4) | cur_op;
  for (int32_t x = 0, y = nruns - 1; x < y; ++x, --y) {
    const uint32_t t = out[x]; out[x] = out[y]; out[y] = t;
  }
  a.cig_len[p] = nruns;
}

int tb_wave_waves(int64_t m, int n, int RL) {
  const int64_t nstrips = (m + 64 * RL - 1) / (64 * RL);
  const int64_t per = (int64_t)(n + 1) * 64 * RL;
  const int64_t stat = kTbTileBytes + 32 * 32 + kTbMaxStrips * 8;
  const int64_t room = (65536 - stat) / per;
  int64_t wv = std::min<int64_t>(std::min<int64_t>(nstrips, kTbMaxWaves), room);
  return (int)(wv < 1 ? 1 : wv);
}

int tb_wave_max_strips() { return kTbMaxStrips; }

template <int RL>
static void launch_tb_wave(const TbArgs &a, const TbWaveJob *jobs, int64_t njobs, int waves,
                           int segs, IntraSync *sync, uint8_t *dirw, int32_t *bnd, hipStream_t st) {
  const size_t lds = (size_t)(a.n + 1) * 64 * RL * waves;
  if (segs > 1) {
    const dim3 g((unsigned)(8 * segs * ((njobs + 7) / 8)));
    hipLaunchKernelGGL((k_tb_wave<RL, true>), g, dim3(64 * waves), lds, st, a, jobs, njobs, segs,
                       sync, dirw, bnd);
    hipLaunchKernelGGL(k_tb_walk<RL>, dim3((unsigned)njobs), dim3(64), 0, st, a, jobs, dirw);
  } else {
    hipLaunchKernelGGL((k_tb_wave<RL, false>), dim3((unsigned)njobs), dim3(64 * waves), lds, st, a,
                       jobs, njobs, 1, sync, dirw, bnd);
  }
}

hipError_t tb_wave(const TbArgs &a, const TbWaveJob *jobs, int64_t njobs, int RL, int waves,
                   int segs, IntraSync *sync, uint8_t *dirw, int32_t *bnd, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  if (waves < 1 || waves > kTbMaxWaves || segs < 1 || (segs > 1 && !sync))
    return hipErrorInvalidValue;
  if (segs > 1) {
    const hipError_t e = intra_sync_init(sync, njobs, st);
    if (e != hipSuccess) return e;
  }
  switch (RL) {
    case 4: launch_tb_wave<4>(a, jobs, njobs, waves, segs, sync, dirw, bnd, st); break;
    case 8: launch_tb_wave<8>(a, jobs, njobs, waves, segs, sync, dirw, bnd, st); break;
    case 16: launch_tb_wave<16>(a, jobs, njobs, waves, segs, sync, dirw, bnd, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The wave job of pair 0 of a one-pair graph, planned on the device: the
// rectangle and safe band of its alignment, codes and hand-over rows at the
// start of their buffers (m = 0: no alignment, nothing to trace), and its
// CIGAR scratch at offset 0.
__global__ void k_tb_wave_job1(TbArgs a, TbWaveJob *job, int64_t *cig_off) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  TbWaveJob jb{};
  jb.pair = 0;
  if (a.score[0] > 0) {
    if (tb_coords_ok(a, 0)) {
      jb.m = a.qend[0] - a.qbeg[0] + 1;
      jb.w = a.rend[0] - a.rbeg[0] + 1;
      safe_band(jb.m, jb.w, a.score[0], a.smax, a.o, a.e, &jb.dlo, &jb.bw);
    } else {
      a.err[0] = 1;
    }
  }
  *job = jb;
  cig_off[0] = 0;
}

hipError_t tb_wave_job1(const TbArgs &a, TbWaveJob *job, int64_t *cig_off, hipStream_t st) {
  hipLaunchKernelGGL(k_tb_wave_job1, dim3(1), dim3(64), 0, st, a, job, cig_off);
  return hipGetLastError();
}

int64_t tb_wave_dir_bytes(int64_t m, int64_t w, int RL) {
  const int64_t SH = 64 * RL, nstrips = (m + SH - 1) / SH;
  return nstrips * (w + 1 + 63) * 64 * (RL / 2);
}

hipError_t tbw_tasks(int64_t n0, int64_t n1, const int64_t *sorted, const TbArgs &a,
                     TbwTask *tasks, int64_t *dir_words, int64_t *bnd_words, hipStream_t st) {
  const int64_t nt = (n1 - n0 + kTbwSlots - 1) / kTbwSlots;
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tbw_tasks, dim3(nblk(nt, 4)), dim3(256), 0, st, n0, n1,
                     (const int64_t *)nullptr, (int64_t)0, sorted, a, tasks, dir_words, bnd_words);
  return hipGetLastError();
}

hipError_t tbw_tasks_range(const int64_t *range, int64_t ntasks_cap, const int64_t *sorted,
                           const TbArgs &a, TbwTask *tasks, int64_t *dir_words, int64_t *bnd_words,
                           hipStream_t st) {
  if (ntasks_cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tbw_tasks, dim3(nblk(ntasks_cap, 4)), dim3(256), 0, st, (int64_t)0,
                     (int64_t)0, range, ntasks_cap, sorted, a, tasks, dir_words, bnd_words);
  return hipGetLastError();
}

hipError_t tbw_offsets(int64_t ntasks, TbwTask *tasks, const int64_t *doff, const int64_t *boff,
                       hipStream_t st) {
  if (!ntasks) return hipSuccess;
  hipLaunchKernelGGL(k_tbw_offsets, dim3(nblk(ntasks, 128)), dim3(128), 0, st, ntasks, tasks, doff,
                     boff);
  return hipGetLastError();
}

hipError_t tb_strip(const TbArgs &a, const TbwTask *tasks, int64_t ntasks, const int64_t *sorted,
                    int32_t *bndbuf, hipStream_t st) {
  if (!ntasks) return hipSuccess;
  const unsigned blocks = nblk(ntasks, 4);
  if (a.n <= 4)
    hipLaunchKernelGGL((k_tb_strip<true>), dim3(blocks), dim3(256), 0, st, a, tasks, ntasks, sorted, bndbuf);
  else
    hipLaunchKernelGGL((k_tb_strip<false>), dim3(blocks), dim3(256), 0, st, a, tasks, ntasks, sorted, bndbuf);
  return hipGetLastError();
}

}  // namespace swx
