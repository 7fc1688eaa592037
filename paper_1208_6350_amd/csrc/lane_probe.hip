// lane_probe.hip -- measured cell rate of the fill recurrence at 8-bit and
// 16-bit lane widths (the method section's narrow saturating lanes).
//
// gfx950 has packed 16-bit integer instructions (two lanes per register) but
// no packed 8-bit add, subtract or max.  Four 8-bit lanes per register need
// SWAR arithmetic: the bytes are added or subtracted with the top bit of each
// byte kept out of the carry chain, the carries and borrows recovered from
// the operands' top bits, and saturation applied from the carry or borrow
// mask.  This probe runs the same biased recurrence (H, E, F, the zero floor
// and the column max) over synthetic pairs at both widths and reports the
// cells per second of each, so that the choice of lane width rests on a
// measurement.  Both widths compute the same pairs; the host checks that their
// best scores agree.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "lanes.h"
#include "swx_kernels.h"

namespace swx {

namespace {

constexpr int kProbeRows = 16;
constexpr uint32_t kTop = 0x80808080u, kLow = 0x7F7F7F7Fu;

// a + b per byte, saturating at 255
__device__ __forceinline__ uint32_t u8_adds(uint32_t a, uint32_t b) {
  uint32_t s = (a & kLow) + (b & kLow);
  const uint32_t x = (a ^ b) & kTop;
  const uint32_t ov = ((a & b) | (x & s)) & kTop;   // carry out of each byte
  s ^= x;
  return s | ((ov >> 7) * 0xFFu);
}

// max(a - b, 0) per byte
__device__ __forceinline__ uint32_t u8_subs(uint32_t a, uint32_t b) {
  const uint32_t d = ((a | kTop) - (b & kLow)) ^ ((a ^ ~b) & kTop);
  const uint32_t bo = ((~a & b) | (~(a ^ b) & d)) & kTop;   // borrow out of each byte
  return d & ~((bo >> 7) * 0xFFu);
}

// max(a, b) per byte: b + max(a - b, 0) never leaves its byte
__device__ __forceinline__ uint32_t u8_max(uint32_t a, uint32_t b) { return b + u8_subs(a, b); }

__device__ __forceinline__ uint32_t mix(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// biased scores (match +2, mismatch -2, bias 2) of query symbols 0..3 against
// reference symbol b, one byte each
__device__ __forceinline__ uint32_t lut_word(uint32_t b) {
  uint32_t w = 0;
  for (uint32_t q = 0; q < 4; ++q) w |= (q == b ? 4u : 0u) << (8 * q);
  return w;
}

// One thread runs PL pairs (PL = 4 at 8 bits, 2 at 16 bits) of kProbeRows
// query rows against `cols` columns; pair p's query symbol of row r is
// mix(p * 16 + r) & 3, column c's reference symbol mix(c + 0x9E37) & 3.
// Writes each pair's best H.
template <int BITS>
__global__ __launch_bounds__(256) void k_lane_probe(int64_t cols, int32_t o, int32_t e,
                                                    uint32_t *best) {
  constexpr int PL = 32 / BITS;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t sel[kProbeRows];
#pragma unroll
  for (int r = 0; r < kProbeRows; ++r) {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const uint32_t q = mix((uint32_t)((t * PL + k) * kProbeRows + r)) & 3u;
      if (BITS == 8) w |= q << (8 * k);
      else w |= (q | (0x0Cu << 8)) << (16 * k);   // byte q, then a zero byte
    }
    sel[r] = w;
  }
  uint32_t H[kProbeRows], E[kProbeRows];
#pragma unroll
  for (int r = 0; r < kProbeRows; ++r) { H[r] = 0; E[r] = 0; }
  uint32_t cmax = 0;
  const uint32_t rep = BITS == 8 ? 0x01010101u : 0x00010001u;
  const uint32_t vb = 2u * rep, vo = (uint32_t)o * rep, ve = (uint32_t)e * rep;
  for (int64_t c = 0; c < cols; ++c) {
    const uint32_t X = lut_word(mix((uint32_t)c + 0x9E37u) & 3u);
    uint32_t hd = 0, F = 0, cm = 0;
#pragma unroll
    for (int r = 0; r < kProbeRows; ++r) {
      const uint32_t sc = perm(0u, X, sel[r]);
      uint32_t hb, hn, ho;
      if constexpr (BITS == 8) {
        const uint32_t u = u8_max(u8_adds(hd, sc), E[r]);
        hb = u8_max(u, F);
        hn = u8_subs(hb, vb);
        cm = u8_max(cm, hn);
        ho = u8_subs(hb, vo);
        E[r] = u8_max(u8_subs(E[r], ve), ho);
        F = u8_max(u8_subs(F, ve), ho);
      } else {
        using T = VT<u16x2>;
        const u16x2 u = T::max(T::add(T::from(hd), T::from(sc)), T::from(E[r]));
        const u16x2 hbv = T::max(u, T::from(F));
        const u16x2 hnv = T::subs(hbv, T::from(vb));
        cm = T::bits(T::max(T::from(cm), hnv));
        const u16x2 hov = T::subs(hbv, T::from(vo));
        E[r] = T::bits(T::max(T::subs(T::from(E[r]), T::from(ve)), hov));
        F = T::bits(T::max(T::subs(T::from(F), T::from(ve)), hov));
        hb = T::bits(hbv);
        hn = T::bits(hnv);
        ho = T::bits(hov);
      }
      (void)hb;
      (void)ho;
      hd = H[r];
      H[r] = hn;
    }
    cmax = BITS == 8 ? u8_max(cmax, cm) : VT<u16x2>::bits(VT<u16x2>::max(VT<u16x2>::from(cmax),
                                                                         VT<u16x2>::from(cm)));
  }
#pragma unroll
  for (int k = 0; k < PL; ++k) best[t * PL + k] = (cmax >> (BITS * k)) & ((1u << BITS) - 1u);
}

// Check of VT<u16x2>::max3 (the batched fill's packed three-way maximum)
// against the unsigned maximum: block a tests every b below lim with c from a
// fixed set, in both halves; the pseudo-random part draws triples from a
// 64-bit mix (splitmix64's finaliser) of the thread index.
__device__ __forceinline__ uint32_t max3_bits(uint32_t a, uint32_t b, uint32_t c) {
  return VT<u16x2>::bits(VT<u16x2>::max3(VT<u16x2>::from(a), VT<u16x2>::from(b), VT<u16x2>::from(c)));
}

__device__ __forceinline__ uint32_t umax2(uint32_t a, uint32_t b) { return a > b ? a : b; }

__device__ __forceinline__ uint64_t half_mismatches(uint32_t r, uint32_t lo_a, uint32_t lo_b,
                                                    uint32_t lo_c, uint32_t hi_a, uint32_t hi_b,
                                                    uint32_t hi_c) {
  return (uint64_t)((r & 0xFFFFu) != umax2(umax2(lo_a, lo_b), lo_c)) +
         (uint64_t)((r >> 16) != umax2(umax2(hi_a, hi_b), hi_c));
}

__global__ __launch_bounds__(256) void k_max3_pairs(uint32_t lim, unsigned long long *bad) {
  const uint32_t a = blockIdx.x;
  if (a >= lim) return;
  const uint32_t cs[8] = {0u, 1u, 0x3FFu, 0x400u, 0x401u, 0x7FFu, 0x123u, lim - 1};
  uint64_t nb = 0;
  for (uint32_t b = threadIdx.x; b < lim; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t c = cs[k];
      nb += half_mismatches(max3_bits(a | (b << 16), b | (c << 16), c | (a << 16)), a, b, c, b, c, a);
    }
  }
  if (nb) atomicAdd(bad, (unsigned long long)nb);
}

__global__ __launch_bounds__(256) void k_max3_random(uint32_t lim, uint64_t n,
                                                     unsigned long long *bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t x = i * 0x9E3779B97F4A7C15ull;
  uint64_t nb = 0;
  for (int it = 0; it < 16; ++it) {
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const uint32_t v0 = (uint32_t)(z % lim), v1 = (uint32_t)((z >> 15) % lim);
    const uint32_t v2 = (uint32_t)((z >> 30) % lim), v3 = (uint32_t)((z >> 45) % lim);
    const uint32_t v4 = (uint32_t)((z >> 7) & 63u), v5 = (uint32_t)((z >> 22) % 1100u);
    nb += half_mismatches(max3_bits(v0 | (v3 << 16), v1 | (v4 << 16), v2 | (v5 << 16)), v0, v1, v2,
                          v3, v4, v5);
  }
  if (nb) atomicAdd(bad, (unsigned long long)nb);
}

}  // namespace

hipError_t max3_check(unsigned long long *bad, uint64_t *checked, hipStream_t st) {
  constexpr uint32_t kLim = 0x7C00u;             // the finite non-negative f16 patterns
  constexpr uint64_t kRandom = uint64_t(1) << 26;   // threads of the random part
  hipLaunchKernelGGL(k_max3_pairs, dim3(kLim), dim3(256), 0, st, kLim, bad);
  hipLaunchKernelGGL(k_max3_random, dim3((unsigned)(kRandom / 256)), dim3(256), 0, st, kLim,
                     kRandom, bad);
  *checked = (uint64_t)kLim * kLim * 16 + kRandom * 32;
  return hipGetLastError();
}

hipError_t lane_probe(int bits, int64_t cols, int64_t blocks, int32_t o, int32_t e,
                      uint32_t *best, hipStream_t st) {
  if (blocks < 1 || cols < 1) return hipErrorInvalidValue;
  if (bits == 8)
    hipLaunchKernelGGL(k_lane_probe<8>, dim3((unsigned)blocks), dim3(256), 0, st, cols, o, e, best);
  else if (bits == 16)
    hipLaunchKernelGGL(k_lane_probe<16>, dim3((unsigned)blocks), dim3(256), 0, st, cols, o, e, best);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace swx
