// lanes.h -- lane arithmetic for the fill kernels.
//
// The fill runs on unsigned saturating integer lanes.  A 32-bit VGPR holds
// either two independent 16-bit lanes (v_pk_* instructions, two cells per
// instruction) or one 32-bit lane.  All operations used by the recurrences are
// here so that the 16- and 32-bit kernels share one body.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swx {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

template <class V> struct VT;

// two 16-bit lanes per register
template <> struct VT<u16x2> {
  static constexpr int kHalves = 2;
  static __device__ __forceinline__ u16x2 from(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
  static __device__ __forceinline__ uint32_t bits(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
  static __device__ __forceinline__ u16x2 splat(uint32_t s) { return from((s & 0xFFFFu) * 0x10001u); }
  static __device__ __forceinline__ u16x2 zero() { return from(0u); }
  static __device__ __forceinline__ u16x2 add(u16x2 a, u16x2 b) { return a + b; }
  static __device__ __forceinline__ u16x2 subs(u16x2 a, u16x2 b) {
    return __builtin_elementwise_sub_sat(a, b);
  }
  static __device__ __forceinline__ u16x2 max(u16x2 a, u16x2 b) {
    return __builtin_elementwise_max(a, b);
  }
  static __device__ __forceinline__ u16x2 min(u16x2 a, u16x2 b) {
    return __builtin_elementwise_min(a, b);
  }
  // Largest of three, in one instruction: the packed f16 three-way maximum.
  // On 16-bit patterns below 0x7C00 (finite non-negative halves; denormals
  // are kept by the kernels' float mode) the f16 order is the unsigned
  // integer order, so this is the exact unsigned maximum there.  Larger
  // patterns read as infinities, NaNs or negatives and give no such
  // guarantee: callers keep every lane value below 0x7C00, or only reach
  // such values in pairs that are already flagged for a 32-bit re-run.
  static __device__ __forceinline__ u16x2 max3(u16x2 a, u16x2 b, u16x2 c) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 x = __builtin_bit_cast(h2, a), y = __builtin_bit_cast(h2, b), z = __builtin_bit_cast(h2, c);
    return __builtin_bit_cast(u16x2, __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
  }
  // value * 32 + code: the row code sits in the low 5 bits so that a max over
  // rows also yields, among rows of equal value, the one with the largest
  // code.  The value must fit the 11-bit field (the fill clamps it first when
  // a score could exceed it)
  static __device__ __forceinline__ u16x2 enc_nosat(u16x2 h, uint32_t code, uint32_t mul32) {
    return h * from(mul32) + (u16x2){(unsigned short)code, (unsigned short)code};
  }
  static __device__ __forceinline__ u16x2 shr5(u16x2 v) { return v >> (u16x2){5, 5}; }
  static __device__ __forceinline__ uint32_t half(u16x2 v, int k) {
    return k ? (bits(v) >> 16) : (bits(v) & 0xFFFFu);
  }
  // byte selectors for v_perm_b32: half 0 from the low source dword, half 1
  // from the high one; byte 0x0C reads as zero.
  static constexpr uint32_t sel_const(int k) {
    return (uint32_t)k | 0x0C00u | ((uint32_t)(k + 4) << 16) | 0x0C000000u;
  }
  static constexpr uint32_t kPadSel = 0x0C0C0C0Cu;
};

// one 32-bit lane per register
template <> struct VT<uint32_t> {
  static constexpr int kHalves = 1;
  static __device__ __forceinline__ uint32_t from(uint32_t x) { return x; }
  static __device__ __forceinline__ uint32_t bits(uint32_t v) { return v; }
  static __device__ __forceinline__ uint32_t splat(uint32_t s) { return s; }
  static __device__ __forceinline__ uint32_t zero() { return 0u; }
  static __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) { return a + b; }
  static __device__ __forceinline__ uint32_t subs(uint32_t a, uint32_t b) {
    return __builtin_elementwise_sub_sat(a, b);
  }
  static __device__ __forceinline__ uint32_t max(uint32_t a, uint32_t b) { return a > b ? a : b; }
  static __device__ __forceinline__ uint32_t min(uint32_t a, uint32_t b) { return a < b ? a : b; }
  static __device__ __forceinline__ uint32_t max3(uint32_t a, uint32_t b, uint32_t c) {
    return max(max(a, b), c);
  }
  static __device__ __forceinline__ uint32_t enc_nosat(uint32_t h, uint32_t code, uint32_t) {
    return h * 32u + code;
  }
  static __device__ __forceinline__ uint32_t shr5(uint32_t v) { return v >> 5; }
  static __device__ __forceinline__ uint32_t half(uint32_t v, int) { return v; }
  static constexpr uint32_t sel_const(int k) { return (uint32_t)k | 0x0C0C0C00u; }
  static constexpr uint32_t kPadSel = 0x0C0C0C0Cu;
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

}  // namespace swx
