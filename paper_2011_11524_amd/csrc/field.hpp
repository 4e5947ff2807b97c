// Arithmetic in F_p for the two word-sized primes of the method, on the
// 32-bit VALU of gfx950.
//
// Both primes have the form p = p_hi * 2^32 + 1 (they are c*3*2^n + 1 with
// n >= 32, Section 4.5), and p < 2^63 = mu/2 with mu = 2^64 (eq. pi_bound).
//
// Multiplication is Montgomery's REDC(x, y) = x*y*R^-1 mod p with R = 2^64
// (Section 4.4.3), in its signed form: with m = T * p^-1 mod 2^64 the
// value (T - m*p) / 2^64 is exact and lies in (-p, p), so one conditional
// +p makes it canonical.  Because p == 1 (mod 2^32), p^-1 == 1 - p_hi*2^32
// (mod 2^64): m needs one 32x32 product (m = (T0, T1 - lo(T0*p_hi))) and
// floor(m*p / 2^64) one more, so the reduction is two v_mad_u64_u32 on top
// of the four of the 64x64->128 product, with no multiply by a p'.
//
// Both operands are below 2^63 (canonical residues are, p < 2^63), so their
// high words are below 2^31 and the two middle partial products plus the
// carry out of the low one stay below 2^64: the product T is four
// v_mad_u64_u32, each adding the previous one's full 64-bit result or its
// high word, with no separate carry chain.  x*y < p*2^64 (Section 8.3)
// keeps the signed REDC value in (-p, p).  Every result leaves here
// canonical in [0, p).

// Additions and subtractions are branch-free (Section 8.1): the borrow of a
// 64-bit subtraction selects the corrected value (v_cndmask).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmi {

struct Prime {
  uint64_t p;      // the modulus
  uint32_t p_hi;   // (p - 1) >> 32
};

__device__ __forceinline__ uint64_t mad_u64_u32(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * (uint64_t)b + c;
}

// REDC(x, y) = x*y*2^-64 mod p, for x, y < 2^63 with x*y < p*2^64 (both
// below p; with p < 2^62 both below 2p).  Result in [0, p).
__device__ __forceinline__ uint64_t mont_mul(uint64_t x, uint64_t y, const Prime& P) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  // T = x*y = Thi*2^64 + T1*2^32 + T0: x0*y1 + x1*y0 + hi(x0*y0) < 2^64
  // because x1, y1 < 2^31
  const uint64_t t0 = mad_u64_u32(x0, y0, 0);
  const uint64_t mid = mad_u64_u32(x1, y0, mad_u64_u32(x0, y1, t0 >> 32));
  const uint64_t th = mad_u64_u32(x1, y1, mid >> 32);
  const uint32_t T0 = (uint32_t)t0, T1 = (uint32_t)mid;
  // m = (T0, T1 - lo(T0*p_hi));  floor(m*p / 2^64) = m1*p_hi + hi(T0*p_hi) + borrow
  const uint64_t h = mad_u64_u32(T0, P.p_hi, 0);
  unsigned bw;
  const uint32_t m1 = __builtin_subc(T1, (uint32_t)h, 0u, &bw);
  const uint64_t mp = mad_u64_u32(m1, P.p_hi, h >> 32);
  // r = Thi - floor(m*p / 2^64), in (-p, p): the borrow enters the subtraction
  unsigned b1, b2;
  const uint32_t r_lo = __builtin_subc((uint32_t)th, (uint32_t)mp, bw, &b1);
  const uint32_t r_hi = __builtin_subc((uint32_t)(th >> 32), (uint32_t)(mp >> 32), b1, &b2);
  const uint64_t r = ((uint64_t)r_hi << 32) | r_lo;
  return b2 ? r + P.p : r;
}

// x + y mod p for x, y < p
__device__ __forceinline__ uint64_t add_mod(uint64_t x, uint64_t y, const Prime& P) {
  const uint64_t s = x + y;
  unsigned b1, b2;
  const uint32_t d_lo = __builtin_subc((uint32_t)s, (uint32_t)P.p, 0u, &b1);
  const uint32_t d_hi = __builtin_subc((uint32_t)(s >> 32), (uint32_t)(P.p >> 32), b1, &b2);
  return b2 ? s : (((uint64_t)d_hi << 32) | d_lo);
}

// x - y mod p for x, y < p
__device__ __forceinline__ uint64_t sub_mod(uint64_t x, uint64_t y, const Prime& P) {
  unsigned b1, b2;
  const uint32_t d_lo = __builtin_subc((uint32_t)x, (uint32_t)y, 0u, &b1);
  const uint32_t d_hi = __builtin_subc((uint32_t)(x >> 32), (uint32_t)(y >> 32), b1, &b2);
  const uint64_t d = ((uint64_t)d_hi << 32) | d_lo;
  return b2 ? d + P.p : d;
}

// ---------------------------------------------------------------------------
// Redundant ranges (Sections 8.3, 9), for primes p < 2^62 = mu/4 only: then
// 4p < 2^64, and REDC(x, y) with x < 4p, y < p has x*y < 4p^2 < mu*p, so the
// signed REDC value lies in (-p, p) and adding p (with no test) leaves it in
// (0, 2p).  Butterfly values then stay below 2p (DIF) or 4p (DIT) and are
// reduced once where they leave a transform.
// ---------------------------------------------------------------------------

// REDC(x, y) + p in (0, 2p), for x < 4p, y < p.  x may reach 2^63 here,
// so the product takes the carry of the middle partial products
// explicitly.
__device__ __forceinline__ uint64_t mont_mul_r(uint64_t x, uint64_t y, const Prime& P) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint64_t t0 = mad_u64_u32(x0, y0, 0);
  const uint64_t t1 = mad_u64_u32(x0, y1, t0 >> 32);
  const uint64_t t2 = mad_u64_u32(x1, y0, (uint32_t)t1);
  const uint64_t t3 = mad_u64_u32(x1, y1, t1 >> 32);
  unsigned c, c2;
  const uint32_t th_lo = __builtin_addc((uint32_t)t3, (uint32_t)(t2 >> 32), 0u, &c);
  const uint32_t th_hi = __builtin_addc((uint32_t)(t3 >> 32), 0u, c, &c2);
  const uint32_t T0 = (uint32_t)t0, T1 = (uint32_t)t2;
  const uint64_t h = mad_u64_u32(T0, P.p_hi, 0);
  unsigned bw, unused;
  const uint32_t m1 = __builtin_subc(T1, (uint32_t)h, 0u, &bw);
  const uint32_t hh = __builtin_addc((uint32_t)(h >> 32), 0u, bw, &unused);
  const uint64_t mp = mad_u64_u32(m1, P.p_hi, (uint64_t)hh);
  const uint64_t th = ((uint64_t)th_hi << 32) | th_lo;
  return th - mp + P.p;    // (th - mp) in (-p, p), as a two's-complement word
}

// x - m if x >= m, else x (one compare and select on the borrow).
__device__ __forceinline__ uint64_t cond_sub(uint64_t x, uint64_t m) {
  unsigned b1, b2;
  const uint32_t d_lo = __builtin_subc((uint32_t)x, (uint32_t)m, 0u, &b1);
  const uint32_t d_hi = __builtin_subc((uint32_t)(x >> 32), (uint32_t)(m >> 32), b1, &b2);
  return b2 ? x : (((uint64_t)d_hi << 32) | d_lo);
}

// [0, 4p) -> [0, p)
__device__ __forceinline__ uint64_t reduce_4p(uint64_t x, const Prime& P) {
  return cond_sub(cond_sub(x, P.p << 1), P.p);
}

// [0, 2p) -> [0, p)
__device__ __forceinline__ uint64_t reduce_2p(uint64_t x, const Prime& P) { return cond_sub(x, P.p); }

}  // namespace dmi
