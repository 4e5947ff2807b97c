// Arithmetic in F_p for the two word-sized primes of the method, on the
// 32-bit VALU of gfx950.
//
// Both primes have the form p = p_hi * 2^32 + 1 (they are c*3*2^n + 1 with
// n >= 32, Section 4.5), and p < 2^63 = mu/2 with mu = 2^64 (eq. pi_bound).
//
// Multiplication is Montgomery's REDC(x, y) = x*y*R^-1 mod p with R = 2^64
// (Section 4.4.3).  Because p == 1 (mod 2^32), -p^-1 == -1 (mod 2^32) and the
// reduction by 2^64 runs as two 32-bit word-serial rounds, each
//     m = -t mod 2^32;   t = (t + m*p) / 2^32
// costing one 32x32->64 multiply by p_hi: there is no multiply by p'.
// The full product takes four v_mad_u64_u32; the reduction two more.
//
// REDC accepts one operand "unadjusted" in [0, 2p) and the other in [0, p):
// then x*y < 2p^2 < mu*p, the input range of MontgomeryReduce (Section 8.3).
// Every result leaves here canonical in [0, p).
//
// Additions and subtractions are branch-free selects (Section 8.1): the
// compiler emits v_cndmask, never a branch.
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

// REDC(x, y) = x*y*2^-64 mod p, for x < 2p, y < p.  Result in [0, p).
__device__ __forceinline__ uint64_t mont_mul(uint64_t x, uint64_t y, const Prime& P) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  // 128-bit product T = t3*2^64 + lo(t2)*2^32 + lo(t0)
  const uint64_t t0 = mad_u64_u32(x0, y0, 0);
  const uint64_t t1 = mad_u64_u32(x0, y1, t0 >> 32);
  const uint64_t t2 = mad_u64_u32(x1, y0, (uint32_t)t1);
  const uint64_t t3 = mad_u64_u32(x1, y1, (t1 >> 32) + (t2 >> 32));
  // round 1: m1 = -T0; (T + m1*p)/2^32 = u + t3*2^32, u = m1*p_hi + T1 + [T0 != 0]
  const uint32_t T0 = (uint32_t)t0;
  const uint32_t m1 = 0u - T0;
  const uint64_t u = mad_u64_u32(m1, P.p_hi, (uint64_t)(uint32_t)t2 + (uint64_t)(T0 != 0u));
  const uint64_t V = t3 + (u >> 32);
  // round 2: m2 = -lo(u); result = m2*p_hi + V + [lo(u) != 0]  (< 2p)
  const uint32_t U0 = (uint32_t)u;
  const uint32_t m2 = 0u - U0;
  const uint64_t r = mad_u64_u32(m2, P.p_hi, V + (uint64_t)(U0 != 0u));
  return r >= P.p ? r - P.p : r;
}

// x + y mod p for x, y < p
__device__ __forceinline__ uint64_t add_mod(uint64_t x, uint64_t y, const Prime& P) {
  const uint64_t s = x + y;
  return s >= P.p ? s - P.p : s;
}

// x - y mod p for x, y < p
__device__ __forceinline__ uint64_t sub_mod(uint64_t x, uint64_t y, const Prime& P) {
  const uint64_t d = x - y;
  return x >= y ? d : d + P.p;
}

// x - y + p in [1, 2p): the unadjusted difference, a valid REDC operand.
__device__ __forceinline__ uint64_t sub_lazy(uint64_t x, uint64_t y, const Prime& P) {
  return x + (P.p - y);
}

}  // namespace dmi
