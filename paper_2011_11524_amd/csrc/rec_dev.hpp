// Device building blocks of the answer recovery (Section 8.2), shared by
// the recovery kernels (carry.hip) and the whole-product kernel
// (small.hip): the recovery constants, the CRT digits, the carry maps and
// their workgroup scan.
#pragma once
#include "ntt_dev.hpp"

namespace dmi {

typedef unsigned __int128 u128;

// Constants of the answer recovery.  Per digit-group size k (13..18):
// B = 10^k, the normalised divisor d = B << sh with its reciprocal
// v = floor((2^128 - 1) / d) - 2^64, and kinv = ceil(2^22 / k)
// (d0 / k = (d0 * kinv) >> 22 for d0 < 2^17).
struct RecTable {
  Prime P2;
  uint64_t p1;
  uint64_t r_tilde;
  uint64_t B[6], d[6], v[6];
  uint32_t sh[6], kinv[6];
  uint64_t Ph[6], Pl[6];      // p1 = Ph*B + Pl
  uint64_t bmag[6];           // floor(x / B) = umulhi(x >> k, bmag) >> bsh  (x < 2^64)
  uint32_t bsh[6];
  double inv_B[6];            // 1/B rounded to double
};

// What one product's recovery needs, taken from the table by its k.
struct RecConsts {
  Prime P2;
  uint64_t p1;
  uint64_t r_tilde;
  uint64_t B;
  uint64_t d;
  uint64_t v;
  int sh;
  int k;
  uint64_t Ph, Pl, bmag;
  uint32_t bsh;
  double inv_B;
  uint32_t kinv;
  uint32_t nblk;
  uint64_t NP;         // n + m coefficient positions
  uint64_t nout;       // output limbs (na + nb)
};

__device__ __forceinline__ RecConsts rec_consts(const RecTable& t, const ProdDesc& d) {
  RecConsts rc;
  const int i = d.pl.k - kMinK;
  rc.P2 = t.P2;
  rc.p1 = t.p1;
  rc.r_tilde = t.r_tilde;
  rc.B = t.B[i];
  rc.d = t.d[i];
  rc.v = t.v[i];
  rc.sh = (int)t.sh[i];
  rc.kinv = t.kinv[i];
  rc.Ph = t.Ph[i];
  rc.Pl = t.Pl[i];
  rc.bmag = t.bmag[i];
  rc.bsh = t.bsh[i];
  rc.inv_B = t.inv_B[i];
  rc.k = d.pl.k;
  rc.nblk = d.nblk;
  rc.NP = d.pl.n + d.pl.m;
  rc.nout = d.pl.na + d.pl.nb;
  return rc;
}

// 64x64 -> 128-bit product from four v_mad_u64_u32.
__device__ __forceinline__ void mul_wide(uint64_t x, uint64_t y, uint64_t& lo, uint64_t& hi) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint64_t t0 = mad_u64_u32(x0, y0, 0);
  const uint64_t t1 = mad_u64_u32(x0, y1, t0 >> 32);
  const uint64_t t2 = mad_u64_u32(x1, y0, (uint32_t)t1);
  hi = mad_u64_u32(x1, y1, (t1 >> 32) + (t2 >> 32));
  lo = (t2 << 32) | (uint32_t)t0;
}

// (u1:u0) / d for normalised d and u1 < d: quotient q < 2^64, remainder r.
__device__ __forceinline__ void div_2by1(uint64_t u1, uint64_t u0, uint64_t d, uint64_t v,
                                         uint64_t& q, uint64_t& r) {
  uint64_t q0, q1;
  mul_wide(v, u1, q0, q1);
  q0 += u0;
  q1 += u1 + (q0 < u0 ? 1 : 0) + 1;
  uint64_t rr = u0 - q1 * d;
  if (rr > q0) { q1 -= 1; rr += d; }
  if (rr >= d) { q1 += 1; rr -= d; }
  q = q1;
  r = rr;
}

// x = q*B + r for a 64-bit x (multiply-high by the reciprocal of 10^k).
__device__ __forceinline__ uint64_t divmod_B64(uint64_t x, const RecConsts& rc, uint64_t& r) {
  const uint64_t q = __umul64hi(x >> rc.k, rc.bmag) >> rc.bsh;
  r = x - q * rc.B;
  return q;
}

// Base-B digits (q0, q1, q2) of coefficient c_i from its two residues.  The
// CRT gives c = a1 + p1*phi (Section 8.2.2).  With p1 = Ph*B + Pl,
// phi = fh*B + fl and a1 = ah*B + al (all digits < B):
//   c = (al + Pl*fl) + B*(ah + Ph*fl + Pl*fh) + B^2*(Ph*fh)
// so one 128-by-64 division (of Pl*fl < B^2) and one quotient of a 65-bit
// value (by a double-precision estimate, corrected exactly) give the digits.
__device__ __forceinline__ void crt_digits(uint64_t a1, uint64_t a2, const RecConsts& rc,
                                           uint64_t& q0, uint64_t& q1, uint64_t& q2) {
  const uint64_t psi = sub_mod(a2, a1, rc.P2);              // a1 < p1 < p2
  const uint64_t phi = mont_mul(psi, rc.r_tilde, rc.P2);    // r * (a2 - a1) mod p2
  uint64_t fl, al;
  const uint64_t fh = divmod_B64(phi, rc, fl);
  const uint64_t ah = divmod_B64(a1, rc, al);
  // Pl*fl = th*B + tl
  uint64_t lo, hi;
  mul_wide(rc.Pl, fl, lo, hi);
  const int sh = rc.sh;                                     // 4 <= sh <= 20
  uint64_t th, tr;
  div_2by1((hi << sh) | (lo >> (64 - sh)), lo << sh, rc.d, rc.v, th, tr);
  uint64_t s0 = al + (tr >> sh);                            // < 2B
  const uint64_t c0 = s0 >= rc.B ? 1 : 0;
  s0 -= c0 * rc.B;
  q0 = s0;
  // mid = ah + Ph*fl + Pl*fh + th + c0 < 2^65, as (mh:ml)
  const uint64_t x = rc.Ph * fl, y = rc.Pl * fh;            // each < 2^63
  uint64_t ml = x + y;
  uint64_t mh = ml < x ? 1 : 0;
  const uint64_t z = th + ah + c0;                          // < 2^61
  ml += z;
  mh += ml < z ? 1 : 0;
  // q = floor(mid / B) from a double estimate (error well below 1), then exact
  const double md = (double)mh * 18446744073709551616.0 + (double)ml;
  uint64_t q = (uint64_t)floor(md * rc.inv_B);
  int64_t r = (int64_t)(ml - q * rc.B);                     // mid - q*B, in (-B, 2B)
  if (r < 0) { q -= 1; r += (int64_t)rc.B; }
  else if (r >= (int64_t)rc.B) { q += 1; r -= (int64_t)rc.B; }
  q1 = (uint64_t)r;
  q2 = rc.Ph * fh + q;
}

// Carry maps {0,1,2} -> {0,1,2}, one byte per argument: byte c holds f(c)
// for c < 3, and byte 3 holds 3.  Composition is then a byte permute:
// (later o earlier) has as byte c the byte of `later` that earlier(c)
// selects, one v_perm_b32 with `earlier` as the selector (byte 3 selects
// byte 3, which stays 3).
constexpr uint32_t kIdentityMap = 0x03020100u;

__device__ __forceinline__ uint32_t carry_map(uint64_t s, uint64_t B) {
  uint32_t m = 0x03000000u;
#pragma unroll
  for (uint32_t c = 0; c < 3; ++c) {
    const uint64_t t = s + c;
    const uint32_t o = t >= 2 * B ? 2u : (t >= B ? 1u : 0u);
    m |= o << (8 * c);
  }
  return m;
}
__device__ __forceinline__ uint32_t apply_map(uint32_t f, uint32_t c) { return (f >> (8 * c)) & 0xffu; }
// (later o earlier)(c) = later(earlier(c))
__device__ __forceinline__ uint32_t compose(uint32_t later, uint32_t earlier) {
  return __builtin_amdgcn_perm(later, later, earlier);
}

// Exclusive scan of the per-thread maps of one workgroup (thread order =
// position order).  Returns the map of everything before this thread;
// *total receives the map of the whole workgroup.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t f, uint32_t* total) {
  __shared__ uint32_t wave_tot[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  uint32_t inc = f;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc = compose(inc, o);
  }
  uint32_t exc = __shfl_up(inc, 1, 64);
  if (lane == 0) exc = kIdentityMap;
  // the last active lane of each wavefront holds the wavefront's map
  const int last = (wid == nw - 1) ? ((blockDim.x - 1) & 63) : 63;
  if (lane == last) wave_tot[wid] = inc;
  __syncthreads();
  uint32_t before = kIdentityMap;
  for (int w = 0; w < wid; ++w) before = compose(wave_tot[w], before);
  uint32_t all = kIdentityMap;
  for (int w = 0; w < nw; ++w) all = compose(wave_tot[w], all);
  *total = all;
  return compose(exc, before);
}

__device__ __forceinline__ uint64_t div_p10(uint64_t x, int e, const DivTable* __restrict__ dt) {
  if (e == 0) return x;
  return __umul64hi(x >> e, dt->mag[e]) >> dt->sh[e];
}

// The recovery table of every digit-group size (host; carry.hip).
RecTable make_rec_table(const Consts& cs, const DivTable* dt_host);

}  // namespace dmi
