// Answer recovery (Section 8.2): two-prime CRT, carry propagation and
// regrouping of base-10^k digits into base-10^19 limbs.
//
// CRT (Section 8.2.2): with p1 < p2 and r = p1^-1 mod p2,
//   psi = (a2 - a1) mod p2,  phi = REDC(r~, psi) with r~ = R*r mod p2,
//   c   = a1 + p1 * phi      (exact, c < p1*p2 < 2^126).
// Carry (eq. sigmai_and_zi): instead of a 127-bit running sigma (eq.
// two_word_bound), each coefficient is cut into three base-B digits
// c_i = q2*B^2 + q1*B + q0 (valid for k >= 13 since p1*p2 < 10^39), so
//   Z = sum_i s_i B^i,  s_i = q0_i + q1_(i-1) + q2_(i-2) <= 3(B-1),
// and the carry into every position is 0, 1 or 2.  Position i then acts on
// the incoming carry as a map {0,1,2} -> {0,1,2}; maps compose
// associatively, so the carries come from a parallel scan: within a
// wavefront by shuffles, across wavefronts through LDS, across workgroups
// by a second small kernel over the per-block maps.
//
// The 128-by-64-bit divisions by B use a precomputed reciprocal (Moller and
// Granlund, "Improved division by invariant integers", 2011, the 2-by-1
// division), the division-by-constant idea of Section 8.2.1.
#include "internal.hpp"

namespace dmi {

typedef unsigned __int128 u128;

constexpr int kRecThreads = 256;
constexpr int kRecPT = 8;                          // positions per thread
constexpr int kRecBlock = kRecThreads * kRecPT;    // positions per workgroup

struct RecConsts {
  Prime P2;
  uint64_t p1;
  uint64_t r_tilde;
  uint64_t B;          // 10^k
  uint64_t d;          // B << sh (normalised divisor)
  uint64_t v;          // floor((2^128 - 1) / d) - 2^64
  int sh;
  int k;
  uint64_t NP;         // n + m coefficient positions
  uint64_t nout;       // output limbs (na + nb)
};

// (u1:u0) / d for normalised d and u1 < d.
__device__ __forceinline__ void div_2by1(uint64_t u1, uint64_t u0, uint64_t d, uint64_t v,
                                         uint64_t& q, uint64_t& r) {
  u128 qq = (u128)v * u1;
  qq += ((u128)u1 << 64) | u0;
  uint64_t q1 = (uint64_t)(qq >> 64) + 1;
  const uint64_t q0 = (uint64_t)qq;
  uint64_t rr = u0 - q1 * d;
  if (rr > q0) { q1 -= 1; rr += d; }
  if (rr >= d) { q1 += 1; rr -= d; }
  q = q1;
  r = rr;
}

// x = q*B + r for a 128-bit x; returns r, writes q.
__device__ __forceinline__ uint64_t divmod_B(u128 x, const RecConsts& rc, u128& q) {
  const uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  const int sh = rc.sh;
  const uint64_t u2 = sh ? hi >> (64 - sh) : 0;
  const uint64_t u1 = sh ? (hi << sh) | (lo >> (64 - sh)) : hi;
  const uint64_t u0 = lo << sh;
  uint64_t qh, qlo, r1, r0;
  div_2by1(u2, u1, rc.d, rc.v, qh, r1);
  div_2by1(r1, u0, rc.d, rc.v, qlo, r0);
  q = ((u128)qh << 64) | qlo;
  return r0 >> sh;
}

// The base-B digits (q0, q1, q2) of coefficient c_i from its residues.
__device__ __forceinline__ void crt_digits(uint64_t a1, uint64_t a2, const RecConsts& rc,
                                           uint64_t& q0, uint64_t& q1, uint64_t& q2) {
  const uint64_t psi = a2 >= a1 ? a2 - a1 : a2 + (rc.P2.p - a1);
  const uint64_t phi = mont_mul(psi, rc.r_tilde, rc.P2);
  const u128 c = (u128)rc.p1 * phi + a1;
  u128 t, u;
  q0 = divmod_B(c, rc, t);
  q1 = divmod_B(t, rc, u);
  q2 = (uint64_t)u;
}

// Carry maps {0,1,2} -> {0,1,2}, two bits per image: bits [2c, 2c+2) = f(c).
constexpr uint32_t kIdentityMap = 0u | (1u << 2) | (2u << 4);

__device__ __forceinline__ uint32_t carry_map(uint64_t s, uint64_t B) {
  uint32_t m = 0;
#pragma unroll
  for (uint32_t c = 0; c < 3; ++c) {
    const uint64_t t = s + c;
    const uint32_t o = t >= 2 * B ? 2u : (t >= B ? 1u : 0u);
    m |= o << (2 * c);
  }
  return m;
}
__device__ __forceinline__ uint32_t apply_map(uint32_t f, uint32_t c) { return (f >> (2 * c)) & 3u; }
// (later o earlier)(c) = later(earlier(c))
__device__ __forceinline__ uint32_t compose(uint32_t later, uint32_t earlier) {
  uint32_t m = 0;
#pragma unroll
  for (uint32_t c = 0; c < 3; ++c) m |= apply_map(later, apply_map(earlier, c)) << (2 * c);
  return m;
}

// Exclusive scan of the per-thread maps of one workgroup (thread order =
// position order).  Returns the map of everything before this thread;
// *total receives the map of the whole workgroup.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t f, uint32_t* total) {
  __shared__ uint32_t wave_tot[kRecThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = f;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc = compose(inc, o);
  }
  uint32_t exc = __shfl_up(inc, 1, 64);
  if (lane == 0) exc = kIdentityMap;
  if (lane == 63) wave_tot[wid] = inc;
  __syncthreads();
  uint32_t before = kIdentityMap;
  for (int w = 0; w < wid; ++w) before = compose(wave_tot[w], before);
  uint32_t all = kIdentityMap;
  for (int w = 0; w < kRecThreads / 64; ++w) all = compose(wave_tot[w], all);
  *total = all;
  return compose(exc, before);
}

// Pass 1: CRT digits, s_i, per-workgroup carry map.
__global__ void __launch_bounds__(kRecThreads)
k_rec_local(RecConsts rc, const uint64_t* __restrict__ res1, const uint64_t* __restrict__ res2,
            uint64_t* __restrict__ s_out, uint32_t* __restrict__ block_map) {
  __shared__ uint64_t tail_q1[kRecThreads], tail_q2a[kRecThreads], tail_q2b[kRecThreads];
  const uint64_t base = (uint64_t)blockIdx.x * kRecBlock + (uint64_t)threadIdx.x * kRecPT;
  uint64_t q0[kRecPT], q1[kRecPT], q2[kRecPT];
#pragma unroll
  for (int u = 0; u < kRecPT; ++u) {
    const uint64_t i = base + u;
    if (i < rc.NP) crt_digits(res1[i], res2[i], rc, q0[u], q1[u], q2[u]);
    else { q0[u] = q1[u] = q2[u] = 0; }
  }
  // q1 of the previous position and q2 of the two previous positions
  tail_q1[threadIdx.x] = q1[kRecPT - 1];
  tail_q2a[threadIdx.x] = q2[kRecPT - 1];
  tail_q2b[threadIdx.x] = q2[kRecPT - 2];
  __syncthreads();
  uint64_t pq1, pq2_1, pq2_2;   // q1[i-1], q2[i-1], q2[i-2] for the thread's first position
  if (threadIdx.x > 0) {
    pq1 = tail_q1[threadIdx.x - 1];
    pq2_1 = tail_q2a[threadIdx.x - 1];
    pq2_2 = tail_q2b[threadIdx.x - 1];
  } else {
    uint64_t a0, a1v, a2v, b0, b1v, b2v;
    if (base >= 1) crt_digits(res1[base - 1], res2[base - 1], rc, a0, a1v, a2v);
    else a0 = a1v = a2v = 0;
    if (base >= 2) crt_digits(res1[base - 2], res2[base - 2], rc, b0, b1v, b2v);
    else b0 = b1v = b2v = 0;
    pq1 = a1v;
    pq2_1 = a2v;
    pq2_2 = b2v;
  }
  uint32_t f = kIdentityMap;
#pragma unroll
  for (int u = 0; u < kRecPT; ++u) {
    const uint64_t prev_q1 = u >= 1 ? q1[u - 1] : pq1;
    const uint64_t prev2_q2 = u >= 2 ? q2[u - 2] : (u == 1 ? pq2_1 : pq2_2);
    const uint64_t s = q0[u] + prev_q1 + prev2_q2;
    const uint64_t i = base + u;
    if (i < rc.NP) {
      s_out[i] = s;
      f = compose(carry_map(s, rc.B), f);
    }
  }
  uint32_t total;
  block_exclusive_scan(f, &total);
  if (threadIdx.x == 0) block_map[blockIdx.x] = total;
}

// Pass 2: carry into every workgroup, cin[0] = 0, cin[b+1] = map_b(cin[b]).
// One workgroup: each thread folds a contiguous chunk of maps, the chunk
// maps are scanned, then each chunk is replayed to emit its carries.
__global__ void __launch_bounds__(kRecThreads)
k_rec_blocks(const uint32_t* __restrict__ block_map, uint32_t* __restrict__ block_cin, uint32_t nb) {
  const uint32_t per = (nb + kRecThreads - 1) / kRecThreads;
  const uint32_t lo = threadIdx.x * per;
  const uint32_t hi = lo + per < nb ? lo + per : nb;
  uint32_t f = kIdentityMap;
  for (uint32_t b = lo; b < hi; ++b) f = compose(block_map[b], f);
  uint32_t total;
  const uint32_t before = block_exclusive_scan(f, &total);
  uint32_t c = apply_map(before, 0);
  for (uint32_t b = lo; b < hi; ++b) {
    block_cin[b] = c;
    c = apply_map(block_map[b], c);
  }
}

// Pass 3: apply carries, z_i = (s_i + cin_i) mod B, then regroup the
// workgroup's base-10^k digits into the base-10^19 limbs that start in it.
__device__ __forceinline__ uint64_t div_p10(uint64_t x, int e, const DivTable* __restrict__ dt) {
  if (e == 0) return x;
  return __umul64hi(x >> e, dt->mag[e]) >> dt->sh[e];
}

__global__ void __launch_bounds__(kRecThreads)
k_rec_apply(RecConsts rc, const DivTable* __restrict__ dt, const uint64_t* __restrict__ s_in,
            const uint32_t* __restrict__ block_map, const uint32_t* __restrict__ block_cin,
            uint64_t* __restrict__ out) {
  __shared__ uint64_t z[kRecBlock + 2];
  const uint64_t bbase = (uint64_t)blockIdx.x * kRecBlock;
  const uint64_t base = bbase + (uint64_t)threadIdx.x * kRecPT;
  const uint64_t B = rc.B;
  uint64_t s[kRecPT];
  uint32_t f = kIdentityMap;
#pragma unroll
  for (int u = 0; u < kRecPT; ++u) {
    const uint64_t i = base + u;
    s[u] = i < rc.NP ? s_in[i] : 0;
    if (i < rc.NP) f = compose(carry_map(s[u], B), f);
  }
  uint32_t total;
  const uint32_t before = block_exclusive_scan(f, &total);
  const uint32_t cin_block = block_cin[blockIdx.x];
  uint32_t c = apply_map(before, cin_block);
#pragma unroll
  for (int u = 0; u < kRecPT; ++u) {
    uint64_t t = s[u] + c;
    uint32_t o = 0;
    if (t >= B) { t -= B; o = 1; }
    if (t >= B) { t -= B; o = 2; }
    z[threadIdx.x * kRecPT + u] = t;
    c = o;
  }
  // two digits past the block end (needed by limbs that start here)
  if (threadIdx.x == 0) {
    uint32_t cc = apply_map(total, cin_block);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint64_t i = bbase + kRecBlock + u;
      uint64_t t = i < rc.NP ? s_in[i] + cc : 0;
      uint32_t o = 0;
      if (t >= B) { t -= B; o = 1; }
      if (t >= B) { t -= B; o = 2; }
      z[kRecBlock + u] = t;
      cc = o;
    }
  }
  __syncthreads();
  // limbs j with first digit 19j in [k*bbase, k*(bbase + kRecBlock))
  const uint64_t k = (uint64_t)rc.k;
  const uint64_t d_lo = k * bbase, d_hi = k * (bbase + kRecBlock);
  const uint64_t j_lo = (d_lo + 18) / 19;
  uint64_t j_hi = (d_hi + 18) / 19;
  if (j_hi > rc.nout) j_hi = rc.nout;
  for (uint64_t j = j_lo + threadIdx.x; j < j_hi; j += kRecThreads) {
    const uint64_t d0 = 19 * j - d_lo;          // digit offset inside the block
    const uint64_t i0 = d0 / k;
    const int o = (int)(d0 - i0 * k);
    const int have0 = rc.k - o;
    uint64_t limb = div_p10(z[i0], o, dt);
    const int need = 19 - have0;
    if (need <= rc.k) {
      const uint64_t z1 = z[i0 + 1];
      limb += (z1 - div_p10(z1, need, dt) * dt->pow10[need]) * dt->pow10[have0];
    } else {
      const int need2 = need - rc.k;
      const uint64_t z2 = z[i0 + 2];
      limb += z[i0 + 1] * dt->pow10[have0];
      limb += (z2 - div_p10(z2, need2, dt) * dt->pow10[need2]) * dt->pow10[have0 + rc.k];
    }
    out[j] = limb;
  }
}

__global__ void k_zero(uint64_t* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0;
}

size_t recover_scratch_words(const PlanDev& pl) {
  const uint64_t NP = pl.n + pl.m;
  const uint64_t nblk = (NP + kRecBlock - 1) / kRecBlock;
  return NP + nblk;   // s (u64 per position) + two u32 per block
}

hipError_t launch_recover(const PlanDev& pl, const Consts& cs, const DivTable* dt,
                          const uint64_t* res1, const uint64_t* res2, uint64_t* out,
                          uint64_t* scratch, hipStream_t st, Marks* marks) {
  RecConsts rc;
  rc.P2 = cs.P[1];
  rc.p1 = cs.P[0].p;
  rc.r_tilde = cs.r_tilde;
  rc.k = pl.k;
  rc.B = 1;
  for (int i = 0; i < pl.k; ++i) rc.B *= 10;
  rc.sh = __builtin_clzll(rc.B);
  rc.d = rc.B << rc.sh;
  rc.v = (uint64_t)((~(u128)0) / rc.d - ((u128)1 << 64));
  rc.NP = pl.n + pl.m;
  rc.nout = pl.na + pl.nb;
  const uint64_t nblk = (rc.NP + kRecBlock - 1) / kRecBlock;
  uint64_t* s = scratch;
  uint32_t* maps = (uint32_t*)(scratch + rc.NP);
  uint32_t* cins = maps + nblk;
  hipLaunchKernelGGL(k_rec_local, dim3((unsigned)nblk), dim3(kRecThreads), 0, st, rc, res1, res2, s, maps);
  if (marks) marks->mark(kRecLocal, st);
  hipLaunchKernelGGL(k_rec_blocks, dim3(1), dim3(kRecThreads), 0, st, maps, cins, (uint32_t)nblk);
  if (marks) marks->mark(kRecBlocks, st);
  hipLaunchKernelGGL(k_rec_apply, dim3((unsigned)nblk), dim3(kRecThreads), 0, st, rc, dt, s, maps, cins, out);
  if (marks) marks->mark(kRecApply, st);
  return hipGetLastError();
}

hipError_t launch_zero(uint64_t* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, out, n);
  return hipGetLastError();
}

}  // namespace dmi
