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
#include <stdlib.h>

#include "rec_dev.hpp"

namespace dmi {

constexpr int kRecThreads = 256;
constexpr int kScanThreads = 1024;

// Pass 1: CRT digits, s_i = q0_i + q1_(i-1) + q2_(i-2), and the carry map of
// every block of kRecThreads * PT positions (Section 8.2: the recovery is a
// sequential carry; the maps make it a scan).  A workgroup loops over
// blocks; thread t takes PT consecutive positions, lanes 0 and 1 also the
// two positions before the block (their q1, q2 feed its first s values).
// The digits are computed branch-free so the PT independent chains of a
// thread interleave.  Each block's map is a plain store: the scan that
// consumes the maps is the next launch.
template <int PT>
__global__ void __launch_bounds__(kRecThreads)
k_rec_crt(Work w, RecTable rt) {
  const ProdDesc d = load_desc(w);
  const RecConsts rc = rec_consts(rt, d);
  const uint64_t* __restrict__ res1 = d.ws;
  const uint64_t* __restrict__ res2 = d.ws + d.pl.N;
  uint64_t* __restrict__ s_out = d.ws + 2 * d.pl.N;
  uint32_t* __restrict__ maps = d.rec_sync;
  constexpr int BLK = kRecThreads * PT;
  __shared__ uint64_t tail_q1[kRecThreads + 1], tail_q2a[kRecThreads + 1], tail_q2b[kRecThreads + 1];
  for (uint32_t blk = blockIdx.x; blk < d.nblk; blk += gridDim.x) {
    const int64_t bbase = (int64_t)blk * BLK;
    const int64_t base = bbase + (int64_t)threadIdx.x * PT;
    uint64_t a1[PT], a2[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int64_t i = base + u;
      const bool in = (uint64_t)i < rc.NP;
      a1[u] = in ? res1[i] : 0;
      a2[u] = in ? res2[i] : 0;
    }
    uint64_t q0[PT], q1[PT], q2[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) crt_digits(a1[u], a2[u], rc, q0[u], q1[u], q2[u]);
    if (threadIdx.x < 2) {
      // position bbase-1 (lane 0) or bbase-2 (lane 1); zero before the start
      const int64_t i = bbase - 1 - (int64_t)threadIdx.x;
      const uint64_t x1 = i >= 0 ? res1[i] : 0, x2 = i >= 0 ? res2[i] : 0;
      uint64_t p0, p1, p2;
      crt_digits(x1, x2, rc, p0, p1, p2);
      if (threadIdx.x == 0) {
        tail_q1[0] = p1;
        tail_q2a[0] = p2;
      } else {
        tail_q2b[0] = p2;
      }
    }
    tail_q1[threadIdx.x + 1] = q1[PT - 1];
    tail_q2a[threadIdx.x + 1] = q2[PT - 1];
    tail_q2b[threadIdx.x + 1] = q2[PT - 2];
    __syncthreads();
    const uint64_t pq1 = tail_q1[threadIdx.x];
    const uint64_t pq2_1 = tail_q2a[threadIdx.x];
    const uint64_t pq2_2 = tail_q2b[threadIdx.x];
    uint32_t f = kIdentityMap;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const uint64_t prev_q1 = u >= 1 ? q1[u - 1] : pq1;
      const uint64_t prev2_q2 = u >= 2 ? q2[u - 2] : (u == 1 ? pq2_1 : pq2_2);
      const uint64_t sv = q0[u] + prev_q1 + prev2_q2;
      if ((uint64_t)(base + u) < rc.NP) {
        s_out[base + u] = sv;
        f = compose(carry_map(sv, rc.B), f);
      }
    }
    uint32_t total;
    block_exclusive_scan(f, &total);
    if (threadIdx.x == 0) maps[blk] = total;
    __syncthreads();   // the tail arrays and scan words are reused by the next block
  }
}

// Scan of the block maps: the incoming carry of every block (the carry into
// position 0 is 0).  One workgroup per product; thread t composes a
// contiguous run of maps, then the runs are scanned across the workgroup.
__global__ void __launch_bounds__(kScanThreads)
k_rec_scan(Work w, RecTable rt) {
  const ProdDesc d = load_desc(w);
  const RecConsts rc = rec_consts(rt, d);
  const uint32_t* __restrict__ maps = d.rec_sync;
  uint32_t* __restrict__ cins = (uint32_t*)(d.ws + 2 * d.pl.N + rc.NP);
  const uint32_t nb = d.nblk;
  const uint32_t per = (nb + kScanThreads - 1) / kScanThreads;
  const uint32_t lo = threadIdx.x * per < nb ? threadIdx.x * per : nb;
  const uint32_t hi = lo + per < nb ? lo + per : nb;
  uint32_t g = kIdentityMap;
  for (uint32_t b = lo; b < hi; ++b) g = compose(maps[b], g);
  uint32_t all;
  const uint32_t before = block_exclusive_scan(g, &all);
  uint32_t c = apply_map(before, 0);
  for (uint32_t b = lo; b < hi; ++b) {
    cins[b] = c;
    c = apply_map(maps[b], c);
  }
}

// Pass 2: z_i = (s_i + carry_i) mod B from the block's incoming carry and a
// scan of its maps, then the base-10^19 limbs whose first digit lies in the
// block's digit range (digits of the two positions after it are included: a
// limb may end there).  The incoming carry comes from k_rec_scan, or with
// PREFIX (products of at most kPrefixBlocks blocks) from composing the maps
// of all earlier blocks here, which saves the scan launch.
constexpr uint32_t kPrefixBlocks = 2048;

template <int PT, bool PREFIX>
__global__ void __launch_bounds__(kRecThreads)
k_rec_apply(Work w, RecTable rt, const DivTable* __restrict__ dt_g) {
  constexpr int BLK = kRecThreads * PT;
  const ProdDesc d = load_desc(w);
  const RecConsts rc = rec_consts(rt, d);
  const uint64_t* __restrict__ s_in = d.ws + 2 * d.pl.N;
  const uint32_t* __restrict__ cins = (const uint32_t*)(s_in + rc.NP);
  uint64_t* __restrict__ out = d.out;
  __shared__ uint64_t z[BLK + 2];
  __shared__ DivTable sdt;
  stage_words<kRecThreads, (int)(sizeof(DivTable) / 4)>(reinterpret_cast<uint32_t*>(&sdt),
                                                        reinterpret_cast<const uint32_t*>(dt_g));
  __syncthreads();   // the table is written by some threads and read by all
  const DivTable* dt = &sdt;
  const uint64_t B = rc.B;
  const uint64_t k = (uint64_t)rc.k;
  for (uint32_t blk = blockIdx.x; blk < d.nblk; blk += gridDim.x) {
    const uint64_t bbase = (uint64_t)blk * BLK;
    const uint64_t base = bbase + (uint64_t)threadIdx.x * PT;
    uint64_t s[PT];
    uint32_t f = kIdentityMap;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const uint64_t i = base + u;
      s[u] = i < rc.NP ? s_in[i] : 0;
      if (i < rc.NP) f = compose(carry_map(s[u], B), f);
    }
    uint32_t cin;
    if constexpr (PREFIX) {
      // maps of blocks 0 .. blk-1 in order: runs per thread, then a scan
      const uint32_t* __restrict__ maps = d.rec_sync;
      const uint32_t per = (blk + kRecThreads - 1) / kRecThreads;
      const uint32_t lo = threadIdx.x * per < blk ? threadIdx.x * per : blk;
      const uint32_t hi = lo + per < blk ? lo + per : blk;
      uint32_t g = kIdentityMap;
      for (uint32_t b = lo; b < hi; ++b) g = compose(maps[b], g);
      uint32_t all;
      block_exclusive_scan(g, &all);
      cin = apply_map(all, 0);
      __syncthreads();   // the scan's shared words are used again below
    } else {
      cin = cins[blk];
    }
    uint32_t total;
    const uint32_t before = block_exclusive_scan(f, &total);
    uint32_t c = apply_map(before, cin);
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      uint64_t t = s[u] + c;
      uint32_t o = 0;
      if (t >= B) { t -= B; o = 1; }
      if (t >= B) { t -= B; o = 2; }
      z[threadIdx.x * PT + u] = t;
      c = o;
    }
    if (threadIdx.x == kRecThreads - 1) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint64_t i = bbase + BLK + u;
        uint64_t t = (i < rc.NP ? s_in[i] : 0) + c;
        uint32_t o = 0;
        if (t >= B) { t -= B; o = 1; }
        if (t >= B) { t -= B; o = 2; }
        z[BLK + u] = t;
        c = o;
      }
    }
    __syncthreads();

    // limbs j with first digit 19j in [k*bbase, k*(bbase + BLK))
    const uint64_t d_lo = k * bbase, d_hi = k * (bbase + BLK);
    const uint64_t j_lo = (d_lo + 18) / 19;
    uint64_t j_hi = (d_hi + 18) / 19;
    if (j_hi > rc.nout) j_hi = rc.nout;
    for (uint64_t j = j_lo + threadIdx.x; j < j_hi; j += kRecThreads) {
      const uint32_t d0 = (uint32_t)(19 * j - d_lo);     // digit offset inside the block, < 2^17
      const uint32_t i0 = (uint32_t)(((uint64_t)d0 * rc.kinv) >> 22);
      const int o = (int)(d0 - i0 * (uint32_t)rc.k);
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
    __syncthreads();   // z is reused by the next block
  }
}

__global__ void k_zero(uint64_t* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0;
}

__global__ void k_fill32(uint32_t* __restrict__ out, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = v;
}

constexpr int kRecPT = 5;
// A lone product whose recovery would take fewer blocks than the device has
// CUs runs it at 2 positions per thread instead (shorter per-thread chains,
// 2.5 times the workgroups); 2 is the least the kernels take (a thread reads
// the digits of the two positions before its first one from its neighbour).
constexpr int kRecPTLean = 2;
constexpr size_t kLeanRecBlocks = 256;

size_t recover_blocks(const PlanDev& pl, bool lean) {
  const size_t blk = (size_t)kRecThreads * (lean ? kRecPTLean : kRecPT);    // positions per block
  return (size_t)((pl.n + pl.m + blk - 1) / blk);
}

bool recover_lean(const PlanDev& pl) { return recover_blocks(pl, false) < kLeanRecBlocks; }

// Workgroups of the grid-stride recovery passes: one round of what the
// device holds at once (four 256-thread workgroups per CU: the recovery
// kernels' registers allow four wavefronts per SIMD), never more than the
// blocks of the longest product.  A larger grid leaves its last workgroups
// as a second, partial round (C3's k_rec_apply 31.1 us with 1536, 28.9 us
// with 1024).
static unsigned recover_grid(uint32_t max_nblk) {
  const uint32_t cap = 256 * 4;
  return max_nblk < cap ? (max_nblk ? max_nblk : 1) : cap;
}

RecTable make_rec_table(const Consts& cs, const DivTable* dt_host) {
  RecTable rt;
  rt.P2 = cs.P[1];
  rt.p1 = cs.P[0].p;
  rt.r_tilde = cs.r_tilde;
  for (int i = 0; i < 6; ++i) {
    const int k = kMinK + i;
    uint64_t B = 1;
    for (int j = 0; j < k; ++j) B *= 10;
    rt.B[i] = B;
    rt.sh[i] = (uint32_t)__builtin_clzll(B);
    rt.d[i] = B << rt.sh[i];
    rt.v[i] = (uint64_t)((~(u128)0) / rt.d[i] - ((u128)1 << 64));
    rt.kinv[i] = (uint32_t)(((1u << 22) + k - 1) / k);
    rt.Ph[i] = rt.p1 / B;
    rt.Pl[i] = rt.p1 % B;
    rt.bmag[i] = dt_host->mag[k];
    rt.bsh[i] = dt_host->sh[k];
    rt.inv_B[i] = 1.0 / (double)B;
  }
  return rt;
}

hipError_t launch_recover(const Work& w, const Shape& sh, const Consts& cs, const DivTable* dt,
                          const DivTable* dt_host, hipStream_t st, Marks* marks) {
  const RecTable rt = make_rec_table(cs, dt_host);
  const unsigned g = recover_grid(sh.max_nblk);
  const bool prefix = sh.max_nblk <= kPrefixBlocks;
  if (sh.rec_lean)
    hipLaunchKernelGGL(k_rec_crt<kRecPTLean>, dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt);
  else
    hipLaunchKernelGGL(k_rec_crt<kRecPT>, dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt);
  if (!prefix) hipLaunchKernelGGL(k_rec_scan, dim3(1, 1, w.count), dim3(kScanThreads), 0, st, w, rt);
  if (marks) marks->mark(kRecCrt, st);
  if (sh.rec_lean && prefix)
    hipLaunchKernelGGL((k_rec_apply<kRecPTLean, true>), dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt, dt);
  else if (sh.rec_lean)
    hipLaunchKernelGGL((k_rec_apply<kRecPTLean, false>), dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt, dt);
  else if (prefix)
    hipLaunchKernelGGL((k_rec_apply<kRecPT, true>), dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt, dt);
  else
    hipLaunchKernelGGL((k_rec_apply<kRecPT, false>), dim3(g, 1, w.count), dim3(kRecThreads), 0, st, w, rt, dt);
  if (marks) marks->mark(kRecApply, st);
  return hipGetLastError();
}

hipError_t launch_fill32(void* out, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill32, dim3(blocks), dim3(256), 0, st, (uint32_t*)out, n, v);
  return hipGetLastError();
}

hipError_t launch_zero(uint64_t* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, out, n);
  return hipGetLastError();
}

}  // namespace dmi
