// Whole products in one workgroup, for short transforms (N <= kSmallMaxN in
// launches of at least kSmallMinCount products, N <= kSmallSoloMaxN else).
//
// A product whose transform fits the LDS of one workgroup runs every step
// of the method in one kernel: digit-group split (Section 3.2), for each
// prime the forward transforms of both operands, the pointwise REDC
// product, the inverse transform and the scale R^2 N^-1 (Sections 5, 6),
// then the CRT digits, the carry scan and the regrouping into base-10^19
// limbs (Section 8.2).  The transform is one in-LDS pass (no inter-pass
// factor): DIF natural -> bit-reversed, DIT back (Section 5.4).  For
// N = 3M the length-3 DFT across the thirds and the factors w_N^(+-s*q)
// come first (forward) or last (inverse), around three M-point transforms
// (Section 7.8).  A batch launches one workgroup per product of the class:
// the many short products of a batch cost one launch instead of seven.
#include <algorithm>

#include "rec_dev.hpp"

namespace dmi {

constexpr int kSmallThreads = 256;

template <int LOGM>
struct SmallGeom {
  static constexpr int LOGE = LOGM < 4 ? LOGM : 4;
  using G = Geometry<LOGM, LOGE>;
};

// LDS words of the whole-product kernel: X and Y (F sub-rows each, padded
// layout) and the digit array Q (N + 2 words).
constexpr size_t small_lds_words(int logm, int f) {
  return 2 * (size_t)f * (((size_t)1 << logm) + (((size_t)1 << logm) >> (logm < 4 ? logm : 4)) + 1) +
         ((size_t)f << logm) + 2;
}

// One whole product by the workgroup, in `lds` (small_lds_words(LOGM, F)
// words); scale[] is R^2 N^-1 in Montgomery form per prime, dt the
// power-of-ten table in LDS.  Leaves the product in d.out; the caller
// synchronises the workgroup before `lds` is reused.
template <int LOGM, bool R3>
__device__ __forceinline__ void small_product(const ProdDesc& d, const Consts& cs, const TwiddleSet& tw,
                                              const uint64_t (&scale)[2], const DivTable* dt,
                                              const RecTable& rt, uint64_t* lds) {
  constexpr int LOGE = SmallGeom<LOGM>::LOGE;
  using G = typename SmallGeom<LOGM>::G;
  constexpr int M = G::L, NT = G::NT, S = G::STRIDE;
  constexpr int F = R3 ? 3 : 1;
  constexpr int N = F * M;
  constexpr bool kWave = NT <= 64;
  static_assert(NT <= kSmallThreads, "one transform per workgroup at most");
  constexpr int PER_PASS = kSmallThreads / NT;       // sub-transforms run side by side
  uint64_t* X = lds;                 // operand a, then the product, then q1
  uint64_t* Y = lds + F * S;         // operand b, then q2
  uint64_t* Q = lds + 2 * F * S;     // residues mod p1, then q0, then the digits z
  const RecConsts rc = rec_consts(rt, d);
  const bool square = d.square != 0;
  const int nsub = square ? F : 2 * F;
  // point n of an operand (natural order) lives at sub-row n / M, slot n mod M
  auto at = [&](uint64_t* A, int n) -> uint64_t& { return A[(n / M) * S + lds_pos<LOGE>(n % M)]; };

#pragma unroll 1
  for (int pi = 0; pi < 2; ++pi) {
    const Prime P = cs.P[pi];
    for (int n = threadIdx.x; n < N; n += kSmallThreads) {
      at(X, n) = split_group(d.a, d.pl.na, d.pl.n, (uint64_t)n, d.pl.k, dt, d.status);
      if (!square) at(Y, n) = split_group(d.b, d.pl.nb, d.pl.m, (uint64_t)n, d.pl.k, dt, d.status);
    }
    __syncthreads();
    if constexpr (R3) {
      const uint64_t* w3 = tw.r3_fwd[pi] + r3_table_offset(LOGM);
      for (int j = threadIdx.x; j < (square ? M : 2 * M); j += kSmallThreads) {
        uint64_t* A = j < M ? X : Y;
        const int q = j % M, o = lds_pos<LOGE>(q);
        uint64_t x0 = A[o], x1 = A[S + o], x2 = A[2 * S + o];
        dft3(x0, x1, x2, cs.kappa[pi][0], P);
        A[o] = x0;
        A[S + o] = mont_mul(x1, w3[q], P);
        A[2 * S + o] = mont_mul(x2, w3[2 * q], P);
      }
      __syncthreads();
    }
    const uint64_t* rf = tw.len_fwd[pi] + root_block_offset(LOGM);
    for (int b0 = 0; b0 < nsub; b0 += PER_PASS) {
      const int idx = b0 + (int)threadIdx.x / NT;
      const bool active = (int)threadIdx.x / NT < PER_PASS && idx < nsub;
      uint64_t* A = !active ? X : (idx < F ? X + idx * S : Y + (idx - F) * S);
      lds_transform<LOGM, LOGE, false, kWave>(A, rf, P, (int)threadIdx.x % NT, active);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += kSmallThreads) {
      uint64_t& x = at(X, n);
      x = mont_mul(x, square ? x : at(Y, n), P);
    }
    __syncthreads();
    const uint64_t* ri = tw.len_inv[pi] + root_block_offset(LOGM);
    for (int b0 = 0; b0 < F; b0 += PER_PASS) {
      const int idx = b0 + (int)threadIdx.x / NT;
      const bool active = (int)threadIdx.x / NT < PER_PASS && idx < F;
      lds_transform<LOGM, LOGE, true, kWave>(active ? X + idx * S : X, ri, P, (int)threadIdx.x % NT, active);
    }
    __syncthreads();
    // (inverse length-3 step), the scale R^2 N^-1; residues of p1 go to Q
    const uint64_t sc = scale[pi];
    for (int q = threadIdx.x; q < M; q += kSmallThreads) {
      const int o = lds_pos<LOGE>(q);
      uint64_t x[F];
#pragma unroll
      for (int s = 0; s < F; ++s) x[s] = canonical<true>(X[s * S + o], P);
      if constexpr (R3) {
        const uint64_t* w3 = tw.r3_inv[pi] + r3_table_offset(LOGM);
        x[1] = mont_mul(x[1], w3[q], P);
        x[2] = mont_mul(x[2], w3[2 * q], P);
        dft3(x[0], x[1], x[2], cs.kappa[pi][1], P);
      }
#pragma unroll
      for (int s = 0; s < F; ++s) {
        const uint64_t v = mont_mul(x[s], sc, P);
        if (pi == 0) Q[s * M + q] = v;
        else X[s * S + o] = v;
      }
    }
    __syncthreads();
  }

  // CRT digits in place: q0 -> Q, q1 -> X, q2 -> Y
  const int NP = (int)rc.NP;
  for (int i = threadIdx.x; i < NP; i += kSmallThreads) {
    uint64_t q0, q1, q2;
    crt_digits(Q[i], at(X, i), rc, q0, q1, q2);
    Q[i] = q0;
    at(X, i) = q1;
    at(Y, i) = q2;
  }
  if (threadIdx.x < 2) Q[N + threadIdx.x] = 0;
  __syncthreads();
  // carries: thread t owns positions [t*per, t*per + per)
  const int per = (NP + kSmallThreads - 1) / kSmallThreads;
  const int lo = (int)threadIdx.x * per < NP ? (int)threadIdx.x * per : NP;
  const int hi = lo + per < NP ? lo + per : NP;
  auto s_at = [&](int i) -> uint64_t {
    return Q[i] + (i >= 1 ? at(X, i - 1) : 0) + (i >= 2 ? at(Y, i - 2) : 0);
  };
  uint32_t f = kIdentityMap;
  for (int i = lo; i < hi; ++i) f = compose(carry_map(s_at(i), rc.B), f);
  uint32_t total;
  const uint32_t before = block_exclusive_scan(f, &total);
  uint32_t c = apply_map(before, 0);
  for (int i = lo; i < hi; ++i) {
    uint64_t t = s_at(i) + c;
    uint32_t o = 0;
    if (t >= rc.B) { t -= rc.B; o = 1; }
    if (t >= rc.B) { t -= rc.B; o = 2; }
    Q[i] = t;
    c = o;
  }
  for (int i = NP + (int)threadIdx.x; i < N; i += kSmallThreads) Q[i] = 0;
  __syncthreads();
  // regroup: limb j holds decimal digits [19j, 19j + 19)
  const int k = rc.k;
  for (uint64_t j = threadIdx.x; j < rc.nout; j += kSmallThreads) {
    const uint32_t d0 = (uint32_t)(19 * j);             // < 2^17
    const uint32_t i0 = (uint32_t)(((uint64_t)d0 * rc.kinv) >> 22);
    const int o = (int)(d0 - i0 * (uint32_t)k);
    const int have0 = k - o;
    uint64_t limb = div_p10(Q[i0], o, dt);
    const int need = 19 - have0;
    if (need <= k) {
      const uint64_t z1 = Q[i0 + 1];
      limb += (z1 - div_p10(z1, need, dt) * dt->pow10[need]) * dt->pow10[have0];
    } else {
      const int need2 = need - k;
      const uint64_t z2 = Q[i0 + 2];
      limb += Q[i0 + 1] * dt->pow10[have0];
      limb += (z2 - div_p10(z2, need2, dt) * dt->pow10[need2]) * dt->pow10[have0 + k];
    }
    d.out[j] = limb;
  }
}

// The power-of-ten table, copied into the workgroup's LDS.
__device__ __forceinline__ void load_div_table(DivTable& sdt, const DivTable* __restrict__ dt_g) {
  stage_words<kSmallThreads, (int)(sizeof(DivTable) / 4)>(reinterpret_cast<uint32_t*>(&sdt),
                                                          reinterpret_cast<const uint32_t*>(dt_g));
  __syncthreads();   // the table is written by some threads and read by all
}

// One workgroup per product of one length (grid.z = product).
template <int LOGM, bool R3>
__global__ void __launch_bounds__(kSmallThreads)
k_small(Work w, Consts cs, TwiddleSet tw, const DivTable* __restrict__ dt_g, RecTable rt) {
  extern __shared__ uint64_t lds[];
  __shared__ DivTable sdt;
  load_div_table(sdt, dt_g);
  small_product<LOGM, R3>(load_desc(w), cs, tw, tw.scale, &sdt, rt, lds);
}

// Persistent form: a grid sized to what the device holds at once takes the
// products of w.many[0 .. count), of mixed lengths within one tier (lengths
// with alike LDS needs), from a queue: each workgroup claims the next
// product with one atomic increment of *head (zero at launch) and returns
// once the queue is empty, so every workgroup exits.  Each product carries
// its own scale.  The host orders the queue longest first.
// One product of the queue, as a call of its own: each length's body gets
// its own register allocation instead of the union of every length's.
template <int LOGM, bool R3>
__device__ __attribute__((noinline)) void queued_product(const ProdDesc* dp, const Consts* cs,
                                                         const TwiddleSet* tw, const DivTable* dt,
                                                         const RecTable* rt, uint64_t* lds) {
  const ProdDesc d = *dp;
  small_product<LOGM, R3>(d, *cs, *tw, d.scale, dt, *rt, lds);
}

// Waves per SIMD the queued kernel of a tier is held to: the occupancy
// of the per-length kernels of its lengths (their registers decide it).
constexpr int queue_waves(int tier) { return tier == 0 ? 3 : (tier == 1 ? 2 : 1); }

template <int TIER>
__global__ void __launch_bounds__(kSmallThreads) __attribute__((amdgpu_waves_per_eu(queue_waves(TIER))))
k_small_queue(Work w, uint32_t* head, Consts cs, TwiddleSet tw, const DivTable* __restrict__ dt_g,
              RecTable rt) {
  extern __shared__ uint64_t lds[];
  __shared__ DivTable sdt;
  __shared__ uint32_t slot;
  load_div_table(sdt, dt_g);
  for (;;) {
    __syncthreads();               // the last product's LDS reads, and every read of slot, are done
    if (threadIdx.x == 0) slot = atomicAdd(head, 1u);
    __syncthreads();
    // the same for the whole workgroup: read as a scalar, so the descriptor
    // below is loaded into scalar registers as with one product per workgroup
    const uint32_t i = __builtin_amdgcn_readfirstlane(slot);
    if (i >= w.count) return;
    const ProdDesc* dp = w.many + i;
    const int logm = dp->pl.logN;    // sub-transforms of 2^logN points (N = 2^logN or 3 * 2^logN)
    // only this tier's lengths are compiled in (registers follow the largest)
#define P2(l) case l: queued_product<l, false>(dp, &cs, &tw, &sdt, &rt, lds); break;
#define P3(l) case l: queued_product<l, true>(dp, &cs, &tw, &sdt, &rt, lds); break;
    if constexpr (TIER == 0) {
      if (dp->pl.rad3) { switch (logm) { P3(4) P3(5) P3(6) P3(7) P3(8) default: break; } }
      else { switch (logm) { P2(2) P2(3) P2(4) P2(5) P2(6) P2(7) P2(8) default: break; } }
    } else if constexpr (TIER == 1) {
      if (dp->pl.rad3) { switch (logm) { P3(9) default: break; } }
      else { switch (logm) { P2(9) P2(10) default: break; } }
    } else {
      if (dp->pl.rad3) { switch (logm) { P3(10) default: break; } }
      else { switch (logm) { P2(11) P2(12) default: break; } }
    }
#undef P2
#undef P3
  }
}

template <int LOGM, bool R3>
static hipError_t small_launch(const Work& w, const Consts& cs, const TwiddleSet& tw, const DivTable* dt,
                               const RecTable& rt, hipStream_t st) {
  const size_t lds = small_lds_words(LOGM, R3 ? 3 : 1) * sizeof(uint64_t);
  auto kern = k_small<LOGM, R3>;
  const hipError_t e = allow_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(1, 1, w.count), dim3(kSmallThreads), lds, st, w, cs, tw, dt, rt);
  return hipGetLastError();
}

int small_tier(const PlanDev& pl) {
  // by the kernels' registers and LDS: tier 0 sub-transforms of up to 2^8
  // points (N <= 256, or 768 with the factor 3; up to ~133 VGPRs, 19 KB),
  // tier 1 of 2^9..2^10 (N <= 1024, or 1536; ~214 VGPRs, 38 KB), tier 2
  // the rest (N <= 4096, or 3072; ~266 VGPRs, 100 KB)
  return pl.logN <= 8 ? 0 : ((pl.logN <= 10 && !(pl.rad3 && pl.logN == 10)) ? 1 : 2);
}

size_t small_lds_bytes(const PlanDev& pl) {
  return small_lds_words((int)pl.logN, pl.rad3 ? 3 : 1) * sizeof(uint64_t);
}

template <int TIER>
static hipError_t small_queue_launch(const Work& w, uint32_t* head, size_t lds, const Consts& cs,
                                     const TwiddleSet& tw, const DivTable* dt, const RecTable& rt,
                                     hipStream_t st) {
  auto kern = k_small_queue<TIER>;
  hipError_t e = allow_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  // as many workgroups as the device holds at once (the queue balances
  // the products' uneven work), never more than there are products
  int per_cu = 0, dev = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, kSmallThreads, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t cap = (size_t)(per_cu > 0 ? per_cu : 1) * (size_t)(cus > 0 ? cus : 1);
  const unsigned grid = (unsigned)std::min<size_t>(cap, w.count);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kSmallThreads), lds, st, w, head, cs, tw, dt, rt);
  return hipGetLastError();
}

hipError_t launch_small_queue(const Work& w, int tier, size_t lds, uint32_t* head, const Consts& cs,
                              const TwiddleSet& tw, const DivTable* dt, const DivTable* dt_host,
                              hipStream_t st, Marks* marks) {
  if (w.count == 0) return hipSuccess;
  const RecTable rt = make_rec_table(cs, dt_host);
  hipError_t e = hipErrorInvalidValue;
  switch (tier) {
    case 0: e = small_queue_launch<0>(w, head, lds, cs, tw, dt, rt, st); break;
    case 1: e = small_queue_launch<1>(w, head, lds, cs, tw, dt, rt, st); break;
    case 2: e = small_queue_launch<2>(w, head, lds, cs, tw, dt, rt, st); break;
    default: break;
  }
  if (e == hipSuccess && marks) marks->mark(kWhole, st);
  return e;
}

bool small_fits(const PlanDev& pl, size_t count) {
  return pl.N <= (count >= kSmallMinCount ? kSmallMaxN : kSmallSoloMaxN);
}

hipError_t launch_small(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                        const DivTable* dt, const DivTable* dt_host, hipStream_t st, Marks* marks) {
  const RecTable rt = make_rec_table(cs, dt_host);
  // N = 2^logN, or 3 * 2^logN with rad3: the sub-transforms have 2^logN points
  const int logm = sh.logR + sh.logC;
  hipError_t e = hipErrorInvalidValue;
  if (sh.rad3) {
    switch (logm) {
#define X(l) case l: e = small_launch<l, true>(w, cs, tw, dt, rt, st); break;
      X(4) X(5) X(6) X(7) X(8) X(9) X(10)
#undef X
      default: break;
    }
  } else {
    switch (logm) {
#define X(l) case l: e = small_launch<l, false>(w, cs, tw, dt, rt, st); break;
      X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#undef X
      default: break;
    }
  }
  if (e == hipSuccess && marks) marks->mark(kWhole, st);
  return e;
}

}  // namespace dmi
