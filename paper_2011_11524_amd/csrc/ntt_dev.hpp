// Device building blocks of the transforms, shared by the pass kernels
// (ntt.hip) and the whole-product kernel (small.hip): the LDS layout, the
// radix-2^k rounds, the digit-group split, the length-3 DFT.
#pragma once
#include "internal.hpp"

namespace dmi {

// ---------------------------------------------------------------------------
// LDS layout: point i of a transform lives at word i + (i >> LOGE), one pad
// word per 2^LOGE points, so that a thread's 2^LOGE contiguous points (the
// lowest-bit round) fall in distinct banks across a wavefront.
// ---------------------------------------------------------------------------
template <int LOGE>
__device__ __forceinline__ int lds_pos(int i) { return i + (i >> LOGE); }

template <int LOGL, int LOGE>
struct Geometry {
  static constexpr int L = 1 << LOGL;
  static constexpr int E = 1 << LOGE;
  static constexpr int NT = L / E;                   // threads per transform
  static constexpr int STRIDE = L + (L >> LOGE) + 1; // words per transform in LDS (+1: column skew)
  static constexpr int ROUNDS = (LOGL + LOGE - 1) / LOGE;
};

// One radix-2^nb round of an in-LDS transform over bits [lo_b, lo_b+nb).
// Thread t holds E = 2^LOGE points: slot j = (jg << nb) | jl addresses point
//   F = t + jg*NT,  idx = (F mod 2^lo_b) | (jl << lo_b) | ((F >> lo_b) << (lo_b+nb)).
// DIF butterflies run from the top bit of the round down, DIT from the
// bottom up; the factor of the stage on bit b for the pair whose lower
// point is idx is w^((idx mod 2^b) * 2^(LOGL-1-b)) (Sections 5.2, 5.3, 5.5),
// entry idx mod 2^b of that stage's root table (tw: the length's block).
template <int LOGL, int LOGE, bool DIT, int LO_B, int NB>
struct Round {
  using G = Geometry<LOGL, LOGE>;
  static __device__ __forceinline__ int index(int t, int j) {
    const int jg = j >> NB, jl = j & ((1 << NB) - 1);
    const int F = t + jg * G::NT;
    const int lowF = F & ((1 << LO_B) - 1);
    const int highF = F >> LO_B;
    return lowF | (jl << LO_B) | (highF << (LO_B + NB));
  }

  static __device__ __forceinline__ void load(const uint64_t* lds, uint64_t (&v)[G::E], int t) {
#pragma unroll
    for (int j = 0; j < G::E; ++j) v[j] = lds[lds_pos<LOGE>(index(t, j))];
  }
  static __device__ __forceinline__ void store(uint64_t* lds, const uint64_t (&v)[G::E], int t) {
#pragma unroll
    for (int j = 0; j < G::E; ++j) lds[lds_pos<LOGE>(index(t, j))] = v[j];
  }

  // The butterflies of the round on the thread's registers.
  // Canonical ranges: every value in [0, p) before and after each stage.
  // Redundant ranges (kLazy, p < 2^62): a DIF takes values in [0, 2p) and
  // keeps them there; a DIT takes values in [0, 4p) (canonical at its first
  // stage), reduces the upper point of each pair to [0, 2p) and leaves its
  // outputs in [0, 4p) (Harvey's butterflies, the p < mu/4 ranges of
  // Section 8.3).
  static __device__ __forceinline__ void compute(uint64_t (&v)[G::E], const uint64_t* __restrict__ tw,
                                                 const Prime& P, int t) {
    if constexpr (kLazy) {
      compute_lazy(v, tw, P, t);
      return;
    }
    constexpr int E = G::E;
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int lb = DIT ? s : (NB - 1 - s);   // local bit of this stage
      const int b = LO_B + lb;                 // global bit
#pragma unroll
      for (int j0 = 0; j0 < E; ++j0) {
        if (j0 & (1 << lb)) continue;
        const int j1 = j0 | (1 << lb);
        const uint64_t x = v[j0], y = v[j1];
        if (b == 0) {                          // every factor of the last/first stage is 1
          v[j0] = add_mod(x, y, P);
          v[j1] = sub_mod(x, y, P);
          continue;
        }
        const int jg = j0 >> NB, jl = j0 & ((1 << NB) - 1);
        const int F = t + jg * G::NT;
        const int lowF = F & ((1 << LO_B) - 1);
        const int e = lowF | ((jl & ((1 << lb) - 1)) << LO_B);     // idx mod 2^b
        const uint64_t w = tw[root_stage_offset(b) + e];
        if (DIT) {
          const uint64_t u = mont_mul(y, w, P);
          v[j0] = add_mod(x, u, P);
          v[j1] = sub_mod(x, u, P);
        } else {
          v[j0] = add_mod(x, y, P);
          v[j1] = mont_mul(sub_mod(x, y, P), w, P);
        }
      }
    }
  }

  static __device__ __forceinline__ void compute_lazy(uint64_t (&v)[G::E], const uint64_t* __restrict__ tw,
                                                      const Prime& P, int t) {
    constexpr int E = G::E;
    const uint64_t p2 = P.p << 1;
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int lb = DIT ? s : (NB - 1 - s);
      const int b = LO_B + lb;
#pragma unroll
      for (int j0 = 0; j0 < E; ++j0) {
        if (j0 & (1 << lb)) continue;
        const int j1 = j0 | (1 << lb);
        const uint64_t x = v[j0], y = v[j1];
        if (b == 0) {
          if (DIT) {                            // the first DIT stage: canonical inputs
            v[j0] = x + y;                      // [0, 2p)
            v[j1] = x - y + P.p;                // (0, 2p)
          } else {                              // [0, 2p) in and out
            v[j0] = cond_sub(x + y, p2);
            v[j1] = cond_sub(x - y + p2, p2);
          }
          continue;
        }
        const int jg = j0 >> NB, jl = j0 & ((1 << NB) - 1);
        const int F = t + jg * G::NT;
        const int lowF = F & ((1 << LO_B) - 1);
        const int e = lowF | ((jl & ((1 << lb) - 1)) << LO_B);     // idx mod 2^b
        const uint64_t w = tw[root_stage_offset(b) + e];
        if (DIT) {                              // [0, 4p) in and out
          const uint64_t xr = cond_sub(x, p2);  // [0, 2p)
          const uint64_t u = mont_mul_r(y, w, P);   // (0, 2p)
          v[j0] = xr + u;
          v[j1] = xr - u + p2;
        } else {                                // [0, 2p) in and out
          v[j0] = cond_sub(x + y, p2);
          v[j1] = mont_mul_r(x - y + p2, w, P);
        }
      }
    }
  }

  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t) {
    uint64_t v[G::E];
    load(lds, v, t);
    compute(v, tw, P, t);
    store(lds, v, t);
  }
};

// A transform's output in canonical range: DIF outputs lie in [0, 2p), DIT
// outputs in [0, 4p) with redundant ranges; unchanged otherwise.
template <bool DIT>
__device__ __forceinline__ uint64_t canonical(uint64_t x, const Prime& P) {
  if constexpr (!kLazy) return x;
  else return DIT ? reduce_4p(x, P) : reduce_2p(x, P);
}

// Synchronisation between the rounds of in-LDS transforms.  When every
// transform is owned by threads of one wavefront (NT <= 64, a power of two,
// so no transform straddles two wavefronts), the wavefront's own LDS writes
// need only be complete before it reads them back: a workgroup-scope fence
// (which waits for them) and a wavefront barrier order that, and the
// workgroup's wavefronts run their rounds without waiting for each other.
// Otherwise the workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void round_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// Rounds R, R+1, ... of a full transform; a round_sync follows every round.
template <int LOGL, int LOGE, bool DIT, int R, bool WAVE>
struct Rounds {
  using G = Geometry<LOGL, LOGE>;
  static constexpr int LO_B = DIT ? R * LOGE : (LOGL - (R + 1) * LOGE > 0 ? LOGL - (R + 1) * LOGE : 0);
  static constexpr int HI_B = DIT ? ((R + 1) * LOGE < LOGL ? (R + 1) * LOGE : LOGL) : LOGL - R * LOGE;
  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t, bool active) {
    if (active) Round<LOGL, LOGE, DIT, LO_B, HI_B - LO_B>::run(lds, tw, P, t);
    round_sync<WAVE>();
    Rounds<LOGL, LOGE, DIT, R + 1, WAVE>::run(lds, tw, P, t, active);
  }
};
template <int LOGL, int LOGE, bool DIT, bool WAVE>
struct Rounds<LOGL, LOGE, DIT, (LOGL + LOGE - 1) / LOGE, WAVE> {
  static __device__ __forceinline__ void run(uint64_t*, const uint64_t* __restrict__, const Prime&,
                                             int, bool) {}
};

// Bounds of round R of a DIF (top bits first) or DIT (bottom bits first) transform.
template <int LOGL, int LOGE, bool DIT, int R>
struct RoundBits {
  static constexpr int LO_B = Rounds<LOGL, LOGE, DIT, R, false>::LO_B;
  static constexpr int NB = Rounds<LOGL, LOGE, DIT, R, false>::HI_B - LO_B;
  using type = Round<LOGL, LOGE, DIT, LO_B, NB>;
};

// Rounds [R, END) through LDS, a round_sync after each.
template <int LOGL, int LOGE, bool DIT, int R, int END, bool WAVE>
struct RoundRange {
  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t) {
    if constexpr (R < END) {
      RoundBits<LOGL, LOGE, DIT, R>::type::run(lds, tw, P, t);
      round_sync<WAVE>();
      RoundRange<LOGL, LOGE, DIT, R + 1, END, WAVE>::run(lds, tw, P, t);
    }
  }
};

// DIF rounds over bits [0, TOP) of a 2^LOGL-point transform, top bits
// first, LOGE bits per round (the last may be shorter): the rest of a DIF
// whose stages on bits >= TOP were done elsewhere.  A round_sync follows
// every round.
template <int LOGL, int LOGE, int TOP, bool WAVE>
struct DifBelow {
  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t) {
    if constexpr (TOP > 0) {
      constexpr int LO = TOP > LOGE ? TOP - LOGE : 0;
      Round<LOGL, LOGE, false, LO, TOP - LO>::run(lds, tw, P, t);
      round_sync<WAVE>();
      DifBelow<LOGL, LOGE, LO, WAVE>::run(lds, tw, P, t);
    }
  }
};

// DIT rounds over bits [LO, TOP), bottom bits first, LOGE bits per round.
template <int LOGL, int LOGE, int LO, int TOP, bool WAVE>
struct DitFrom {
  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t) {
    if constexpr (LO < TOP) {
      constexpr int HI = LO + LOGE < TOP ? LO + LOGE : TOP;
      Round<LOGL, LOGE, true, LO, HI - LO>::run(lds, tw, P, t);
      round_sync<WAVE>();
      DitFrom<LOGL, LOGE, HI, TOP, WAVE>::run(lds, tw, P, t);
    }
  }
};

// In-LDS transform of 2^LOGL points (DIF natural->bit-reversed, or DIT
// bit-reversed->natural), run by the workgroup; `active` threads own a
// transform, the others only take part in the synchronisation.  With WAVE
// the caller synchronises the workgroup before other wavefronts read the
// result.
template <int LOGL, int LOGE, bool DIT, bool WAVE>
__device__ __forceinline__ void lds_transform(uint64_t* lds, const uint64_t* __restrict__ tw,
                                              const Prime& P, int t, bool active) {
  Rounds<LOGL, LOGE, DIT, 0, WAVE>::run(lds, tw, P, t, active);
}

// ---------------------------------------------------------------------------
// Digit-group split (Section 3.2 with B = 10^k): group g of an operand is
// decimal digits [k*g, k*g + k), taken from at most two adjacent base-10^19
// limbs by multiply-high division by powers of ten.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t div_pow10(uint64_t x, int e, const DivTable* __restrict__ dt) {
  if (e == 0) return x;
  return __umul64hi(x >> e, dt->mag[e]) >> dt->sh[e];
}

__device__ __forceinline__ uint64_t split_group(const uint64_t* __restrict__ limbs, uint64_t nl,
                                                uint64_t ng, uint64_t g, int k,
                                                const DivTable* __restrict__ dt, int* status) {
  if (g >= ng) return 0;
  const uint64_t d0 = g * (uint64_t)k;
  const uint64_t L = __umul64hi(d0, 0xD79435E50D79435FULL) >> 4;   // d0 / 19
  const int o = (int)(d0 - L * 19);
  const uint64_t lo = L < nl ? limbs[L] : 0;
  if (lo >= kLimbBase) atomicOr(status, 1);
  uint64_t x = div_pow10(lo, o, dt);                 // 19 - o digits
  const int have = 19 - o;
  if (have >= k) {
    x -= div_pow10(x, k, dt) * dt->pow10[k];         // keep k digits
  } else {
    const uint64_t hi = L + 1 < nl ? limbs[L + 1] : 0;
    if (hi >= kLimbBase) atomicOr(status, 1);
    const int need = k - have;
    const uint64_t top = hi - div_pow10(hi, need, dt) * dt->pow10[need];
    x += top * dt->pow10[have];
  }
  return x;
}

// split_group without the atomic: a limb >= 10^19 sets `bad` (reported once by the caller)
__device__ __forceinline__ uint64_t split_group_nf(const uint64_t* __restrict__ limbs, uint64_t nl,
                                                   uint64_t ng, uint64_t g, int k,
                                                   const DivTable* __restrict__ dt, int& bad) {
  if (g >= ng) return 0;
  const uint64_t d0 = g * (uint64_t)k;
  const uint64_t L = __umul64hi(d0, 0xD79435E50D79435FULL) >> 4;
  const int o = (int)(d0 - L * 19);
  const uint64_t lo = L < nl ? limbs[L] : 0;
  const uint64_t hi = L + 1 < nl ? limbs[L + 1] : 0;
  const int have = 19 - o;
  bad |= (lo >= kLimbBase) | (have < k && hi >= kLimbBase);
  uint64_t x = div_pow10(lo, o, dt);
  if (have >= k) {
    x -= div_pow10(x, k, dt) * dt->pow10[k];
  } else {
    const int need = k - have;
    const uint64_t top = hi - div_pow10(hi, need, dt) * dt->pow10[need];
    x += top * dt->pow10[have];
  }
  return x;
}

// dst[i] = src[i] for i < n (global memory to LDS), by the NTH threads of a
// workgroup with a compile-time stride, so a thread's loads are all issued
// before its first store (a loop striding by the runtime blockDim.x waits
// for each load in turn).
template <int NTH, int n, typename W>
__device__ __forceinline__ void stage_words(W* __restrict__ dst, const W* __restrict__ src) {
#pragma unroll
  for (int s = 0; s < (n + NTH - 1) / NTH; ++s) {
    const int i = (int)threadIdx.x + s * NTH;
    if (i < n) dst[i] = src[i];
  }
}

__device__ __forceinline__ uint32_t bitrev(uint32_t i, int bits) {
  return bits == 0 ? 0u : (__brev(i) >> (32 - bits));
}

// Inter-pass factor xi_N^(+-e) (times the inverse scale), e = e_hi*2^lb + e_lo.
// Exponents are below N <= 2^28 and fit 32 bits.
__device__ __forceinline__ uint64_t pass_factor(const uint64_t* __restrict__ hi,
                                                const uint64_t* __restrict__ lo, uint32_t e,
                                                int lb, const Prime& P) {
  const uint32_t L1 = (1u << lb) - 1;
  return mont_mul(hi[e >> lb], lo[e & L1], P);
}

// x / 2 mod p for x < p (p odd): x >> 1, or (x + p) / 2 for odd x.
__device__ __forceinline__ uint64_t half_mod(uint64_t x, const Prime& P) {
  return (x >> 1) + ((x & 1) ? (P.p >> 1) + 1 : 0);
}

// Length-3 DFT of (a, b, c) with the cube root of unity w of the direction
// (Section 7.8): y0 = a + b + c, y1 = a + w b + w^2 c, y2 = a + w^2 b + w c.
// Since 1 + w + w^2 = 0, y1 = m + v and y2 = m - v with m = a - (b + c)/2
// and v = kappa (b - c), kappa = (w - w^2)/2 held in Montgomery form: one
// REDC per three outputs.
__device__ __forceinline__ void dft3(uint64_t& a, uint64_t& b, uint64_t& c, uint64_t kappa,
                                     const Prime& P) {
  const uint64_t bc = add_mod(b, c, P);
  const uint64_t m = sub_mod(a, half_mod(bc, P), P);
  const uint64_t v = mont_mul(sub_mod(b, c, P), kappa, P);
  a = add_mod(a, bc, P);
  b = add_mod(m, v, P);
  c = sub_mod(m, v, P);
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  This bijection of [0, n) gives
// every XCD a contiguous range of tiles, so tiles that share cache lines
// (adjacent column tiles, whose rows meet inside 128-byte lines) meet in
// the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b % 8, i = b / 8, per = n / 8, rem = n % 8;
  return x * per + (x < rem ? x : rem) + i;
}

// The product a kernel works on: the launch's single descriptor, or entry
// blockIdx.z of the launch's descriptor array (a batch of products that
// share one transform length).
__device__ __forceinline__ ProdDesc load_desc(const Work& w) {
  return w.many ? w.many[blockIdx.z] : w.one;
}

}  // namespace dmi
