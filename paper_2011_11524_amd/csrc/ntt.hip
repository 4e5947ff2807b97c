// Number-theoretic transforms for the two-pass ("six-step" without its
// transpositions) layout of Section 7, on gfx950.
//
// A length-N transform, N = R*C (R = 2^logR rows, C = 2^logC columns,
// row-major, Section 7.9's split R = 2^floor(logN/2)), runs as
//   forward:  pass A  R-point DIF on every column, then x *= xi_N^(k1*n2)
//             pass B  C-point DIF on every row
//   inverse:  pass B  pointwise REDC(X, Y), C-point DIT on every row
//             pass A  x *= xi_N^(-k1*n2) * R^2 N^-1, R-point DIT on every column
// DIF leaves its outputs in bit-reversed order and DIT consumes that order,
// so no bit reversal and no transposition is ever done (Sections 5.4, 7.4);
// the pointwise product does not care about the order (eq.
// cdot_permutation_invariance).  Row k1 of the forward output is held at
// row position i = rev(k1), which is why the inter-pass factor uses rev(i).
//
// Inside a pass, one workgroup owns whole columns (pass A: a tile of T
// adjacent columns, so every global access is a T-word contiguous segment)
// or whole rows (pass B), staged in LDS.  Each thread keeps 2^LOGE points in
// registers and runs LOGE butterfly stages there (a radix-2^LOGE round),
// then the points are exchanged through LDS for the next round.
//
// All products are REDC (Section 4.4.3) against root tables kept in
// Montgomery form, so the transforms of plain residues come out plain
// (Section 6); the one factor R^-1 left by the pointwise REDC is cancelled,
// together with N^-1, by the scale R^2 N^-1 folded into the inverse
// inter-pass table (the linearity trick, Section 6, merged with the
// twiddle as Section 7.9 suggests).
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
// point is idx is w^((idx mod 2^b) * 2^(LOGL-1-b)) (Sections 5.2, 5.3, 5.5).
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

  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t) {
    constexpr int E = G::E;
    uint64_t v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = lds[lds_pos<LOGE>(index(t, j))];
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
        const int e = (lowF | ((jl & ((1 << lb) - 1)) << LO_B)) << (LOGL - 1 - b);
        const uint64_t w = tw[e];
        if (DIT) {
          const uint64_t u = mont_mul(y, w, P);
          v[j0] = add_mod(x, u, P);
          v[j1] = sub_mod(x, u, P);
        } else {
          v[j0] = add_mod(x, y, P);
          v[j1] = mont_mul(sub_lazy(x, y, P), w, P);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) lds[lds_pos<LOGE>(index(t, j))] = v[j];
  }
};

// Rounds R, R+1, ... of a full transform; a __syncthreads() separates rounds.
template <int LOGL, int LOGE, bool DIT, int R>
struct Rounds {
  using G = Geometry<LOGL, LOGE>;
  static constexpr int LO_B = DIT ? R * LOGE : (LOGL - (R + 1) * LOGE > 0 ? LOGL - (R + 1) * LOGE : 0);
  static constexpr int HI_B = DIT ? ((R + 1) * LOGE < LOGL ? (R + 1) * LOGE : LOGL) : LOGL - R * LOGE;
  static __device__ __forceinline__ void run(uint64_t* lds, const uint64_t* __restrict__ tw,
                                             const Prime& P, int t, bool active) {
    if (active) Round<LOGL, LOGE, DIT, LO_B, HI_B - LO_B>::run(lds, tw, P, t);
    __syncthreads();
    Rounds<LOGL, LOGE, DIT, R + 1>::run(lds, tw, P, t, active);
  }
};
template <int LOGL, int LOGE, bool DIT>
struct Rounds<LOGL, LOGE, DIT, (LOGL + LOGE - 1) / LOGE> {
  static __device__ __forceinline__ void run(uint64_t*, const uint64_t* __restrict__, const Prime&,
                                             int, bool) {}
};

// In-LDS transform of 2^LOGL points (DIF natural->bit-reversed, or DIT
// bit-reversed->natural), run by the workgroup; `active` threads own a
// transform, the others only take part in the barriers.
template <int LOGL, int LOGE, bool DIT>
__device__ __forceinline__ void lds_transform(uint64_t* lds, const uint64_t* __restrict__ tw,
                                              const Prime& P, int t, bool active) {
  Rounds<LOGL, LOGE, DIT, 0>::run(lds, tw, P, t, active);
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

__device__ __forceinline__ uint32_t bitrev(uint32_t i, int bits) {
  return bits == 0 ? 0u : (__brev(i) >> (32 - bits));
}

// Inter-pass factor xi_N^(+-e) (times the inverse scale), e = e_hi*C + e_lo.
__device__ __forceinline__ uint64_t pass_factor(const uint64_t* __restrict__ hi,
                                                const uint64_t* __restrict__ lo, uint64_t e,
                                                int logC, const Prime& P) {
  const uint64_t C1 = ((uint64_t)1 << logC) - 1;
  return mont_mul(hi[e >> logC], lo[e & C1], P);
}

// ---------------------------------------------------------------------------
// Pass A, forward: split + column DIF + inter-pass factor.
// grid.x = C / T column tiles, grid.y = 2 primes x (1 or 2) operands.
// ---------------------------------------------------------------------------
template <int LOGR, int LOGE, int T>
__global__ void __launch_bounds__((T * Geometry<LOGR, LOGE>::NT))
k_fwd_cols(PlanDev pl, Consts cs, TwiddleSet tw, const DivTable* __restrict__ dt,
           const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
           uint64_t* __restrict__ bufs, int* status) {
  using G = Geometry<LOGR, LOGE>;
  extern __shared__ uint64_t lds[];
  const int y = blockIdx.y;
  const int pi = y & 1, op = y >> 1;
  const Prime P = cs.P[pi];
  const uint64_t* src = op ? b : a;
  const uint64_t nl = op ? pl.nb : pl.na;
  const uint64_t ng = op ? pl.m : pl.n;
  uint64_t* dst = bufs + (size_t)y * pl.N;
  const uint64_t C = (uint64_t)1 << pl.logC;
  const uint64_t j0 = (uint64_t)blockIdx.x * T;
  constexpr int R = G::L;

  for (int q = threadIdx.x; q < R * T; q += blockDim.x) {
    const int row = q / T, col = q % T;
    uint64_t v = 0;
    if (j0 + col < C) v = split_group(src, nl, ng, (uint64_t)row * C + j0 + col, pl.k, dt, status);
    lds[col * G::STRIDE + lds_pos<LOGE>(row)] = v;
  }
  __syncthreads();
  const int col = threadIdx.x / G::NT, t = threadIdx.x % G::NT;
  lds_transform<LOGR, LOGE, false>(lds + col * G::STRIDE, tw.len_fwd[pi] + root_table_offset(LOGR),
                                   P, t, true);
  for (int q = threadIdx.x; q < R * T; q += blockDim.x) {
    const int row = q / T, c = q % T;
    if (j0 + c >= C) continue;
    const uint64_t e = (uint64_t)bitrev(row, LOGR) * (j0 + c);
    uint64_t v = lds[c * G::STRIDE + lds_pos<LOGE>(row)];
    v = mont_mul(v, pass_factor(tw.hi_fwd[pi], tw.lo_fwd[pi], e, pl.logC, P), P);
    dst[(uint64_t)row * C + j0 + c] = v;
  }
}

// ---------------------------------------------------------------------------
// Pass B: row transforms.  Forward: DIF in place on every row of every
// (operand, prime) buffer.  Inverse: pointwise REDC(X, Y) then DIT, written
// over X.
// ---------------------------------------------------------------------------
template <int LOGC, int LOGE, int RPW, bool INV>
__global__ void __launch_bounds__((RPW * Geometry<LOGC, LOGE>::NT))
k_rows(PlanDev pl, Consts cs, TwiddleSet tw, uint64_t* __restrict__ bufs, int square) {
  using G = Geometry<LOGC, LOGE>;
  extern __shared__ uint64_t lds[];
  constexpr int C = G::L;
  const int y = blockIdx.y;
  const int pi = y & 1;
  const Prime P = cs.P[pi];
  uint64_t* X = bufs + (size_t)y * pl.N;                       // inverse: y = prime
  const uint64_t* Y = bufs + (size_t)(square ? pi : 2 + pi) * pl.N;
  const uint64_t R = (uint64_t)1 << pl.logR;
  const uint64_t r0 = (uint64_t)blockIdx.x * RPW;

  for (int q = threadIdx.x; q < C * RPW; q += blockDim.x) {
    const int r = q / C, c = q % C;
    uint64_t v = 0;
    if (r0 + r < R) {
      const uint64_t gi = (r0 + r) * C + c;
      v = X[gi];
      if (INV) v = mont_mul(v, Y[gi], P);
    }
    lds[r * G::STRIDE + lds_pos<LOGE>(c)] = v;
  }
  __syncthreads();
  const int r = threadIdx.x / G::NT, t = threadIdx.x % G::NT;
  const uint64_t* roots = (INV ? tw.len_inv[pi] : tw.len_fwd[pi]) + root_table_offset(LOGC);
  lds_transform<LOGC, LOGE, INV>(lds + r * G::STRIDE, roots, P, t, true);
  for (int q = threadIdx.x; q < C * RPW; q += blockDim.x) {
    const int rr = q / C, c = q % C;
    if (r0 + rr < R) X[(r0 + rr) * C + c] = lds[rr * G::STRIDE + lds_pos<LOGE>(c)];
  }
}

// ---------------------------------------------------------------------------
// Pass A, inverse: inter-pass factor with scale, then column DIT; the
// result is the residue of each convolution coefficient, in natural order.
// ---------------------------------------------------------------------------
template <int LOGR, int LOGE, int T>
__global__ void __launch_bounds__((T * Geometry<LOGR, LOGE>::NT))
k_inv_cols(PlanDev pl, Consts cs, TwiddleSet tw, uint64_t* __restrict__ bufs) {
  using G = Geometry<LOGR, LOGE>;
  extern __shared__ uint64_t lds[];
  const int pi = blockIdx.y;
  const Prime P = cs.P[pi];
  uint64_t* X = bufs + (size_t)pi * pl.N;
  const uint64_t C = (uint64_t)1 << pl.logC;
  const uint64_t j0 = (uint64_t)blockIdx.x * T;
  constexpr int R = G::L;

  for (int q = threadIdx.x; q < R * T; q += blockDim.x) {
    const int row = q / T, c = q % T;
    uint64_t v = 0;
    if (j0 + c < C) {
      const uint64_t e = (uint64_t)bitrev(row, LOGR) * (j0 + c);
      v = X[(uint64_t)row * C + j0 + c];
      v = mont_mul(v, pass_factor(tw.hi_inv[pi], tw.lo_inv[pi], e, pl.logC, P), P);
    }
    lds[c * G::STRIDE + lds_pos<LOGE>(row)] = v;
  }
  __syncthreads();
  const int col = threadIdx.x / G::NT, t = threadIdx.x % G::NT;
  lds_transform<LOGR, LOGE, true>(lds + col * G::STRIDE, tw.len_inv[pi] + root_table_offset(LOGR),
                                  P, t, true);
  for (int q = threadIdx.x; q < R * T; q += blockDim.x) {
    const int row = q / T, c = q % T;
    if (j0 + c < C) X[(uint64_t)row * C + j0 + c] = lds[c * G::STRIDE + lds_pos<LOGE>(row)];
  }
}

// ---------------------------------------------------------------------------
// Launch configuration and dispatch over the compile-time lengths.
// ---------------------------------------------------------------------------
constexpr int loge_for(int logl) { return logl < 4 ? logl : 4; }
constexpr int cols_per_tile(int logl) {
  // about 512 threads per workgroup, at most 64 columns
  return (512 >> (logl - loge_for(logl))) < 1 ? 1
         : ((512 >> (logl - loge_for(logl))) > 64 ? 64 : (512 >> (logl - loge_for(logl))));
}
constexpr int rows_per_wg(int logl) {
  return (256 >> (logl - loge_for(logl))) < 1 ? 1 : (256 >> (logl - loge_for(logl)));
}

template <typename K>
static hipError_t prepare(K kernel, size_t lds_bytes) {
  if (lds_bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
  return hipSuccess;
}

template <int LOGR>
static hipError_t fwd_cols_l(const PlanDev& pl, const Consts& cs, const TwiddleSet& tw,
                             const DivTable* dt, const uint64_t* a, const uint64_t* b, bool square,
                             uint64_t* bufs, int* status, hipStream_t st) {
  constexpr int LOGE = loge_for(LOGR), T = cols_per_tile(LOGR);
  using G = Geometry<LOGR, LOGE>;
  const size_t lds = (size_t)T * G::STRIDE * sizeof(uint64_t);
  auto kern = k_fwd_cols<LOGR, LOGE, T>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint64_t C = (uint64_t)1 << pl.logC;
  dim3 grid((unsigned)((C + T - 1) / T), square ? 2 : 4);
  hipLaunchKernelGGL(kern, grid, dim3(T * G::NT), lds, st, pl, cs, tw, dt, a, b, bufs, status);
  return hipGetLastError();
}

template <int LOGC, bool INV>
static hipError_t rows_l(const PlanDev& pl, const Consts& cs, const TwiddleSet& tw, uint64_t* bufs,
                         bool square, hipStream_t st) {
  constexpr int LOGE = loge_for(LOGC), RPW = rows_per_wg(LOGC);
  using G = Geometry<LOGC, LOGE>;
  const size_t lds = (size_t)RPW * G::STRIDE * sizeof(uint64_t);
  auto kern = k_rows<LOGC, LOGE, RPW, INV>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint64_t R = (uint64_t)1 << pl.logR;
  const unsigned ny = INV ? 2 : (square ? 2 : 4);
  dim3 grid((unsigned)((R + RPW - 1) / RPW), ny);
  hipLaunchKernelGGL(kern, grid, dim3(RPW * G::NT), lds, st, pl, cs, tw, bufs, square ? 1 : 0);
  return hipGetLastError();
}

template <int LOGR>
static hipError_t inv_cols_l(const PlanDev& pl, const Consts& cs, const TwiddleSet& tw,
                             uint64_t* bufs, hipStream_t st) {
  constexpr int LOGE = loge_for(LOGR), T = cols_per_tile(LOGR);
  using G = Geometry<LOGR, LOGE>;
  const size_t lds = (size_t)T * G::STRIDE * sizeof(uint64_t);
  auto kern = k_inv_cols<LOGR, LOGE, T>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint64_t C = (uint64_t)1 << pl.logC;
  dim3 grid((unsigned)((C + T - 1) / T), 2);
  hipLaunchKernelGGL(kern, grid, dim3(T * G::NT), lds, st, pl, cs, tw, bufs);
  return hipGetLastError();
}

#define DMUL_LEN_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)

hipError_t launch_forward(const PlanDev& pl, const Consts& cs, const TwiddleSet& tw,
                          const DivTable* dt, const uint64_t* a, const uint64_t* b, bool square,
                          uint64_t* bufs, int* status, hipStream_t st, Marks* marks) {
  hipError_t e = hipErrorInvalidValue;
  switch (pl.logR) {
#define X(l) case l: e = fwd_cols_l<l>(pl, cs, tw, dt, a, b, square, bufs, status, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kFwdCols, st);
  switch (pl.logC) {
#define X(l) case l: e = rows_l<l, false>(pl, cs, tw, bufs, square, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess && marks) marks->mark(kFwdRows, st);
  return e;
}

hipError_t launch_inverse(const PlanDev& pl, const Consts& cs, const TwiddleSet& tw,
                          uint64_t* bufs, bool square, hipStream_t st, Marks* marks) {
  hipError_t e = hipErrorInvalidValue;
  switch (pl.logC) {
#define X(l) case l: e = rows_l<l, true>(pl, cs, tw, bufs, square, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kInvRows, st);
  switch (pl.logR) {
#define X(l) case l: e = inv_cols_l<l>(pl, cs, tw, bufs, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess && marks) marks->mark(kInvCols, st);
  return e;
}

}  // namespace dmi
