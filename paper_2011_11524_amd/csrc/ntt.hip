// Number-theoretic transforms for the two-pass ("six-step" without its
// transpositions) layout of Section 7, on gfx950.
//
// A length-N transform, N = R*C (R = 2^logR rows, C = 2^logC or 3*2^logC
// columns, row-major, Section 7.9's split R = 2^floor(logN/2)), runs as
//   forward:  pass A  R-point DIF on every column, then x *= xi_N^(k1*n2)
//             pass B  C-point DIF on every row
//   inverse:  pass B  pointwise REDC(X, Y), C-point DIT on every row
//             pass A  x *= xi_N^(-k1*n2) * R^2 N^-1, R-point DIT on every column
// The forward pass B, the pointwise product and the inverse pass B act on
// each row alone, so a product whose operands are both transformed here
// runs them as one kernel (k_rows_fused); the separate row kernels serve
// cached transforms (spectra), which must be stored between the two.
// DIF leaves its outputs in bit-reversed order and DIT consumes that order,
// so no bit reversal and no transposition is ever done (Sections 5.4, 7.4);
// a row of C = 3M points runs a length-3 DFT across its thirds first (DIF)
// or last (DIT) around three M-point transforms (Section 7.8);
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
#include "ntt_dev.hpp"

namespace dmi {

// LDS words a workgroup may use (160 KB per CU, less the static tables).
constexpr int kLdsWords = (160 * 1024 - 1024) / 8;
// Whether a workgroup holding `lines` transform lines of 2^LOGL points
// (LDS layout of LOGE) stages its `tables` per-stage root-table blocks of
// that length (2^LOGL - 1 words each) in LDS: where they fit, and where
// they would not cost the CU its second workgroup (lines that leave room
// for two workgroups without the tables, but only one with them).  Else
// the kernel reads its root tables from global memory (L2-resident, the
// same layout, so a stage's reads are contiguous there too): measured on
// the fused row pass, 4096-point rows run 12-14% faster that way (two
// workgroups per CU instead of one), 2048-point rows 12% slower (four
// instead of three).
template <int LOGL, int LOGE>
constexpr bool root_tables_fit(int lines, int tables) {
  const int data = lines * Geometry<LOGL, LOGE>::STRIDE;
  const int with = data + tables * ((1 << LOGL) - 1);
  return with <= kLdsWords && !(2 * data <= kLdsWords && 2 * with > kLdsWords);
}

// Rows of a column (or column triple) are dealt to its U threads as runs
// of consecutive rv: PB = R / U each, and one more for PX = R mod U of
// them.  The PX longer runs are spread evenly over the thread index (thread
// u has one iff floor((u+1) PX / U) > floor(u PX / U)), so that every
// wavefront, which a barrier then waits for, gets nearly the same share.

// ---------------------------------------------------------------------------
// Pass A tiles.  A tile is T column slots of the R x C matrix.  For C = 2^c
// they are the T adjacent columns j0 + l.  For C = 3M (R3) they are TS = T/3
// column triples: slot s*TS + l holds column s*M + q0 + l (s < 3), so the
// tile holds, for each row, the three points q, q+M, q+2M that the
// length-3 step of the row transform combines (Section 7.8).
// ---------------------------------------------------------------------------
template <int T, bool R3>
struct Tile {
  static constexpr int TS = R3 ? T / 3 : T;
  uint64_t first;     // j0 (C = 2^c) or q0 (C = 3M)
  uint64_t M, C;
  __device__ Tile(uint64_t blk, int logC, int rad3)
      : first(blk * TS), M((uint64_t)1 << logC), C(row_len(logC, rad3)) {}
  __device__ uint64_t column(int slot) const {
    return R3 ? (uint64_t)(slot / TS) * M + first + slot % TS : first + slot;
  }
  __device__ bool valid(int slot) const { return R3 ? first + slot % TS < M : first + slot < C; }
};

// ---------------------------------------------------------------------------
// Pass A, forward: split + column DIF + inter-pass factor (+ for C = 3M the
// length-3 DFT across the thirds of each row and the factor w_C^(s*q)).
// grid.x = column tiles, grid.y = operand, grid.z = product.  The digit
// groups of the tile are split once, kept in registers, and transformed for
// each prime in turn (the groups are below 10^k < p, the same residues for
// both primes).  The root tables of length R for both primes and the
// power-of-ten table are staged in LDS.
// ---------------------------------------------------------------------------
template <int LOGR, int LOGE, int T, bool R3>
__global__ void __launch_bounds__((T * Geometry<LOGR, LOGE>::NT))
k_fwd_cols(Work w, Consts cs, TwiddleSet tw, const DivTable* __restrict__ dt_g) {
  using G = Geometry<LOGR, LOGE>;
  constexpr int R = G::L;
  constexpr int NTH = T * G::NT;                 // threads
  constexpr int PER = R * T / NTH;               // tile points per thread (2^LOGE)
  constexpr int TS = Tile<T, R3>::TS;
  constexpr bool kWave = G::NT <= 64;            // each column within one wavefront
  // The DIF stage on the top bit pairs rows r and r + R/2, which are the
  // thread's points s and s + PER/2.  Where the rounds of LOGE bits would
  // leave a round of that bit alone, the stage is done as the tile is
  // written to LDS, and the rounds cover the bits below it.
  constexpr bool kTop = LOGR % LOGE == 1 && LOGR > 1;
  static_assert(PER * NTH == R * T, "a tile is whole rows of whole columns");
  extern __shared__ uint64_t lds[];
  constexpr bool kLdsTables = root_tables_fit<LOGR, LOGE>(T, 2);
  uint64_t* troots = lds + T * G::STRIDE;        // [prime][R - 1] when kLdsTables
  const ProdDesc d = load_desc(w);
  const int op = blockIdx.y;
  if (!transforms_operand(d, op)) return;         // squared product, or a cached spectrum
  const uint64_t* src = op ? d.b : d.a;
  const uint64_t nl = op ? d.pl.nb : d.pl.na;
  const uint64_t ng = op ? d.pl.m : d.pl.n;
  const uint64_t N = d.pl.N;
  const Tile<T, R3> tile(xcd_tile(blockIdx.x, gridDim.x), d.pl.logC, d.pl.rad3);
  const uint64_t C = tile.C;
  const int lb = pass_split_bits(d.pl.logC, d.pl.rad3);
  __shared__ DivTable sdt;
  stage_words<NTH, (int)(sizeof(DivTable) / 4)>(reinterpret_cast<uint32_t*>(&sdt),
                                                 reinterpret_cast<const uint32_t*>(dt_g));
  const DivTable* dt = &sdt;

  if constexpr (kLdsTables) {
    stage_words<NTH, R - 1>(troots, tw.len_fwd[0] + root_block_offset(LOGR));
    stage_words<NTH, R - 1>(troots + (R - 1), tw.len_fwd[1] + root_block_offset(LOGR));
  }
  __syncthreads();
  // the split tile, in registers for both primes: point s of the thread is
  // row threadIdx.x / T + s * NT of column slot threadIdx.x % T; every load
  // of the thread is issued before the divisions that use them
  uint64_t v[PER];
  {
    int bad = 0;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int q = threadIdx.x + s * NTH;
      const int row = q / T, sl = q % T;
      v[s] = tile.valid(sl) ? split_group_nf(src, nl, ng, (uint64_t)row * C + tile.column(sl), d.pl.k, dt, bad)
                            : 0;
    }
    if (bad) atomicOr(d.status, 1);
  }
  const int col = threadIdx.x / G::NT, t = threadIdx.x % G::NT;
#pragma unroll 1
  for (int pi = 0; pi < 2; ++pi) {
    const Prime P = cs.P[pi];
    const uint64_t* rts = kLdsTables ? troots + pi * (R - 1) : tw.len_fwd[pi] + root_block_offset(LOGR);
    uint64_t* dst = d.ws + (size_t)(2 * op + pi) * N;
    // the tile of this prime (the groups are below 10^k < p: the same
    // residues for both primes)
    if constexpr (kTop) {
#pragma unroll
      for (int s = 0; s < PER / 2; ++s) {
        const int q = threadIdx.x + s * NTH;
        const int row = q / T, sl = q % T;       // row < R/2; v[s + PER/2] is row + R/2
        const uint64_t a = v[s], b = v[s + PER / 2];
        lds[sl * G::STRIDE + lds_pos<LOGE>(row)] = add_mod(a, b, P);
        lds[sl * G::STRIDE + lds_pos<LOGE>(row + R / 2)] =
            mont_mul(sub_mod(a, b, P), rts[root_stage_offset(LOGR - 1) + row], P);
      }
    } else {
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int q = threadIdx.x + s * NTH;
        lds[(q % T) * G::STRIDE + lds_pos<LOGE>(q / T)] = v[s];
      }
    }
    __syncthreads();
    if constexpr (kTop) {
      DifBelow<LOGR, LOGE, LOGR - 1, kWave>::run(lds + col * G::STRIDE, rts, P, t);
    } else {
      lds_transform<LOGR, LOGE, false, kWave>(lds + col * G::STRIDE, rts, P, t, true);
    }
    if constexpr (kWave) __syncthreads();
    // Inter-pass factor xi_N^(rev(row) * j) for column j.  Each thread takes
    // one column (slot) and a run of consecutive rv = rev(row), so its
    // factors form a chain f(rv + 1) = f(rv) * xi^j: one table product to
    // start it, one Montgomery product per row after that.
    if constexpr (!R3) {
      constexpr int U = NTH / T;                 // threads per column
      constexpr int PB = R / U, PX = R % U;      // rows per thread: PB, or PB + 1 for PX spread ones
      const int c = threadIdx.x % T, u = threadIdx.x / T;
      const int v0 = u * PB + u * PX / U, v1 = v0 + PB + ((u + 1) * PX / U - u * PX / U);
      if (tile.valid(c) && v0 < v1) {
        const uint32_t j = (uint32_t)tile.column(c);
        const uint64_t step = tw.lo_fwd[pi][j];                       // xi^j, j < C <= 2^lb
        uint64_t f = pass_factor(tw.hi_fwd[pi], tw.lo_fwd[pi], (uint32_t)v0 * j, lb, P);   // < N
        // each row's LDS read is issued one row ahead of its product (the
        // split tile held for the second prime leaves no registers for more)
        auto rd = [&](int i) {
          return v0 + i < v1 ? lds[c * G::STRIDE + lds_pos<LOGE>((int)bitrev((uint32_t)(v0 + i), LOGR))] : 0;
        };
        uint64_t x = rd(0);
#pragma unroll 1
        for (int i = 0; v0 + i < v1; ++i) {
          const uint64_t nx = rd(i + 1);
          const uint32_t row = bitrev((uint32_t)(v0 + i), LOGR);
          dst[row * (uint32_t)C + j] = mont_mul(x, f, P);
          f = mont_mul(f, step, P);
          x = nx;
        }
      }
    } else {
      const uint64_t* w3 = tw.r3_fwd[pi] + r3_table_offset(d.pl.logC);
      const uint32_t M = (uint32_t)tile.M;
      constexpr int U = NTH / TS;                // threads per column triple
      constexpr int PB = R / U, PX = R % U;      // rows per thread: PB, or PB + 1 for PX spread ones
      const int c = threadIdx.x % TS, u = threadIdx.x / TS;
      const int v0 = u * PB + u * PX / U, v1 = v0 + PB + ((u + 1) * PX / U - u * PX / U);
      if (tile.valid(c) && v0 < v1) {
        const uint32_t qc = (uint32_t)tile.first + c;
        const uint64_t w31 = w3[qc], w32 = w3[2 * qc];
        uint64_t f[3], st[3];
#pragma unroll
        for (int sx = 0; sx < 3; ++sx) {
          const uint32_t j = qc + (uint32_t)sx * M;                  // < C = 3M < 2^lb
          st[sx] = tw.lo_fwd[pi][j];
          f[sx] = pass_factor(tw.hi_fwd[pi], tw.lo_fwd[pi], (uint32_t)v0 * j, lb, P);
        }
        // each row's LDS reads are issued one row ahead of its products (the
        // split tile held for the second prime leaves no registers for more)
        auto rd = [&](int i, uint64_t (&x)[3]) {
          const int o = lds_pos<LOGE>((int)bitrev((uint32_t)(v0 + i), LOGR));
#pragma unroll
          for (int sx = 0; sx < 3; ++sx) x[sx] = v0 + i < v1 ? lds[(sx * TS + c) * G::STRIDE + o] : 0;
        };
        const uint64_t kappa = cs.kappa[pi][0];
        uint64_t xc[3], xn[3];
        rd(0, xc);
#pragma unroll 1
        for (int i = 0; v0 + i < v1; ++i) {
          rd(i + 1, xn);
          {
            const uint32_t row = bitrev((uint32_t)(v0 + i), LOGR);
            uint64_t x0 = mont_mul(xc[0], f[0], P);
            uint64_t x1 = mont_mul(xc[1], f[1], P);
            uint64_t x2 = mont_mul(xc[2], f[2], P);
            dft3(x0, x1, x2, kappa, P);
            x1 = mont_mul(x1, w31, P);
            x2 = mont_mul(x2, w32, P);
            uint64_t* rowp = dst + (row * (uint32_t)C + qc);
            rowp[0] = x0;
            rowp[M] = x1;
            rowp[2 * M] = x2;
#pragma unroll
            for (int sx = 0; sx < 3; ++sx) f[sx] = mont_mul(f[sx], st[sx], P);
          }
#pragma unroll
          for (int sx = 0; sx < 3; ++sx) xc[sx] = xn[sx];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pass B: row transforms.  Forward: DIF in place on every row of every
// (operand, prime) buffer.  Inverse: pointwise REDC(X, Y) then DIT, written
// over X.  With C = 3M the rows are the 3R sub-rows of M points (the
// length-3 step across each row's thirds is done by the column passes), so
// a "row" here is always 2^LOGC contiguous points.
//
// grid.y selects the buffer (forward: prime + 2*operand; inverse: prime),
// grid.z the product; the workgroups along x loop over groups of RPW rows
// of that buffer.  A thread holds points t + j*NT of its row (j < E): that
// is the coalesced layout of the global loads, the first DIF round (top
// bits) runs on it without an LDS round trip, and the last DIT round ends
// in it and is stored straight to global memory.  With TWL the row
// length's root table is staged in LDS once per workgroup.
// ---------------------------------------------------------------------------
template <int LOGC, int LOGE, int RPW, bool INV, bool TWL>
__global__ void __launch_bounds__((RPW * Geometry<LOGC, LOGE>::NT))
k_rows(Work w, Consts cs, TwiddleSet tw) {
  using G = Geometry<LOGC, LOGE>;
  constexpr int C = G::L, E = G::E, NT = G::NT;
  constexpr int NR = G::ROUNDS;
  constexpr bool kWave = NT <= 64;               // each row within one wavefront
  extern __shared__ uint64_t lds[];
  const ProdDesc d = load_desc(w);
  const int y = blockIdx.y;
  if (!INV && !transforms_operand(d, y >> 1)) return;
  const int pi = y & 1;
  const Prime P = cs.P[pi];
  uint64_t* X = d.ws + (size_t)y * d.pl.N;                       // inverse: y = prime
  // inverse: the two spectra, from the workspace or from cached transforms
  const uint64_t* Xs = d.xs ? d.xs + (size_t)pi * d.pl.N : X;
  const uint64_t* Y = d.square ? Xs : (d.ys ? d.ys + (size_t)pi * d.pl.N : d.ws + (size_t)(2 + pi) * d.pl.N);
  const uint64_t R = (uint64_t)(d.pl.rad3 ? 3 : 1) << d.pl.logR;  // rows of C points
  const uint32_t groups = (uint32_t)((R + RPW - 1) / RPW);
  const int r = threadIdx.x / NT, t = threadIdx.x % NT;
  uint64_t* row_lds = lds + r * G::STRIDE;

  const uint64_t* roots_g = (INV ? tw.len_inv[pi] : tw.len_fwd[pi]) + root_block_offset(LOGC);
  const uint64_t* roots = roots_g;
  if constexpr (TWL) {
    uint64_t* tl = lds + RPW * G::STRIDE;
    stage_words<RPW * NT, C - 1>(tl, roots_g);
    roots = tl;
    __syncthreads();
  }

  uint64_t cur[E];
  for (uint32_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const uint64_t row = (uint64_t)g * RPW + r;
    if (row < R) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (INV) cur[j] = mont_mul(Xs[row * C + t + j * NT], Y[row * C + t + j * NT], P);
        else cur[j] = X[row * C + t + j * NT];
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) cur[j] = 0;
    }
    if constexpr (!INV) {
      // round 0 (top bits) straight from the loaded registers
      using R0 = typename RoundBits<LOGC, LOGE, false, 0>::type;
      R0::compute(cur, roots, P, t);
      R0::store(row_lds, cur, t);
      round_sync<kWave>();
      RoundRange<LOGC, LOGE, false, 1, NR, kWave>::run(row_lds, roots, P, t);
      // points back to the coalesced layout
#pragma unroll
      for (int j = 0; j < E; ++j) cur[j] = row_lds[lds_pos<LOGE>(t + j * NT)];
      if (row < R) {
#pragma unroll
        for (int j = 0; j < E; ++j) X[row * C + t + j * NT] = canonical<false>(cur[j], P);
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) row_lds[lds_pos<LOGE>(t + j * NT)] = cur[j];
      round_sync<kWave>();
      RoundRange<LOGC, LOGE, true, 0, NR - 1, kWave>::run(row_lds, roots, P, t);
      // last round (top bits) ends in the coalesced layout
      using RL = typename RoundBits<LOGC, LOGE, true, NR - 1>::type;
      RL::load(row_lds, cur, t);
      RL::compute(cur, roots, P, t);
      if (row < R) {
#pragma unroll
        for (int j = 0; j < E; ++j) X[row * C + RL::index(t, j)] = canonical<true>(cur[j], P);
      }
    }
    round_sync<kWave>();   // the next group reuses the LDS rows
  }
}

// ---------------------------------------------------------------------------
// Pass B in both directions at once, for products whose operands are both
// transformed here (no cached spectra): once the forward column pass is
// done, each row's forward DIF, its pointwise REDC product and its inverse
// DIT involve that row alone (Section 7.4), so one workgroup takes a row
// through all three and the forward spectra never go back to HBM.  X's
// spectrum waits in registers, as the points t + j*NT that the inverse
// starts from, while Y's goes through the same LDS row; the product is
// formed in LDS and the inverse rounds run on it.  Rows beyond R are
// computed on zeros and not stored.  grid.y = prime, grid.z = product.
// ---------------------------------------------------------------------------
template <int LOGC, int LOGE, int RPW>
__global__ void __launch_bounds__((RPW * Geometry<LOGC, LOGE>::NT), (LOGE == 3 ? 4 : 1))
k_rows_fused(Work w, Consts cs, TwiddleSet tw) {
  using G = Geometry<LOGC, LOGE>;
  constexpr int C = G::L, E = G::E, NT = G::NT;
  constexpr int NR = G::ROUNDS;
  constexpr bool kWave = NT <= 64;               // each row within one wavefront
  extern __shared__ uint64_t lds[];
  const ProdDesc d = load_desc(w);
  const int pi = blockIdx.y;
  const Prime P = cs.P[pi];
  uint64_t* X = d.ws + (size_t)pi * d.pl.N;
  const uint64_t* Y = d.ws + (size_t)(2 + pi) * d.pl.N;
  const bool square = d.square != 0;
  const uint64_t R = (uint64_t)(d.pl.rad3 ? 3 : 1) << d.pl.logR;  // rows of C points
  const uint32_t groups = (uint32_t)((R + RPW - 1) / RPW);
  const int r = threadIdx.x / NT, t = threadIdx.x % NT;
  uint64_t* row_lds = lds + r * G::STRIDE;
  // forward and inverse roots of the row length, staged in LDS where they fit
  constexpr bool kLdsTables = root_tables_fit<LOGC, LOGE>(RPW, 2);
  const uint64_t* rf = tw.len_fwd[pi] + root_block_offset(LOGC);
  const uint64_t* ri = tw.len_inv[pi] + root_block_offset(LOGC);
  if constexpr (kLdsTables) {
    uint64_t* lf = lds + RPW * G::STRIDE;
    uint64_t* li = lf + (C - 1);
    stage_words<RPW * NT, C - 1>(lf, rf);
    stage_words<RPW * NT, C - 1>(li, ri);
    rf = lf;
    ri = li;
  }
  __syncthreads();

  using R0 = typename RoundBits<LOGC, LOGE, false, 0>::type;
  using RL = typename RoundBits<LOGC, LOGE, true, NR - 1>::type;
  // With two or more rounds, the forward DIF's last round (the low bits)
  // and the inverse DIT's first round (bits [0, LOGE)) both act within runs
  // of 2^LOGE consecutive points: a thread loads its run once (the DIT's
  // first-round layout), finishes the DIF there, forms the pointwise product
  // and runs the DIT's first round, all in registers.
  using DL = typename RoundBits<LOGC, LOGE, false, NR - 1>::type;   // the DIF's last round
  using D0 = typename RoundBits<LOGC, LOGE, true, 0>::type;         // the DIT's first round
  constexpr bool kJoin = NR >= 2;
  uint64_t cur[E], xs[E];
  for (uint32_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const uint64_t row = (uint64_t)g * RPW + r;
    const bool in = row < R;
    if constexpr (kJoin) {
      // forward DIF of X's row: round 0 on the loaded registers, the middle
      // rounds in LDS, the last on the thread's run of consecutive points
#pragma unroll
      for (int j = 0; j < E; ++j) cur[j] = in ? X[row * C + t + j * NT] : 0;
      R0::compute(cur, rf, P, t);
      R0::store(row_lds, cur, t);
      round_sync<kWave>();
      RoundRange<LOGC, LOGE, false, 1, NR - 1, kWave>::run(row_lds, rf, P, t);
      D0::load(row_lds, xs, t);
      DL::compute(xs, rf, P, t);
      if (!square) {
        round_sync<kWave>();                     // X's run read before Y's overwrites the row
#pragma unroll
        for (int j = 0; j < E; ++j) cur[j] = in ? Y[row * C + t + j * NT] : 0;
        R0::compute(cur, rf, P, t);
        R0::store(row_lds, cur, t);
        round_sync<kWave>();
        RoundRange<LOGC, LOGE, false, 1, NR - 1, kWave>::run(row_lds, rf, P, t);
        D0::load(row_lds, cur, t);
        DL::compute(cur, rf, P, t);
      }
#pragma unroll
      for (int j = 0; j < E; ++j) cur[j] = mont_mul(xs[j], square ? xs[j] : cur[j], P);
      D0::compute(cur, ri, P, t);
      round_sync<kWave>();                       // every run read before the product overwrites the row
      D0::store(row_lds, cur, t);
      round_sync<kWave>();
      RoundRange<LOGC, LOGE, true, 1, NR - 1, kWave>::run(row_lds, ri, P, t);
    } else {
      // forward DIF of X's row: round 0 on the loaded registers, the rest in LDS
#pragma unroll
      for (int j = 0; j < E; ++j) cur[j] = in ? X[row * C + t + j * NT] : 0;
      R0::compute(cur, rf, P, t);
      R0::store(row_lds, cur, t);
      round_sync<kWave>();
      RoundRange<LOGC, LOGE, false, 1, NR, kWave>::run(row_lds, rf, P, t);
#pragma unroll
      for (int j = 0; j < E; ++j) xs[j] = row_lds[lds_pos<LOGE>(t + j * NT)];
      if (square) {
#pragma unroll
        for (int j = 0; j < E; ++j) row_lds[lds_pos<LOGE>(t + j * NT)] = mont_mul(xs[j], xs[j], P);
      } else {
        round_sync<kWave>();                     // X's spectrum read before Y's overwrites the row
#pragma unroll
        for (int j = 0; j < E; ++j) cur[j] = in ? Y[row * C + t + j * NT] : 0;
        R0::compute(cur, rf, P, t);
        R0::store(row_lds, cur, t);
        round_sync<kWave>();
        RoundRange<LOGC, LOGE, false, 1, NR, kWave>::run(row_lds, rf, P, t);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int o = lds_pos<LOGE>(t + j * NT);
          row_lds[o] = mont_mul(xs[j], row_lds[o], P);
        }
      }
      round_sync<kWave>();
      // inverse DIT: all rounds but the last in LDS, the last ends in registers
      RoundRange<LOGC, LOGE, true, 0, NR - 1, kWave>::run(row_lds, ri, P, t);
    }
    RL::load(row_lds, cur, t);
    RL::compute(cur, ri, P, t);
    if (in) {
#pragma unroll
      for (int j = 0; j < E; ++j) X[row * C + RL::index(t, j)] = canonical<true>(cur[j], P);
    }
    round_sync<kWave>();   // the next group reuses the LDS rows
  }
}

// ---------------------------------------------------------------------------
// Pass A, inverse: (for C = 3M first the factor w_C^(-s*q) and the inverse
// length-3 DFT across the thirds of each row, completing the row
// transform), inter-pass factor with scale, then column DIT; the result is
// the residue of each convolution coefficient, in natural order.
// grid.x = column tiles, grid.y = prime, grid.z = product.
// ---------------------------------------------------------------------------
template <int LOGR, int LOGE, int T, bool R3>
__global__ void __launch_bounds__((T * Geometry<LOGR, LOGE>::NT))
k_inv_cols(Work w, Consts cs, TwiddleSet tw) {
  using G = Geometry<LOGR, LOGE>;
  constexpr int TS = Tile<T, R3>::TS;
  constexpr int NTH = T * G::NT;
  constexpr bool kWave = G::NT <= 64;            // each column within one wavefront
  // DIT rounds go bottom bit up; where the rounds of LOGE bits would leave
  // the top bit alone, its stage (rows r and r + R/2) is done as the tile is
  // stored to global memory.
  constexpr bool kTop = LOGR % LOGE == 1 && LOGR > 1;
  extern __shared__ uint64_t lds[];
  constexpr bool kLdsTables = root_tables_fit<LOGR, LOGE>(T, 1);
  const ProdDesc d = load_desc(w);
  const int pi = blockIdx.y;
  uint64_t* const troots_l = lds + T * G::STRIDE;
  const uint64_t* const troots = kLdsTables ? troots_l : tw.len_inv[pi] + root_block_offset(LOGR);
  const Prime P = cs.P[pi];
  uint64_t* X = d.ws + (size_t)pi * d.pl.N;
  const Tile<T, R3> tile(xcd_tile(blockIdx.x, gridDim.x), d.pl.logC, d.pl.rad3);
  const uint64_t C = tile.C;
  const uint32_t N = (uint32_t)d.pl.N;
  const int lb = pass_split_bits(d.pl.logC, d.pl.rad3);
  constexpr int R = G::L;

  if constexpr (kLdsTables) stage_words<NTH, R - 1>(troots_l, tw.len_inv[pi] + root_block_offset(LOGR));
  // Inter-pass factor with the scale, xi_N^(-rev(row) * j) * R^2 N^-1: per
  // thread one column (slot) and a run of consecutive rv = rev(row), the
  // factors a chain f(rv + 1) = f(rv) * xi^-j (xi^-j = xi^(N - j)).
  auto step_inv = [&](uint32_t j) {
    return j ? pass_factor(tw.hi_fwd[pi], tw.lo_fwd[pi], N - j, lb, P) : tw.lo_fwd[pi][0];
  };
  // Every global load of the thread (its rows, and the factor tables that
  // start its chain) is issued before the first product that uses one:
  // the rows are at most PMAX, so they live in registers, and a thread
  // waits for HBM once instead of once per row.
  if constexpr (!R3) {
    constexpr int U = NTH / T;
    constexpr int PB = R / U, PX = R % U;        // rows per thread: PB, or PB + 1 for PX spread ones
    constexpr int PMAX = PB + (PX ? 1 : 0);
    const int c = threadIdx.x % T, u = threadIdx.x / T;
    const int v0 = u * PB + u * PX / U, v1 = v0 + PB + ((u + 1) * PX / U - u * PX / U);
    const uint32_t j = (uint32_t)tile.column(c);
    const bool ok = tile.valid(c);
    uint64_t f = 0, st = 0;
    if (ok && v0 < v1) {
      st = step_inv(j);
      f = pass_factor(tw.hi_inv[pi], tw.lo_inv[pi], (uint32_t)v0 * j, lb, P);
    }
    uint64_t xr[PMAX];
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int rv = v0 + i;
      xr[i] = ok && rv < v1 ? X[bitrev((uint32_t)rv, LOGR) * (uint32_t)C + j] : 0;
    }
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int rv = v0 + i;
      if (rv < v1) {
        const uint32_t row = bitrev((uint32_t)rv, LOGR);
        uint64_t x = 0;
        if (ok) {
          x = mont_mul(xr[i], f, P);
          f = mont_mul(f, st, P);
        }
        lds[c * G::STRIDE + lds_pos<LOGE>((int)row)] = x;
      }
    }
  } else {
    const uint64_t* w3 = tw.r3_inv[pi] + r3_table_offset(d.pl.logC);
    const uint32_t M = (uint32_t)tile.M;
    constexpr int U = NTH / TS;
    constexpr int PB = R / U, PX = R % U;        // rows per thread: PB, or PB + 1 for PX spread ones
    constexpr int PMAX = PB + (PX ? 1 : 0);
    const int c = threadIdx.x % TS, u = threadIdx.x / TS;
    const int v0 = u * PB + u * PX / U, v1 = v0 + PB + ((u + 1) * PX / U - u * PX / U);
    const bool ok = tile.valid(c);
    const uint32_t qc = (uint32_t)tile.first + c;
    const uint64_t kappa = cs.kappa[pi][1];
    uint64_t w31 = 0, w32 = 0, f[3] = {0, 0, 0}, st[3] = {0, 0, 0};
    if (ok && v0 < v1) {
      w31 = w3[qc];
      w32 = w3[2 * qc];
#pragma unroll
      for (int sx = 0; sx < 3; ++sx) {
        const uint32_t j = qc + (uint32_t)sx * M;
        st[sx] = step_inv(j);
        f[sx] = pass_factor(tw.hi_inv[pi], tw.lo_inv[pi], (uint32_t)v0 * j, lb, P);
      }
    }
    uint64_t xr[PMAX][3];
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int rv = v0 + i;
      const bool in = ok && rv < v1;
      const uint64_t* rowp = X + (bitrev((uint32_t)rv, LOGR) * (uint32_t)C + qc);
#pragma unroll
      for (int sx = 0; sx < 3; ++sx) xr[i][sx] = in ? rowp[sx * M] : 0;
    }
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int rv = v0 + i;
      if (rv < v1) {
        const uint32_t row = bitrev((uint32_t)rv, LOGR);
        const int o = lds_pos<LOGE>((int)row);
        uint64_t x0 = 0, x1 = 0, x2 = 0;
        if (ok) {
          x0 = xr[i][0];
          x1 = mont_mul(xr[i][1], w31, P);
          x2 = mont_mul(xr[i][2], w32, P);
          dft3(x0, x1, x2, kappa, P);
          x0 = mont_mul(x0, f[0], P);
          x1 = mont_mul(x1, f[1], P);
          x2 = mont_mul(x2, f[2], P);
#pragma unroll
          for (int sx = 0; sx < 3; ++sx) f[sx] = mont_mul(f[sx], st[sx], P);
        }
        lds[c * G::STRIDE + o] = x0;
        lds[(TS + c) * G::STRIDE + o] = x1;
        lds[(2 * TS + c) * G::STRIDE + o] = x2;
      }
    }
  }
  __syncthreads();
  const int col = threadIdx.x / G::NT, t = threadIdx.x % G::NT;
  if constexpr (kTop) {
    DitFrom<LOGR, LOGE, 0, LOGR - 1, kWave>::run(lds + col * G::STRIDE, troots, P, t);
    if constexpr (kWave) __syncthreads();
    // a compile-time count of tile positions per thread: the LDS reads of
    // all of them are issued before the first product
    static_assert((R / 2) * T % NTH == 0, "whole rows of the tile per thread");
#pragma unroll
    for (int s = 0; s < (R / 2) * T / NTH; ++s) {
      const int q = threadIdx.x + s * NTH;
      const int row = q / T, c = q % T;
      if (tile.valid(c)) {
        const uint64_t x = canonical<true>(lds[c * G::STRIDE + lds_pos<LOGE>(row)], P);
        const uint64_t y = mont_mul(canonical<true>(lds[c * G::STRIDE + lds_pos<LOGE>(row + R / 2)], P),
                                    troots[root_stage_offset(LOGR - 1) + row], P);
        const uint32_t j = (uint32_t)tile.column(c);
        X[(uint32_t)row * (uint32_t)C + j] = add_mod(x, y, P);
        X[(uint32_t)(row + R / 2) * (uint32_t)C + j] = sub_mod(x, y, P);
      }
    }
  } else {
    lds_transform<LOGR, LOGE, true, kWave>(lds + col * G::STRIDE, troots, P, t, true);
    if constexpr (kWave) __syncthreads();
    static_assert(R * T % NTH == 0, "whole rows of the tile per thread");
#pragma unroll
    for (int s = 0; s < R * T / NTH; ++s) {
      const int q = threadIdx.x + s * NTH;
      const int row = q / T, c = q % T;
      if (tile.valid(c))
        X[(uint32_t)row * (uint32_t)C + (uint32_t)tile.column(c)] =
            canonical<true>(lds[c * G::STRIDE + lds_pos<LOGE>(row)], P);
    }
  }
}

// ---------------------------------------------------------------------------
// Launch configuration and dispatch over the compile-time lengths.
// ---------------------------------------------------------------------------
constexpr int loge_for(int logl) { return logl < 4 ? logl : 4; }
// Points per thread (log2) in the column passes.
constexpr int col_loge(int logl) { return loge_for(logl); }
// Launches too small to give every CU a workgroup (a lone short product)
// take a lean configuration for transforms of up to 2^kLeanMaxLog points:
// 4 points per thread, so the same transform runs on four times the
// threads in a quarter of the per-thread chain, and narrower tiles (more
// workgroups).  A 10^5-digit product (N = 3*2^12) runs 0.065 -> 0.045 ms
// with the 4 points per thread, 0.034 ms with the narrower tiles as well,
// a 10^6-digit one (N = 3*2^16) 0.075 -> 0.041 ms; in the batched
// workload, whose launches are large, 4 points per thread cost 2%, so
// those keep 16.
constexpr int kLeanMaxLog = 9;
constexpr int lean_loge(int logl) { return logl < 2 ? logl : 2; }
constexpr int kLeanMinGroups = 256;   // one workgroup per CU
constexpr int col_stride(int logl, int loge) { return (1 << logl) + ((1 << logl) >> loge) + 1; }
// Column tiles: as many columns as fit a target workgroup size (at most 64)
// and the LDS next to `extra` words (one per point for the forward pass,
// half a word for the inverse).  Wide tiles matter: every global access of
// a column pass is a run of T contiguous words of one row, and runs below
// a 128-byte line waste HBM transactions.  The per-stage root tables take
// the LDS beside the tile where they fit (root_tables_fit) and are read
// from global memory otherwise, so they never narrow a tile.
constexpr int cols_for(int logl, int loge, int threads, int extra) {
  int t = 1;
  while (t < 64 && 2 * t * (1 << (logl - loge)) <= threads && 2 * t * col_stride(logl, loge) + extra <= kLdsWords)
    t *= 2;
  return t;
}
// Column triples per tile (C = 3M): the largest power of two, 1..16, within
// the thread target and the LDS.
constexpr int triples_for(int logl, int loge, int threads, int extra) {
  int t = 1;
  while (t < 16 && 2 * t * 3 * (1 << (logl - loge)) <= threads &&
         2 * t * 3 * col_stride(logl, loge) + extra <= kLdsWords)
    t *= 2;
  return t;
}
// Forward tiles (whose kernel also keeps the split tile in registers) aim at
// 512 threads, 768 with column triples; inverse tiles at 1024.  Columns of
// 2048 points and more would get only 4-column tiles (32-byte row runs) at
// 512 threads: there the forward tile takes 1024 threads and 8 columns,
// whose register cap of 128 costs a small spill but took C3's forward
// column pass from 198 to 173 us.
// Lean launches aim at a quarter of these thread targets: narrower tiles,
// four times the workgroups (C1's column passes 8 -> 32 tiles per operand
// or prime; 0.042 -> 0.034 ms).
constexpr int lean_div(int logl, int loge) {
  return logl <= kLeanMaxLog && loge == lean_loge(logl) && loge != col_loge(logl) ? 4 : 1;
}
constexpr int fwd_cols_per_tile(int logl, int loge) {
  return cols_for(logl, loge, (logl >= 11 ? 1024 : 512) / lean_div(logl, loge), 1 << logl);
}
constexpr int cols_per_tile(int logl, int loge) {
  return cols_for(logl, loge, 1024 / lean_div(logl, loge), (1 << logl) / 2);
}
constexpr int fwd_triples_per_tile(int logl, int loge) {
  return triples_for(logl, loge, 768 / lean_div(logl, loge), 1 << logl);
}
constexpr int triples_per_tile(int logl, int loge) {
  return triples_for(logl, loge, 1024 / lean_div(logl, loge), (1 << logl) / 2);
}
constexpr uint64_t kRowMinGroups = 1024;
// Points per thread (log2) and rows per workgroup in the row passes.
constexpr int row_loge(int logl) { return loge_for(logl); }
constexpr int kRowThreads = 256;
constexpr int rows_per_wg(int logl) {
  return (kRowThreads >> (logl - row_loge(logl))) < 1 ? 1 : (kRowThreads >> (logl - row_loge(logl)));
}

template <typename K>
static hipError_t prepare(K kernel, size_t lds_bytes) {
  return allow_lds((const void*)kernel, lds_bytes);
}

// Column tiles (slots per tile) and workgroups of a column-pass launch.
template <int LOGR, int LOGE, bool R3, bool FWD>
struct ColLaunch {
  static constexpr int T = R3 ? 3 * (FWD ? fwd_triples_per_tile(LOGR, LOGE) : triples_per_tile(LOGR, LOGE))
                              : (FWD ? fwd_cols_per_tile(LOGR, LOGE) : cols_per_tile(LOGR, LOGE));
  static constexpr int TS = R3 ? T / 3 : T;
  static uint64_t tiles(const Shape& sh) {
    const uint64_t span = R3 ? (uint64_t)1 << sh.logC : row_len(sh.logC, 0);   // tiles cover M or C
    return (span + TS - 1) / TS;
  }
};

template <int LOGR, int LOGE, bool R3>
static hipError_t fwd_cols_launch(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                                  const DivTable* dt, hipStream_t st) {
  constexpr int T = ColLaunch<LOGR, LOGE, R3, true>::T;
  using G = Geometry<LOGR, LOGE>;
  const size_t tables = root_tables_fit<LOGR, LOGE>(T, 2) ? 2 * ((size_t)G::L - 1) : 0;
  const size_t lds = ((size_t)T * G::STRIDE + tables) * sizeof(uint64_t);
  auto kern = k_fwd_cols<LOGR, LOGE, T, R3>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)ColLaunch<LOGR, LOGE, R3, true>::tiles(sh), sh.any_nonsquare ? 2 : 1, w.count);
  hipLaunchKernelGGL(kern, grid, dim3(T * G::NT), lds, st, w, cs, tw, dt);
  return hipGetLastError();
}

// The default configuration, or the lean one where the default launch
// would leave CUs without a workgroup.
template <int LOGR, bool R3>
static hipError_t fwd_cols_pick(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                                const DivTable* dt, hipStream_t st) {
  constexpr int LOGE = col_loge(LOGR);
  if constexpr (LOGR <= kLeanMaxLog && lean_loge(LOGR) != LOGE) {
    const uint64_t wgs = ColLaunch<LOGR, LOGE, R3, true>::tiles(sh) * (sh.any_nonsquare ? 2 : 1) * w.count;
    if (wgs < kLeanMinGroups) return fwd_cols_launch<LOGR, lean_loge(LOGR), R3>(w, sh, cs, tw, dt, st);
  }
  return fwd_cols_launch<LOGR, LOGE, R3>(w, sh, cs, tw, dt, st);
}

template <int LOGR>
static hipError_t fwd_cols_l(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                             const DivTable* dt, hipStream_t st) {
  if constexpr (LOGR <= kMaxLogR3) {
    if (sh.rad3) return fwd_cols_pick<LOGR, true>(w, sh, cs, tw, dt, st);
  } else {
    if (sh.rad3) return hipErrorInvalidValue;
  }
  return fwd_cols_pick<LOGR, false>(w, sh, cs, tw, dt, st);
}

template <int LOGC, bool INV>
static hipError_t rows_l(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                         hipStream_t st) {
  constexpr int LOGE = row_loge(LOGC), RPW = rows_per_wg(LOGC);
  using G = Geometry<LOGC, LOGE>;
  constexpr bool TWL = root_tables_fit<LOGC, LOGE>(RPW, 1);
  const size_t lds = ((size_t)RPW * G::STRIDE + (TWL ? (size_t)G::L - 1 : 0)) * sizeof(uint64_t);
  auto kern = k_rows<LOGC, LOGE, RPW, INV, TWL>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint64_t R = (uint64_t)(sh.rad3 ? 3 : 1) << sh.logR;    // rows of 2^logC points
  const uint64_t groups = (R + RPW - 1) / RPW;
  const unsigned ny = INV ? 2 : (sh.any_nonsquare ? 4 : 2);
  // the tuned loop count, but never so long that the launch has fewer than
  // about four workgroups per CU
  const uint64_t cap = groups * ny * w.count / kRowMinGroups;
  int iters = sh.row_iters > 0 ? sh.row_iters : 1;
  if ((uint64_t)iters > cap) iters = cap > 1 ? (int)cap : 1;
  const unsigned gx = (unsigned)((groups + iters - 1) / iters);
  hipLaunchKernelGGL(kern, dim3(gx, ny, w.count), dim3(RPW * G::NT), lds, st, w, cs, tw);
  return hipGetLastError();
}

// Fused rows: 16 points per thread up to rows of 2^8 points; from 2^9 on,
// 8, with at most 128 registers (four wavefronts per SIMD).  X's spectrum
// is held in registers across Y's transform, and with 16 points per thread
// the long rows need about 170 registers (two wavefronts per SIMD): the
// fused pass of C2's 1024-point rows took 60 us that way, 52 us this way.
constexpr int fused_loge(int logl) { return logl <= 8 ? loge_for(logl) : 3; }
// Threads of a fused row-pass workgroup: kRowThreads, a quarter of them in
// a lean launch (four times the workgroups).
constexpr int fused_threads(int logl, int loge) {
  return logl <= kLeanMaxLog && loge == lean_loge(logl) && loge != fused_loge(logl) ? kRowThreads / 4 : kRowThreads;
}
constexpr int fused_rows_per_wg(int logl, int loge) {
  return (fused_threads(logl, loge) >> (logl - loge)) < 1 ? 1 : (fused_threads(logl, loge) >> (logl - loge));
}

// Workgroups of a fused row-pass launch: row groups over the tuned loop
// count, within the same launch-size cap as the row passes.
static unsigned fused_groups_x(const Shape& sh, uint32_t count, int rpw) {
  const uint64_t R = (uint64_t)(sh.rad3 ? 3 : 1) << sh.logR;    // rows of 2^logC points
  const uint64_t groups = (R + rpw - 1) / rpw;
  const uint64_t cap = groups * 2 * count / kRowMinGroups;
  int iters = sh.row_iters > 0 ? sh.row_iters : 1;
  if ((uint64_t)iters > cap) iters = cap > 1 ? (int)cap : 1;
  return (unsigned)((groups + iters - 1) / iters);
}

template <int LOGC, int LOGE>
static hipError_t rows_fused_launch(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                                    hipStream_t st) {
  constexpr int RPW = fused_rows_per_wg(LOGC, LOGE);
  using G = Geometry<LOGC, LOGE>;
  const size_t tables = root_tables_fit<LOGC, LOGE>(RPW, 2) ? 2 * ((size_t)G::L - 1) : 0;
  const size_t lds = ((size_t)RPW * G::STRIDE + tables) * sizeof(uint64_t);
  auto kern = k_rows_fused<LOGC, LOGE, RPW>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(fused_groups_x(sh, w.count, RPW), 2, w.count), dim3(RPW * G::NT), lds, st, w,
                     cs, tw);
  return hipGetLastError();
}

template <int LOGC>
static hipError_t rows_fused_l(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                               hipStream_t st) {
  if constexpr (LOGC > kMaxLogLdsTables) {
    // rows of 2^14 points would need 2048 threads in the fused pass: the
    // forward rows, then the pointwise product with the inverse rows, as two
    // row passes (the forward spectra go through HBM)
    hipError_t e = rows_l<LOGC, false>(w, sh, cs, tw, st);
    if (e == hipSuccess) e = rows_l<LOGC, true>(w, sh, cs, tw, st);
    return e;
  } else {
    constexpr int LOGE = fused_loge(LOGC);
    if constexpr (LOGC <= kLeanMaxLog && lean_loge(LOGC) != LOGE) {
      const uint64_t wgs = (uint64_t)fused_groups_x(sh, w.count, fused_rows_per_wg(LOGC, LOGE)) * 2 * w.count;
      if (wgs < kLeanMinGroups) return rows_fused_launch<LOGC, lean_loge(LOGC)>(w, sh, cs, tw, st);
    }
    return rows_fused_launch<LOGC, LOGE>(w, sh, cs, tw, st);
  }
}

template <int LOGR, int LOGE, bool R3>
static hipError_t inv_cols_launch(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                                  hipStream_t st) {
  constexpr int T = ColLaunch<LOGR, LOGE, R3, false>::T;
  using G = Geometry<LOGR, LOGE>;
  const size_t tables = root_tables_fit<LOGR, LOGE>(T, 1) ? (size_t)G::L - 1 : 0;
  const size_t lds = ((size_t)T * G::STRIDE + tables) * sizeof(uint64_t);
  auto kern = k_inv_cols<LOGR, LOGE, T, R3>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)ColLaunch<LOGR, LOGE, R3, false>::tiles(sh), 2, w.count);
  hipLaunchKernelGGL(kern, grid, dim3(T * G::NT), lds, st, w, cs, tw);
  return hipGetLastError();
}

template <int LOGR, bool R3>
static hipError_t inv_cols_pick(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                                hipStream_t st) {
  constexpr int LOGE = col_loge(LOGR);
  if constexpr (LOGR <= kLeanMaxLog && lean_loge(LOGR) != LOGE) {
    const uint64_t wgs = ColLaunch<LOGR, LOGE, R3, false>::tiles(sh) * 2 * w.count;
    if (wgs < kLeanMinGroups) return inv_cols_launch<LOGR, lean_loge(LOGR), R3>(w, sh, cs, tw, st);
  }
  return inv_cols_launch<LOGR, LOGE, R3>(w, sh, cs, tw, st);
}

template <int LOGR>
static hipError_t inv_cols_l(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                             hipStream_t st) {
  if constexpr (LOGR <= kMaxLogR3) {
    if (sh.rad3) return inv_cols_pick<LOGR, true>(w, sh, cs, tw, st);
  } else {
    if (sh.rad3) return hipErrorInvalidValue;
  }
  return inv_cols_pick<LOGR, false>(w, sh, cs, tw, st);
}

#define DMUL_LEN_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t launch_forward(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                          const DivTable* dt, hipStream_t st, Marks* marks) {
  hipError_t e = hipErrorInvalidValue;
  switch (sh.logR) {
#define X(l) case l: e = fwd_cols_l<l>(w, sh, cs, tw, dt, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kFwdCols, st);
  switch (sh.logC) {
#define X(l) case l: e = rows_l<l, false>(w, sh, cs, tw, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess && marks) marks->mark(kFwdRows, st);
  return e;
}

hipError_t launch_inverse(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                          hipStream_t st, Marks* marks) {
  hipError_t e = hipErrorInvalidValue;
  switch (sh.logC) {
#define X(l) case l: e = rows_l<l, true>(w, sh, cs, tw, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kInvRows, st);
  switch (sh.logR) {
#define X(l) case l: e = inv_cols_l<l>(w, sh, cs, tw, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess && marks) marks->mark(kInvCols, st);
  return e;
}

hipError_t launch_fused(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                        const DivTable* dt, hipStream_t st, Marks* marks) {
  hipError_t e = hipErrorInvalidValue;
  switch (sh.logR) {
#define X(l) case l: e = fwd_cols_l<l>(w, sh, cs, tw, dt, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kFwdCols, st);
  switch (sh.logC) {
#define X(l) case l: e = rows_fused_l<l>(w, sh, cs, tw, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (marks) marks->mark(kRows, st);
  switch (sh.logR) {
#define X(l) case l: e = inv_cols_l<l>(w, sh, cs, tw, st); break;
    DMUL_LEN_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess && marks) marks->mark(kInvCols, st);
  return e;
}

}  // namespace dmi
