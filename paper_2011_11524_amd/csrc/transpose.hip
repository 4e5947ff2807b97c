// In-place transposition of an R x C matrix of words in device memory, for
// C = R, C = 2R ("n x 2n") and R = 2C ("2n x n"), by the scheme of
// Section 7.6: an n x 2n matrix is transposed by permuting the columns of
// every row with rho (row position j takes column 2j for j < n and
// 2(j - n) + 1 for j >= n) and then transposing its left and right n x n
// squares in place; a 2n x n matrix, the inverse operation, by transposing
// the two squares (of the same n x 2n view) and then applying rho^-1 to
// every row of 2n words.  The scratch a row permutation needs (2n words,
// Section 7.6) is the LDS of the workgroup that permutes that row.
//
// The same row kernel also applies bit-reversal permutations to the row
// order and to the columns of every row, which is what turns a spectrum of
// the two-pass layout (row position rev(k1), column position rev(k2) for
// frequency k1 + R k2, Sections 5.4 and 7.4) into natural order before its
// transposition (dmul_spectrum_export).
#include <dmul.h>

#include "ctx.hpp"
#include "ntt_dev.hpp"

namespace dmi {

namespace {

constexpr int kTile = 32;             // square-transpose tiles of 32 x 32 words
constexpr int kTileThreads = 256;
constexpr int kRowThreads = 256;

// Column of the source row that lands at position j of the permuted row:
// optionally bit reversal of the column index (within log2 cols bits), then
// optionally rho (fwd) or rho^-1 (inverse), composed as
//   new[j] = old[rev(sigma(j))]    (rho:     sigma(j) = 2j or 2(j - n) + 1)
//   new[j] = old[sigma^-1(j)]      (rho^-1:  new[2i] = old[i], new[2i+1] = old[i + n])
struct RowPerm {
  uint32_t cols;
  int log_cols;
  int bitrev_cols;   // 1: reverse the column index bits
  int rho;           // 0: none, 1: rho, -1: rho^-1
  __device__ uint32_t source(uint32_t j) const {
    const uint32_t n = cols / 2;
    uint32_t s = j;
    if (rho == 1) s = j < n ? 2 * j : 2 * (j - n) + 1;
    else if (rho == -1) s = (j & 1) ? n + (j >> 1) : (j >> 1);
    return bitrev_cols ? bitrev(s, log_cols) : s;
  }
};

// Row pass: workgroup b takes row i = b and its partner r = rev(i) (or i
// itself without row reversal), skipping pairs it does not own (i > r), so
// every row is read and written by exactly one workgroup.  Both rows are
// read into LDS first, then row i's permuted words are written to row r
// and row r's to row i.
__global__ void __launch_bounds__(kRowThreads)
k_permute_rows(uint64_t* __restrict__ data, uint32_t rows, int log_rows, int bitrev_rows, RowPerm pm) {
  extern __shared__ uint64_t zeta[];       // 2 * cols words: the two rows
  const uint32_t i = blockIdx.x;
  const uint32_t r = bitrev_rows ? bitrev(i, log_rows) : i;
  if (r < i) return;
  const uint32_t C = pm.cols;
  uint64_t* row_i = data + (size_t)i * C;
  uint64_t* row_r = data + (size_t)r * C;
  for (uint32_t j = threadIdx.x; j < C; j += blockDim.x) {
    zeta[j] = row_i[j];
    zeta[C + j] = row_r[j];
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < C; j += blockDim.x) {
    const uint32_t s = pm.source(j);
    row_r[j] = zeta[s];
    if (r != i) row_i[j] = zeta[C + s];
  }
}

// In-place transposition of n x n squares of a matrix with row pitch
// `pitch`; square q (blockIdx.z) starts at column q * n.  Workgroup
// (bx, by) with bx <= by swaps tile (by, bx) with tile (bx, by), each
// transposed through LDS; a diagonal tile is transposed onto itself.
__global__ void __launch_bounds__(kTileThreads)
k_square_transpose(uint64_t* __restrict__ data, uint32_t n, uint32_t pitch) {
  __shared__ uint64_t ta[kTile][kTile + 1], tb[kTile][kTile + 1];
  const uint32_t bx = blockIdx.x, by = blockIdx.y;
  if (bx > by) return;
  uint64_t* base = data + (size_t)blockIdx.z * n;
  const uint32_t tx = threadIdx.x % kTile, ty0 = threadIdx.x / kTile;
  constexpr uint32_t kStep = kTileThreads / kTile;
  // tile A = rows by*T.., cols bx*T..;  tile B = rows bx*T.., cols by*T..
  for (uint32_t y = ty0; y < kTile; y += kStep) {
    ta[y][tx] = base[(size_t)(by * kTile + y) * pitch + bx * kTile + tx];
    if (bx != by) tb[y][tx] = base[(size_t)(bx * kTile + y) * pitch + by * kTile + tx];
  }
  __syncthreads();
  for (uint32_t y = ty0; y < kTile; y += kStep) {
    // transposed A goes to B's place, transposed B to A's place
    base[(size_t)(bx * kTile + y) * pitch + by * kTile + tx] = ta[tx][y];
    if (bx != by) base[(size_t)(by * kTile + y) * pitch + bx * kTile + tx] = tb[tx][y];
  }
}

bool pow2_at_least(uint64_t x, uint64_t lo, int* lg) {
  if (x < lo || (x & (x - 1))) return false;
  int l = 0;
  while (((uint64_t)1 << l) < x) ++l;
  *lg = l;
  return true;
}

hipError_t launch_permute_rows(uint64_t* data, uint32_t rows, uint32_t cols, bool bitrev_rows,
                               bool bitrev_cols, int rho, hipStream_t st) {
  int lr = 0, lc = 0;
  pow2_at_least(rows, 1, &lr);
  pow2_at_least(cols, 1, &lc);
  const size_t lds = 2 * (size_t)cols * sizeof(uint64_t);
  hipError_t e = allow_lds((const void*)k_permute_rows, lds);
  if (e != hipSuccess) return e;
  RowPerm pm{cols, lc, bitrev_cols ? 1 : 0, rho};
  hipLaunchKernelGGL(k_permute_rows, dim3(rows), dim3(kRowThreads), lds, st, data, rows, lr,
                     bitrev_rows ? 1 : 0, pm);
  return hipGetLastError();
}

hipError_t launch_squares(uint64_t* data, uint32_t n, uint32_t pitch, uint32_t squares, hipStream_t st) {
  const uint32_t t = n / kTile;
  hipLaunchKernelGGL(k_square_transpose, dim3(t, t, squares), dim3(kTileThreads), 0, st, data, n, pitch);
  return hipGetLastError();
}

}  // namespace

// rows x cols -> cols x rows in place; with bitrev set, the row order and
// the columns of every row are bit-reversed first (the transpose then
// yields the natural order of a two-pass spectrum).
int transpose_inplace(uint64_t* data, uint64_t rows, uint64_t cols, bool bitrev, hipStream_t st) {
  int lr = 0, lc = 0;
  if (!pow2_at_least(rows, kTile, &lr) || !pow2_at_least(cols, kTile, &lc)) return DMUL_EINVAL;
  if (lr > kMaxLogLdsTables || lc > kMaxLogLdsTables) return DMUL_EINVAL;
  hipError_t e = hipSuccess;
  if (rows == cols) {
    if (bitrev) e = launch_permute_rows(data, (uint32_t)rows, (uint32_t)cols, true, true, 0, st);
    if (e == hipSuccess) e = launch_squares(data, (uint32_t)rows, (uint32_t)cols, 1, st);
  } else if (cols == 2 * rows) {
    // n x 2n: rho on the columns of every row (after the bit reversals),
    // then the two n x n squares
    e = launch_permute_rows(data, (uint32_t)rows, (uint32_t)cols, bitrev, bitrev, 1, st);
    if (e == hipSuccess) e = launch_squares(data, (uint32_t)rows, (uint32_t)cols, 2, st);
  } else if (rows == 2 * cols) {
    // 2n x n: the two squares of the n x 2n view, then rho^-1 on each of its
    // n rows of 2n words
    if (bitrev) return DMUL_EINVAL;
    e = launch_squares(data, (uint32_t)cols, (uint32_t)rows, 2, st);
    if (e == hipSuccess) e = launch_permute_rows(data, (uint32_t)cols, (uint32_t)rows, false, false, -1, st);
  } else {
    return DMUL_EINVAL;
  }
  return from_hip(e);
}

}  // namespace dmi
