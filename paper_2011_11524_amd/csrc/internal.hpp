// Shared declarations of the host library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "field.hpp"

// The redundant-range build (libdmul_lazy.so, Sections 8.3 and 9): primes
// below 2^62 = mu/4 let butterfly values stay in [0, 2p) or [0, 4p) between
// stages instead of being reduced to [0, p) after every operation.
#ifndef DMUL_LAZY_FIELD
#define DMUL_LAZY_FIELD 0
#endif

namespace dmi {

constexpr bool kLazy = DMUL_LAZY_FIELD != 0;
constexpr int kMaxLogN = 28;       // two LDS passes of at most 2^14 points each
constexpr int kMaxLogLen = 14;     // longest sub-transform held in one workgroup's LDS
// Rows of up to 2^13 points take the fused row pass (8 points per thread);
// a 2^14-point row would need 2048 threads there, so such rows run the
// forward and inverse row passes separately.  (Root tables are staged in
// LDS wherever they fit beside a pass's data, and read from global memory,
// L2-resident, where they do not.)
constexpr int kMaxLogLdsTables = 13;
constexpr int kMaxLogC3 = 11;      // rows of 3 * 2^logC points: logC <= 11
constexpr int kMaxLogR3 = 12;      // with C = 3M a column tile holds three columns of 2^logR points
constexpr int kMinLogN3 = 4;       // lengths 3 * 2^e are used for e >= 4
constexpr uint64_t kSmallMaxN = 4096;   // whole product in one workgroup up to this length
// ... for a lone product (or fewer than kSmallMinCount of one length): one
// workgroup against the lean pass launches, which win from N = 384 (0.027
// against 0.028 ms, and 0.031 against 0.083 ms at N = 3072; the kernel wins
// at N = 192, 0.023 against 0.025 ms)
constexpr uint64_t kSmallSoloMaxN = 256;
constexpr size_t kSmallMinCount = 8;       // products of a class that make 4096 worth it
constexpr int kMinK = 13;          // p1*p2 < 10^(3k): three base-10^k parts per coefficient
// Allocation-free products (dmul_ex_noalloc) run in a static device array of
// 4 * kStaticMaxN workspace words plus kStaticMapWords words of carry maps.
constexpr uint64_t kStaticMaxN = (uint64_t)1 << 21;
constexpr size_t kStaticMapWords = 2048;   // >= (kStaticMaxN / 1024 + 1) 32-bit maps
constexpr uint64_t kLimbBase = 10000000000000000000ULL;  // 10^19

// Magic multipliers for floor(x / 10^e), x < 2^64, e in [0, 19]:
//   q = umulhi(x >> e, mag[e]) >> sh[e]    (e >= 1),  q = x  (e = 0)
// i.e. division by 2^e by shifting, then by 5^e by a Granlund-Montgomery
// multiply-high (division by invariant integers using multiplication).
struct DivTable {
  uint64_t mag[20];
  uint32_t sh[20];
  uint64_t pow10[20];
};

// Everything a kernel needs about one product, passed by value.
// The transform length is N = 2^logN (rad3 = 0) or 3 * 2^logN (rad3 = 1;
// the primes' form c*3*2^n + 1 admits these lengths, Sections 4.5, 7.8).
// It is laid out as R x C with R = 2^logR rows and C = 2^logC (rad3 = 0)
// or 3 * 2^logC (rad3 = 1) columns.
struct PlanDev {
  uint64_t na, nb;          // limbs of a and b (base 10^19)
  uint64_t n, m;            // base-10^k groups of a and b
  uint64_t N;               // transform length
  int k;                    // digits per group
  int logN, logR, logC;     // logR + logC = logN
  int rad3;                 // 1: N and C carry a factor 3
};

__host__ __device__ constexpr uint64_t row_len(int logC, int rad3) {
  return (uint64_t)(rad3 ? 3 : 1) << logC;
}
// The inter-pass exponent e < N is split as e = e_hi * 2^lb + e_lo.
__host__ __device__ constexpr int pass_split_bits(int logC, int rad3) { return logC + (rad3 ? 2 : 0); }

// Device-side constant data for both primes, built once per context.
struct Consts {
  Prime P[2];
  uint64_t r_tilde;         // R * (p1^-1 mod p2) mod p2 (Montgomery form for the CRT)
  uint64_t kappa[2][2];     // [prime][0 forward, 1 inverse]: R * (w - w^2) / 2 mod p, w the
                            // cube root of unity of that direction (radix-3 butterfly)
};

// Per transform-length tables for the inter-pass factor xi_N^(+-e), e < N,
// split e = e_hi*2^lb + e_lo with lb = pass_split_bits (Montgomery form; the
// inverse low table also carries the scale R^2 N^-1 of the linearity trick).
struct TwiddleSet {
  const uint64_t* len_fwd[2];   // [prime] -> base of per-length root tables (forward roots)
  const uint64_t* len_inv[2];   // [prime] -> same for inverse roots
  const uint64_t* r3_fwd[2];    // [prime] -> base of the radix-3 row tables (forward)
  const uint64_t* r3_inv[2];    // [prime] -> same, inverse
  uint64_t scale[2];            // [prime] R^2 N^-1 mod p (Montgomery form of R N^-1)
  const uint64_t* hi_fwd[2];
  const uint64_t* lo_fwd[2];
  const uint64_t* hi_inv[2];
  const uint64_t* lo_inv[2];
};

// Root tables of a transform of L = 2^l points, one per butterfly stage:
// the stage on bit b multiplies by w_L^(i * 2^(l-1-b)), i < 2^b (Sections
// 5.2, 5.3), and its table holds exactly those factors, indexed by i, at
// offset 2^b - 1 of the length's block (2^l - 1 words).  A stage's factor
// reads are then contiguous in i, which keeps the lanes of a wavefront on
// distinct LDS banks (a single table of w^e read at e = i * 2^(l-1-b)
// would be a strided read).  Blocks for l = 1, 2, ... are stored back to
// back in a per-prime, per-direction region of kRootWords words.
__host__ __device__ constexpr size_t root_block_offset(int l) { return ((size_t)1 << l) - (size_t)l - 1; }
__host__ __device__ constexpr int root_stage_offset(int b) { return (1 << b) - 1; }
constexpr size_t kRootWords = root_block_offset(kMaxLogLen + 1);
// Offset of the table of w_C^i (i < 2M) for a row of C = 3M points, M = 2^l,
// inside a per-prime radix-3 block: tables for l = 0, 1, ... back to back.
__host__ __device__ constexpr size_t r3_table_offset(int l) { return 2 * (((size_t)1 << l) - 1); }
constexpr size_t kR3TableWords = 2 * (((size_t)1 << (kMaxLogC3 + 1)) - 1);

// Optional per-kernel timing: when set, a launch wrapper records an event on
// the stream after each kernel it launches (phase ids below).
enum Phase { kFwdCols = 0, kFwdRows, kInvRows, kInvCols, kRecCrt, kRecApply, kWhole, kRows, kNumPhases };
struct Marks {
  virtual void mark(int phase, hipStream_t st) = 0;
  virtual ~Marks() = default;
};

// One product as the kernels see it.
struct ProdDesc {
  PlanDev pl;
  const uint64_t* a;        // operands (device)
  const uint64_t* b;
  uint64_t* out;            // na + nb result limbs
  uint64_t* ws;             // 4N words: X1 X2 Y1 Y2 (recovery scratch reuses Y)
  int* status;              // bit 1: a limb >= 10^19 (set by the split)
  uint32_t* rec_sync;       // recovery: the carry map of each block (nblk words)
  uint32_t nblk;            // recovery workgroups
  int square;               // a == b: one operand transformed
  const uint64_t* xs;       // cached forward transforms of a (2N words: mod p1, mod p2), or null
  const uint64_t* ys;       // the same for b, or null
  uint64_t scale[2];        // R^2 N^-1 per prime (Montgomery form): read by the queued whole-product kernel
};

// Whether the forward passes transform operand op (0 = a, 1 = b) of d:
// not a squared product's second operand, nor an operand with a cached
// spectrum.
__host__ __device__ inline bool transforms_operand(const ProdDesc& d, int op) {
  return op == 0 ? d.xs == nullptr : (!d.square && d.ys == nullptr);
}

// A launch over products of one transform length: `one` when many is null,
// else many[0 .. count) (device memory), one per blockIdx.z.
struct Work {
  ProdDesc one;
  const ProdDesc* many;
  uint32_t count;
};

// Grid shape shared by the products of a launch.
struct Shape {
  int logR, logC, rad3;
  int any_nonsquare;        // some product transforms two operands
  int row_iters;            // row groups per workgroup in the row pass
  uint32_t max_nblk;        // largest recovery grid among the products
  int rec_lean;             // the recovery in short blocks (recover_blocks(pl, true))
};

// Launch wrappers (ntt.hip, carry.hip).  All enqueue on `stream` and return
// hipSuccess or the launch error.
hipError_t launch_forward(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                          const DivTable* dt, hipStream_t stream, Marks* marks);
hipError_t launch_inverse(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                          hipStream_t stream, Marks* marks);
// The three transform passes of products without cached spectra: forward
// columns, then the rows in both directions with the pointwise product, then
// inverse columns (the same residues as launch_forward + launch_inverse).
hipError_t launch_fused(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                        const DivTable* dt, hipStream_t stream, Marks* marks);
hipError_t launch_recover(const Work& w, const Shape& sh, const Consts& cs, const DivTable* dt,
                          const DivTable* dt_host, hipStream_t stream, Marks* marks);
// Whole products in one workgroup (small.hip): for N <= kSmallMaxN when a
// launch carries at least kSmallMinCount products of the length, else for
// N <= kSmallSoloMaxN (beyond it a lone product is faster on the passes,
// which use the whole device).
bool small_fits(const PlanDev& pl, size_t count);
hipError_t launch_small(const Work& w, const Shape& sh, const Consts& cs, const TwiddleSet& tw,
                        const DivTable* dt, const DivTable* dt_host, hipStream_t stream, Marks* marks);
// The persistent whole-product kernel over w.many[0 .. count) of mixed
// lengths of one tier (small_tier), each descriptor with its scale: a grid
// of what the device holds at once, each workgroup taking products from the
// queue *head (zero at launch).  lds: the largest small_lds_bytes of them.
constexpr int kQueueTiers = 3;
int small_tier(const PlanDev& pl);
size_t small_lds_bytes(const PlanDev& pl);
hipError_t launch_small_queue(const Work& w, int tier, size_t lds, uint32_t* head, const Consts& cs,
                              const TwiddleSet& tw, const DivTable* dt, const DivTable* dt_host,
                              hipStream_t stream, Marks* marks);
// Raises a kernel's dynamic-LDS limit to lds_bytes when above the default
// 64 KB (once per kernel and size: the attribute call is host work).
hipError_t allow_lds(const void* kernel, size_t lds_bytes);
// Recovery blocks of a product: the default size, or (lean) the shorter
// blocks of a lone product whose default recovery would not fill the CUs.
size_t recover_blocks(const PlanDev& pl, bool lean);
bool recover_lean(const PlanDev& pl);
hipError_t launch_zero(uint64_t* out, size_t n, hipStream_t stream);
// n 32-bit words of v (the scratch poisoning of contexts made with
// DMUL_POISON set: workspaces start as garbage, never as the last product's).
hipError_t launch_fill32(void* out, size_t n, uint32_t v, hipStream_t stream);
constexpr uint32_t kPoison = 0xffffffffu;

}  // namespace dmi
