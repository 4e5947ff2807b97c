/*
 * dmul -- exact product of two decimal integers on an AMD Instinct MI355X
 * (gfx950), by the two-prime number-theoretic-transform method of
 * "Speeding up decimal multiplication" (V. Krapivensky, 2020).
 *
 * Number format (Section 3.2, with base B = 10^19 for input and output):
 *   an integer X = sum_i a[i] * 10^(19 i) is an array of little-endian
 *   uint64_t limbs, every limb in [0, 10^19).  Leading zero limbs are
 *   allowed; an empty array (length 0) is the integer 0.
 *
 * Result: Z = X * Y as exactly na + nb limbs in [0, 10^19); the top limb(s)
 *   may be zero, nothing is normalised away (Section 3.2: the product of an
 *   n-digit and an m-digit number has n + m digits).
 *
 * Method (done entirely by HIP kernels on the device): the limbs are re-cut
 * into base-10^k digit groups with the largest k in [13, 18] such that
 * (10^k - 1)^2 * min(n_k, m_k) < p1 * p2 (eq. ci_bound as the range
 * condition of eq. product_inequality; n_k = ceil(19 na / k) counts every
 * limb as 19 digits), the groups are convolved cyclically at the length N,
 * the shortest 2^e or 3 * 2^e that holds n_k + m_k coefficients (Sections
 * 3.2 and 7.8), modulo the two primes
 *   p1 = 9223371564408373249 = 1073741769 * 2^33 + 1,
 *   p2 = 9223371938070528001 = 2147483625 * 2^32 + 1
 * (the two largest primes c*3*2^n + 1 < 2^63 with c odd and n >= 32,
 * Section 4.5) by two-pass NTTs with Montgomery arithmetic (Sections 4.4.3,
 * 5, 6, 7), and every coefficient is recovered by the two-prime CRT and
 * carried into base 10^19 (Section 8.2).  The result is bit-exact.
 *
 * The same interface is built twice: libdmul.so as above, and
 * libdmul_lazy.so with the two largest such primes below 2^62 = mu/4,
 *   p1 = 4611685318347718657, p2 = 4611685692009873409,
 * whose butterflies keep values in the redundant ranges [0, 2p) and
 * [0, 4p) between stages (Sections 8.3, 9); its digit-group bound uses its
 * own p1 * p2 (about 2^124), so k may be one less.  dmul_primes and
 * dmul_plan report the primes and plans of the build they belong to.
 *
 * Pointers: unless a function says "host", every limb pointer is a DEVICE
 * pointer (HBM, e.g. a torch tensor's data_ptr()) on the context's device.
 * The caller owns a, b and out; the library never frees them and does not
 * keep them past the call (dmul) or past dmul_sync (dmul_ex, dmul_batch).
 * The library owns its scratch, tables and status words, released by
 * dmul_ctx_destroy.
 *
 * Aliasing: a == b with na == nb (squaring, the self-convolution case the
 * paper supports in Section 6) is allowed and takes a cheaper path.  out must
 * not overlap a or b (DMUL_EINVAL).
 *
 * Threads: a context is used by one host thread at a time.  dmul() uses a
 * default context per device, guarded by a lock.
 */
#ifndef DMUL_H
#define DMUL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (0 = success, negative = error). */
#define DMUL_OK 0
#define DMUL_EINVAL (-1)   /* NULL pointer with nonzero length, overlap, bad flags */
#define DMUL_EDIGIT (-2)   /* some limb >= 10^19 (found on the device; out unspecified) */
#define DMUL_ERANGE (-3)   /* transform longer than the device path supports (N > 2^28:
                              two passes of at most 2^14 points), or a forced k that breaks
                              the convolution bound */
#define DMUL_ENOMEM (-4)   /* workspace above the context budget, or allocation failed */
#define DMUL_EDEVICE (-5)  /* a HIP runtime error */

/* Flags.  DMUL_FLAG_FORCE_K(k) forces the digit-group size k (13..18); the
 * call fails with DMUL_ERANGE if that k breaks the bound.  The product does
 * not depend on k. */
#define DMUL_FLAG_FORCE_K(k) ((unsigned)(k) & 0x1fu)
#define DMUL_FLAG_K_MASK 0x1fu
/* dmul_batch only: capture the batch's kernels in a HIP graph and replay
 * that graph when an identical batch (same pointers, sizes and flags) is
 * submitted again on the same context.  Needs a context stream set by
 * dmul_ctx_set_stream (the legacy null stream cannot be captured); without
 * one the flag is ignored.  Captured batches are dropped when the context's
 * batch buffers grow or its tuning changes (at most 8 are kept).  A batch in
 * which some product fails planning is run without capture. */
#define DMUL_FLAG_GRAPH 0x100u
/* Use a power-of-two transform length even where 3 * 2^e is shorter (for
 * tests and comparisons; the product is the same). */
#define DMUL_FLAG_POW2 0x200u

typedef struct dmul_ctx dmul_ctx;

/* Plan of one product, as chosen by the library: Section 3.2 padding to a
 * length N = factor * 2^log2_n (factor 1, or 3 as in Section 7.8), laid out
 * as R x C (Section 7.9) with R = 2^log2_rows rows and
 * C = factor * 2^log2_cols columns, log2_rows + log2_cols = log2_n, and
 * log2_rows = floor(log2_n / 2) except where a row of 3 * 2^log2_cols
 * points would pass 6144 points. */
typedef struct dmul_plan_info {
  int32_t k;            /* decimal digits per group */
  int32_t log2_n;
  int32_t log2_rows;
  int32_t log2_cols;
  uint64_t groups_a;    /* n_k */
  uint64_t groups_b;    /* m_k */
  uint64_t workspace_bytes;
  uint64_t transform_len;  /* N */
  int32_t factor;          /* 1 or 3 */
  int32_t reserved;
} dmul_plan_info;

/* dmul: Z = X * Y, blocking.  a, b, out: device pointers on the current HIP
 * device; na, nb: limb counts.  Runs on that device's default context and
 * stream (the null stream unless dmul_ctx_set_stream was called on the
 * default context) and returns once out is complete.  Returns DMUL_OK or a
 * negative DMUL_E* code.  na == 0 or nb == 0 writes na + nb zero limbs. */
int dmul(const uint64_t* a, size_t na, const uint64_t* b, size_t nb, uint64_t* out);

/* Context on `device` with a workspace budget in bytes (0 = no limit).
 * Returns DMUL_OK and *ctx, or DMUL_EDEVICE / DMUL_ENOMEM / DMUL_EINVAL.
 * Every call on a context (or a spectrum) works on the context's device and leaves the
 * calling thread's current HIP device as it found it.
 *
 * Environment, read here once per context (the default contexts of dmul
 * and dmul_host included):
 *   DMUL_HBM_BUDGET=<bytes>  the budget when hbm_budget_bytes is 0 (0 = no
 *       limit);
 *   DMUL_FORCE_K=<k>, 13 <= k <= 18: the group size k (Section 3.1) of
 *       every product of the context whose flags leave k to the library
 *       (dmul_debug_residues excepted),
 *       as if they held DMUL_FLAG_FORCE_K(k) (a product beyond the bound
 *       of eq. ci_bound then fails with DMUL_ERANGE); flags naming a k win;
 *   DMUL_POISON (set, and not "0"): fill the scratch of every product
 *       with 0xff first;
 *   DMUL_TUNE_TABLE  see dmul_ctx_tune.
 * An unset or empty DMUL_HBM_BUDGET or DMUL_FORCE_K is ignored; any other
 * value that is not a whole decimal number in its range makes this call
 * fail with DMUL_EINVAL.
 * dmul_plan, dmul_workspace_bytes and dmul_spectrum_bytes take no context
 * and read none of them. */
int dmul_ctx_create(dmul_ctx** ctx, int device, size_t hbm_budget_bytes);
/* Waits for the context's work, then frees everything it owns. */
int dmul_ctx_destroy(dmul_ctx* ctx);
/* The HIP stream (hipStream_t passed as void*) the context enqueues on;
 * NULL selects the null stream.  The stream stays owned by the caller.
 * Waits for the work already queued on the previous stream (it shares the
 * context's buffers); a pending device error is still reported by the next
 * dmul_sync. */
int dmul_ctx_set_stream(dmul_ctx* ctx, void* hip_stream);

/* Asynchronous product: enqueues the whole product on the context's stream
 * and returns.  Argument errors are returned at once; a bad limb is
 * reported by the next dmul_sync.  `flags`: 0 or DMUL_FLAG_FORCE_K(k). */
int dmul_ex(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
            uint64_t* out, unsigned flags);
/* dmul_ex_noalloc: dmul_ex for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and error reporting as dmul_ex, but
 * the call allocates nothing: the product's scratch (its 4N-word workspace
 * and its carry-map words) is a static device array of the library
 * (64 MiB + 16 KiB on every device the library runs on, held until the
 * process ends), and the tables of every transform length up to 2^21 are
 * built when the context is created.  Returns DMUL_ENOMEM for a product
 * whose transform length N (dmul_plan) exceeds 2^21 (at most about
 * 1.5 * 10^7 digits in all).  Every call on one device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device -- on two streams or two contexts of that device, without a
 * dmul_sync or stream ordering between them -- race and give wrong
 * products.  Profiling and completion timing do not record these
 * products.  DMUL_EDEVICE if the runtime could not give the array's address
 * when the context was made. */
int dmul_ex_noalloc(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                    uint64_t* out, unsigned flags);

/* Waits for everything enqueued on the context; returns DMUL_OK, or the
 * first error seen on the device since the last dmul_sync (DMUL_EDIGIT /
 * DMUL_EDEVICE).  */
int dmul_sync(dmul_ctx* ctx);

/* Batched products: count independent products, operand i given by the
 * device pointers a[i], b[i] and limb counts na[i], nb[i], result in out[i]
 * (na[i] + nb[i] limbs).  a, na, b, nb, out and status are HOST arrays of
 * length count.  All products are enqueued on the context's stream, grouped
 * into one launch per phase and transform length (so a batch needs a fixed
 * number of launches, not one set per product); dmul_sync completes it.
 * status[i] (host memory, written by dmul_sync) receives each product's own
 * code; the array must stay valid until that dmul_sync.  Several batches
 * may be enqueued before one dmul_sync: each reports to its own status
 * array.  Returns DMUL_OK or the first argument error (then nothing is
 * enqueued).  `flags` as for dmul_ex, applied to every product. */
int dmul_batch(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
               const uint64_t* const* b, const size_t* nb, uint64_t* const* out,
               int32_t* status, unsigned flags);

/* Planning, no device work: the plan for na x nb limbs (DMUL_OK, or
 * DMUL_ERANGE / DMUL_EINVAL). */
int dmul_plan(size_t na, size_t nb, unsigned flags, dmul_plan_info* info);
/* Device workspace one product of na x nb limbs needs, in bytes (used for
 * admission by footprint); 0 if the product is out of range. */
size_t dmul_workspace_bytes(size_t na, size_t nb);

/* Human-readable text for a status code (static storage). */
const char* dmul_strerror(int code);

/* Host-pointer convenience: copies a and b (HOST arrays) to the device,
 * multiplies on `device`, copies the na + nb limbs back into out (HOST).
 * For tests and tools; not for throughput. */
int dmul_host(int device, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
              uint64_t* out, unsigned flags);

/* The two primes (p[0] < p[1]) and the smallest generators g[] of their
 * multiplicative groups used for the roots of unity xi_N = g^((p-1)/N). */
void dmul_primes(uint64_t p[2], uint64_t g[2]);

/* Debug view of the convolution step alone: writes res[0..N) and
 * res[N..2N) = the cyclic convolution of the digit groups of a and b modulo
 * p1 and modulo p2 (device pointer `res` of 2N words, N from dmul_plan
 * with the same flags: DMUL_FORCE_K does not apply here), blocking.  For
 * tests of the transform separately from answer recovery. */
int dmul_debug_residues(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b,
                        size_t nb, uint64_t* res, unsigned flags);

/* Measurement hooks.  dmul_ctx_profile(ctx, 1) makes every later product on
 * the context record a HIP event on its stream after each kernel (and one
 * before the first), and resets the totals; 0 turns it off.  The events
 * cost a little time, so throughput is measured with profiling off.
 * dmul_ctx_profile_read fills total_ms[i] (summed duration) and
 * launches[i] (count) for kernel phase i < n, for products completed by a
 * dmul_sync, and returns the number of phases; dmul_phase_name(i) names
 * phase i ("fwd_cols", "fwd_rows", "inv_rows", "inv_cols", "rec_crt",
 * "rec_apply", "whole" for the one-workgroup kernel that runs a whole
 * product of transform length N <= 4096, and "rows" for the pass that runs
 * the row transforms of both directions and the pointwise product at once,
 * which products without cached spectra take instead of fwd_rows and
 * inv_rows). */
int dmul_ctx_profile(dmul_ctx* ctx, int enable);
int dmul_ctx_profile_read(dmul_ctx* ctx, double* total_ms, uint64_t* launches, int n);
/* The kernels of the work completed by the last dmul_sync, in launch order:
 * phases[i] and end_ms[i] = the end of kernel i in milliseconds after the
 * first event of that work (profiling must be on).  Returns the number of
 * kernels (fills at most n). */
int dmul_ctx_profile_events(dmul_ctx* ctx, int32_t* phases, double* end_ms, int n);
const char* dmul_phase_name(int phase);

/* Completion timing, for latency measurement without changing the
 * schedule.  dmul_ctx_timing(ctx, 1) makes every later product on the
 * context record one HIP event when it completes: after each dmul_ex
 * product on the context stream, and after each transform-length class of
 * a batch on the stream that class runs on (batches keep running their
 * classes concurrently; only hipGraph capture is skipped while timing is
 * on), plus one start event before the first work enqueued after a
 * dmul_sync.  0 turns it off.  Returns DMUL_OK, DMUL_EINVAL or
 * DMUL_ENOMEM.
 * dmul_ctx_timing_read fills ms[i] for i < n with the completion time, in
 * milliseconds after that start event, of the i-th product (in submission
 * order: dmul_ex products one by one, batch products in batch order) of
 * the work completed by the last dmul_sync; -1 where no time was recorded
 * (an argument error).  Returns the number of products, or DMUL_EINVAL. */
int dmul_ctx_timing(dmul_ctx* ctx, int enable);
long dmul_ctx_timing_read(dmul_ctx* ctx, double* ms, size_t n);

/* Cached transforms (transform reuse, the self-convolution idea of
 * Section 6 carried across products): the forward transforms of one operand
 * modulo both primes, kept on the device so that products with it skip
 * them.  A spectrum is made for the plan (dmul_plan) of its operand with a
 * partner of nb limbs under `flags` (DMUL_FLAG_FORCE_K, DMUL_FLAG_POW2), and
 * serves every product whose plan has the same digit-group size k and
 * transform length N, whatever the partner; other products fail with
 * DMUL_EINVAL.
 *
 * dmul_spectrum_create: a: device pointer to na limbs (only read by the
 *   work enqueued here: it may be freed once that work is done).  Enqueues
 *   the transforms on ctx's stream; a limb >= 10^19 is reported by the next
 *   dmul_sync (DMUL_EDIGIT).  The transforms take dmul_spectrum_bytes(na,
 *   nb, flags) = 16 N bytes of device memory: the caller's (mem, at least
 *   that many bytes, 8-byte aligned, owned by the caller and not touched
 *   until the spectrum is destroyed), or, with mem NULL, the library's own
 *   allocation, outside the context's budget.  Returns DMUL_OK and *spec,
 *   or DMUL_EINVAL (NULL, empty operand, bad flags, mem too small or
 *   misaligned), DMUL_ERANGE, DMUL_ENOMEM, DMUL_EDEVICE.
 * dmul_spectrum_destroy: releases it (and frees the library's allocation);
 *   the caller makes sure no queued work still reads it (dmul_sync on every
 *   context that used it).
 * Spectra belong to the device of the context that made them (a context of
 * another device refuses them with DMUL_EINVAL); use them on another stream
 * only after dmul_sync on the creating context. */
typedef struct dmul_spectrum dmul_spectrum;
int dmul_spectrum_create(dmul_ctx* ctx, const uint64_t* a, size_t na, size_t nb, unsigned flags,
                         void* mem, size_t mem_bytes, dmul_spectrum** spec);
int dmul_spectrum_destroy(dmul_spectrum* spec);
size_t dmul_spectrum_bytes(size_t na, size_t nb, unsigned flags);

/* dmul_spectrum_export: the spectrum's transforms in natural frequency
 * order: out (device, 2N words) receives out[i * N + k] = sum_j x_j xi^(jk)
 * mod p_(i+1), k < N, where x_j are the operand's base-10^k digit groups
 * (zero beyond its n_k groups) and xi = g^((p-1)/N) with the generators of
 * dmul_primes.  The library keeps a transform as an R x C matrix holding
 * frequency k1 + R k2 at row rev(k1), column rev(k2) (DIF without bit
 * reversal, Sections 5.4 and 7.4); the export copies it to out and puts it
 * in order there in place: bit reversal of the rows and of every row's
 * columns, then the in-place transposition of Section 7.6 (C = R, or
 * C = 2R: the column permutation rho on every row, then the two R x R
 * squares), whose row scratch is on chip.  For power-of-two plans with
 * R >= 32 (N >= 2^10); DMUL_EINVAL otherwise.  Asynchronous on ctx's
 * stream (dmul_sync completes it). */
int dmul_spectrum_export(dmul_ctx* ctx, const dmul_spectrum* spec, uint64_t* out);

/* dmul_debug_transpose: transposes the rows x cols matrix of 64-bit words
 * at data (device, row-major) in place into cols x rows, by the scheme of
 * Section 7.6 (cols == rows; cols == 2 rows: rho on every row, then the two
 * squares; rows == 2 cols: the two squares of the cols x rows view, then
 * rho^-1 on each of its rows).  rows and cols: powers of two in [32, 8192].
 * Asynchronous on ctx's stream.  Returns DMUL_OK or DMUL_EINVAL. */
int dmul_debug_transpose(dmul_ctx* ctx, uint64_t* data, size_t rows, size_t cols);

/* dmul_ex_spectrum: like dmul_ex with X given by its spectrum sa (X has
 * sa's na limbs), and Y given either by limbs (b, nb: device pointer, sb
 * NULL) or by its spectrum sb (then b must be NULL and nb equal sb's limb
 * count).  sa == sb squares.  out: na + nb limbs, not overlapping b.  flags
 * as for the spectra.  Asynchronous on ctx's stream (dmul_sync completes
 * it).  Returns DMUL_OK or a negative DMUL_E* code (DMUL_EINVAL also when
 * the product's plan differs from a spectrum's). */
int dmul_ex_spectrum(dmul_ctx* ctx, const dmul_spectrum* sa, const uint64_t* b, size_t nb,
                     const dmul_spectrum* sb, uint64_t* out, unsigned flags);

/* dmul_batch_ex: dmul_batch where operands may come as spectra.  sa and sb
 * are NULL or host arrays of count spectrum pointers; where sa[i] is not
 * NULL, a[i] is ignored and na[i] must equal its limb count (likewise b).
 * A product whose plan does not match its spectra gets status DMUL_EINVAL. */
int dmul_batch_ex(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
                  const dmul_spectrum* const* sa, const uint64_t* const* b, const size_t* nb,
                  const dmul_spectrum* const* sb, uint64_t* const* out, int32_t* status,
                  unsigned flags);

/* Size-class tuning: for products of transform length transform_len
 * (2^e or 3 * 2^e), every workgroup of the row pass loops over `row_iters`
 * groups of rows (0 = the default).  Contexts start from the table written
 * by the project's autotuner (dmul_tune.txt beside the library, or the file
 * named by DMUL_TUNE_TABLE; an empty name means no table: lines
 * "transform_len row_iters [path]" and "streams S").  Returns DMUL_OK or
 * DMUL_EINVAL (a length that is not a supported size class, or row_iters
 * outside 0..64). */
int dmul_ctx_tune(dmul_ctx* ctx, uint64_t transform_len, int row_iters);
/* Kernel path of launches of 8 or more products of transform length
 * transform_len (a batch class): 0 the default rule (the whole-product
 * kernel up to N = 4096), 1 always the whole-product kernel (N <= 4096
 * only), 2 always the pass kernels.  Fewer products of a length (a lone
 * product, a small class) always take the default rule for them: the
 * whole-product kernel up to N = 256, the pass kernels beyond.  Table lines
 * "transform_len row_iters path" set it too.  Returns DMUL_OK or
 * DMUL_EINVAL. */
int dmul_ctx_tune_path(dmul_ctx* ctx, uint64_t transform_len, int path);
/* Number of side streams (1..16; 0 = the default 8) over which a batch's
 * transform-length classes run concurrently; the table line "streams S"
 * sets it too.  Returns DMUL_OK or DMUL_EINVAL. */
int dmul_ctx_tune_streams(dmul_ctx* ctx, int streams);
/* Persistent whole-product launches in batches: with queue = 1 (table
 * line "queue Q"), the classes of a batch that take the whole-product
 * kernel are not launched one per transform length but gathered into at
 * most three launches by register and LDS need (sub-transforms of up to
 * 2^8 points, 2^9..2^10, longer), each a grid of as many workgroups as the
 * device holds at once that take the products, longest first, from a queue
 * in device memory; with 0 (the default), one launch per length with one
 * workgroup per product.  Results are identical.  Returns DMUL_OK or
 * DMUL_EINVAL. */
int dmul_ctx_tune_queue(dmul_ctx* ctx, int queue);

/* Library version string. */
const char* dmul_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DMUL_H */
