// C ABI of the decimal multiplier: contexts, planning, the single-product
// path (dmul, dmul_ex), batches (dmul_batch) and status handling.
//
// Host-side work here is only the plan (Section 3.2 padding rule, the base
// choice of Section 4.3 as a bound check, the N = R*C split of Section 7.9),
// the one-time constants of the field (Section 4.4.3 Montgomery form,
// Section 6 scale R^2 N^-1, Section 8.2.2 r~) and root tables (Section 5.5).
// Every step of a product runs in the kernels of ntt.hip and carry.hip.
#include <dmul.h>

#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace dmi;
typedef unsigned __int128 u128;

namespace {

// The primes: FindPrimes(w = 64, n_min = 32, l = 2) of Section 4.5, i.e.
// the two largest primes c*3*2^n + 1 < 2^63 with c odd and n >= 32; the
// redundant-range build takes FindPrimes(63, 32, 2), the two largest below
// 2^62 = mu/4 (Section 8.3).  n >= 32 makes p == 1 (mod 2^32), which the
// word-serial REDC relies on.
constexpr uint64_t kP[2] = {kLazy ? 4611685318347718657ULL : 9223371564408373249ULL,
                            kLazy ? 4611685692009873409ULL : 9223371938070528001ULL};
// Smallest generators of F_p^*, and the prime factors of p - 1 that prove it.
constexpr uint64_t kG[2] = {kLazy ? 5ULL : 13ULL, 19};
const std::vector<uint64_t> kPm1Factors[2] = {
    kLazy ? std::vector<uint64_t>{2, 3, 19, 41, 153151ULL} : std::vector<uint64_t>{2, 3, 119304641ULL},
    kLazy ? std::vector<uint64_t>{2, 3, 277, 323027ULL} : std::vector<uint64_t>{2, 3, 5, 7, 199, 4111}};
constexpr uint64_t kPrimeLimit = kLazy ? (1ULL << 62) : (1ULL << 63);

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }
uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1;
  a %= p;
  while (e) {
    if (e & 1) r = mulmod(r, a, p);
    a = mulmod(a, a, p);
    e >>= 1;
  }
  return r;
}
uint64_t inv_mod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }
// Montgomery form x*R mod p, R = 2^64 (Section 4.4.3).
uint64_t to_mont(uint64_t x, uint64_t p) { return (uint64_t)(((u128)(x % p) << 64) % p); }

bool check_field() {
  for (int i = 0; i < 2; ++i) {
    const uint64_t p = kP[i];
    if ((p & 0xffffffffULL) != 1) return false;
    if (p >= kPrimeLimit) return false;
    uint64_t m = p - 1;
    for (uint64_t q : kPm1Factors[i]) {
      if (powmod(kG[i], (p - 1) / q, p) == 1) return false;
      while (m % q == 0) m /= q;
    }
    if (m != 1) return false;   // the factor list is complete
  }
  return kP[0] < kP[1];
}

// Granlund-Montgomery magic numbers for floor(x / 10^e), x < 2^64:
// floor(x / 10^e) = floor((x >> e) / 5^e), and for inputs below 2^(64-e)
// the multiplier m = floor(2^(64-e+l) / 5^e) + 1 with l = ceil(log2 5^e)
// gives floor(x' / 5^e) = (x' * m) >> (64 - e + l).
DivTable make_div_table() {
  DivTable t{};
  uint64_t p10 = 1, p5 = 1;
  for (int e = 0; e < 20; ++e) {
    t.pow10[e] = p10;
    if (e == 0) {
      t.mag[0] = 1;
      t.sh[0] = 0;
    } else {
      int l = 0;
      while (((u128)1 << l) < p5) ++l;
      const int nbits = 64 - e;
      const u128 m = (((u128)1 << (nbits + l)) / p5) + 1;
      t.mag[e] = (uint64_t)m;
      t.sh[e] = (uint32_t)(nbits + l - 64);
    }
    if (e < 19) p10 *= 10;
    if (e < 19) p5 *= 5;
    if (e == 19) break;
  }
  return t;
}

bool check_div_table(const DivTable& t) {
  uint64_t s = 0x9e3779b97f4a7c15ULL;
  for (int e = 1; e < 20; ++e) {
    const uint64_t d = t.pow10[e];
    for (int it = 0; it < 4000; ++it) {
      s ^= s << 13; s ^= s >> 7; s ^= s << 17;
      uint64_t x;
      switch (it & 3) {
        case 0: x = s; break;
        case 1: x = s % 10000000000000000000ULL; break;
        case 2: x = d * (s % (~0ULL / d)) + (it & 4 ? d - 1 : 0); break;
        default: x = ~0ULL - (s & 0xffff); break;
      }
      const uint64_t q = (uint64_t)(((u128)(x >> e) * t.mag[e]) >> 64) >> t.sh[e];
      if (q != x / d) return false;
    }
  }
  return true;
}


}  // namespace


namespace dmi {

hipError_t allow_lds(const void* kernel, size_t lds_bytes) {
  if (lds_bytes <= 64 * 1024) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> done;   // (kernel, device) -> bytes set
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find({kernel, dev});
  if (it != done.end() && it->second >= lds_bytes) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e == hipSuccess) done[{kernel, dev}] = lds_bytes;
  return e;
}

int from_hip(hipError_t e) { return e == hipSuccess ? DMUL_OK : (e == hipErrorOutOfMemory ? DMUL_ENOMEM : DMUL_EDEVICE); }

// Rows of the R x C layout of a length 2^e (rad3 = 0) or 3 * 2^e (rad3 = 1):
// R = 2^floor(e/2) (Section 7.9), with fewer columns for 3 * 2^e where a
// row would pass 3 * 2^kMaxLogC3 points.
int layout_logR(int e, int rad3) {
  int r = e / 2;
  if (rad3 && e - r > kMaxLogC3) r = e - kMaxLogC3;
  return r;
}

int make_plan(size_t na, size_t nb, unsigned flags, PlanDev* pl) {
  if (flags & ~(DMUL_FLAG_K_MASK | DMUL_FLAG_POW2)) return DMUL_EINVAL;
  const int fk = (int)(flags & DMUL_FLAG_K_MASK);
  if (fk && (fk < kMinK || fk > 18)) return DMUL_EINVAL;
  if (na == 0 || nb == 0) return DMUL_EINVAL;
  if (na > ((size_t)1 << 40) || nb > ((size_t)1 << 40)) return DMUL_ERANGE;
  // largest group count allowed per k: (10^k - 1)^2 * min < p1*p2
  static const struct Limits {
    uint64_t lim[19];
    Limits() {
      const u128 P = (u128)kP[0] * kP[1];
      uint64_t B1 = 1;
      for (int kk = 0; kk <= 18; ++kk) {
        const u128 L = (u128)(B1 - 1) * (B1 - 1);
        const u128 q = kk ? (P - 1) / L : ~(u128)0;
        lim[kk] = q > ~(u128)0 >> 64 ? ~0ULL : (uint64_t)q;
        B1 *= 10;
      }
    }
  } limits;
  int k = 0;
  uint64_t nk = 0, mk = 0;
  for (int kk = 18; kk >= kMinK; --kk) {
    if (fk && kk != fk) continue;
    const uint64_t a = (19 * (uint64_t)na + kk - 1) / kk;
    const uint64_t b = (19 * (uint64_t)nb + kk - 1) / kk;
    const uint64_t mn = a < b ? a : b;
    if (mn <= limits.lim[kk]) { k = kk; nk = a; mk = b; break; }
  }
  if (!k) return DMUL_ERANGE;
  // Transform length: the shortest 2^e or 3*2^e (Section 7.8) holding all
  // n_k + m_k coefficients (Section 3.2); each layout within its LDS limits.
  const uint64_t need = nk + mk;
  int e2 = 2;
  while (((uint64_t)1 << e2) < need) ++e2;
  int e3 = kMinLogN3;
  while (((uint64_t)3 << e3) < need) ++e3;
  const int logR3 = layout_logR(e3, 1);
  const bool fit3 = logR3 <= kMaxLogR3;
  const bool fit2 = e2 <= kMaxLogN;
  const bool use3 = !(flags & DMUL_FLAG_POW2) && fit3 && (!fit2 || ((uint64_t)3 << e3) < ((uint64_t)1 << e2));
  if (!use3 && !fit2) return DMUL_ERANGE;
  pl->na = na;
  pl->nb = nb;
  pl->n = nk;
  pl->m = mk;
  pl->k = k;
  if (use3) {
    pl->rad3 = 1;
    pl->logN = e3;
    pl->N = (uint64_t)3 << e3;
    pl->logR = logR3;
  } else {
    pl->rad3 = 0;
    pl->logN = e2;
    pl->N = (uint64_t)1 << e2;
    pl->logR = layout_logR(e2, 0);
  }
  pl->logC = pl->logN - pl->logR;
  return DMUL_OK;
}

size_t workspace_words(const PlanDev& pl) { return 4 * (size_t)pl.N; }

// Inter-pass factor tables of a transform of length N = R*C with split bits
// lb (Section 7.9's twiddle xi_N^(+-e), e < N, as hi[e >> lb] * lo[e mod 2^lb];
// the inverse low table also carries R^2 N^-1, Section 6), in Montgomery
// form: 2 * (HI + LO) words per prime, written to h.  scale[] receives
// R^2 N^-1 in Montgomery form per prime.
static size_t pass_words(uint64_t N, int lb) {
  return 2 * 2 * ((size_t)(N >> lb) + ((size_t)1 << lb));
}

static void fill_pass_tables(uint64_t N, int lb, uint64_t* h, uint64_t scale[2]) {
  const size_t LO = (size_t)1 << lb, HI = N >> lb;
  const size_t per = 2 * (HI + LO);
  for (int i = 0; i < 2; ++i) {
    const uint64_t p = kP[i];
    const uint64_t xi = powmod(kG[i], (p - 1) / N, p);   // primitive N-th root
    const uint64_t xinv = inv_mod(xi, p);
    const uint64_t rn = mulmod(to_mont(1, p), inv_mod(N % p, p), p);   // R * N^-1
    uint64_t* hf = h + (size_t)i * per;
    uint64_t* lf = hf + HI;
    uint64_t* hi = lf + LO;
    uint64_t* li = hi + HI;
    const uint64_t xiS = powmod(xi, LO, p), xinvS = powmod(xinv, LO, p);
    uint64_t a = 1, b = 1;
    for (size_t e = 0; e < HI; ++e) {
      hf[e] = to_mont(a, p);
      hi[e] = to_mont(b, p);
      a = mulmod(a, xiS, p);
      b = mulmod(b, xinvS, p);
    }
    a = 1;
    b = 1;
    for (size_t e = 0; e < LO; ++e) {
      lf[e] = to_mont(a, p);
      li[e] = to_mont(mulmod(b, rn, p), p);
      a = mulmod(a, xi, p);
      b = mulmod(b, xinv, p);
    }
    scale[i] = to_mont(rn, p);
  }
}

// The tables of every length up to kStaticMaxN, in one allocation made when
// the context is created (so products of those lengths, dmul_ex_noalloc's
// included, never allocate tables).
int prebuild_pass_tables(dmul_ctx* ctx) {
  struct Len { uint64_t N; int lb; size_t off; };
  std::vector<Len> lens;
  size_t total = 0;
  for (int rad3 = 0; rad3 < 2; ++rad3) {
    for (int e = rad3 ? kMinLogN3 : 2; e <= kMaxLogN; ++e) {
      const uint64_t N = (uint64_t)(rad3 ? 3 : 1) << e;
      const int logR = layout_logR(e, rad3);
      if (N > kStaticMaxN || (rad3 && logR > kMaxLogR3)) break;
      const int lb = pass_split_bits(e - logR, rad3);
      lens.push_back({N, lb, total});
      total += pass_words(N, lb);
    }
  }
  std::vector<uint64_t> h(total);
  std::vector<std::pair<uint64_t, PassTables>> ents;
  for (const Len& l : lens) {
    PassTables pt;
    fill_pass_tables(l.N, l.lb, h.data() + l.off, pt.scale);
    pt.owned = false;
    ents.push_back({l.N, pt});
  }
  hipError_t e = hipMalloc(&ctx->pass_block, total * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemcpy(ctx->pass_block, h.data(), total * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return from_hip(e);
  for (size_t i = 0; i < lens.size(); ++i) {
    ents[i].second.dev = ctx->pass_block + lens[i].off;
    ctx->pass.emplace(ents[i].first, ents[i].second);
  }
  return DMUL_OK;
}

static void set_twiddles(const dmul_ctx* ctx, const PlanDev& pl, const PassTables& pt, TwiddleSet* tw) {
  for (int i = 0; i < 2; ++i) {
    tw->len_fwd[i] = ctx->d_roots + (size_t)(2 * i) * kRootWords;
    tw->len_inv[i] = ctx->d_roots + (size_t)(2 * i + 1) * kRootWords;
    tw->r3_fwd[i] = ctx->d_r3 + (size_t)(2 * i) * kR3TableWords;
    tw->r3_inv[i] = ctx->d_r3 + (size_t)(2 * i + 1) * kR3TableWords;
  }
  const int lb = pass_split_bits(pl.logC, pl.rad3);
  const size_t LO = (size_t)1 << lb, HI = pl.N >> lb;
  const size_t per = 2 * (HI + LO);
  for (int i = 0; i < 2; ++i) {
    const uint64_t* base = pt.dev + (size_t)i * per;
    tw->hi_fwd[i] = base;
    tw->lo_fwd[i] = base + HI;
    tw->hi_inv[i] = base + HI + LO;
    tw->lo_inv[i] = base + 2 * HI + LO;
    tw->scale[i] = pt.scale[i];
  }
}

// The tables of a plan's length, if they exist already (no allocation).
bool find_twiddles(const dmul_ctx* ctx, const PlanDev& pl, TwiddleSet* tw) {
  auto it = ctx->pass.find(pl.N);
  if (it == ctx->pass.end()) return false;
  set_twiddles(ctx, pl, it->second, tw);
  return true;
}

// Builds (once per length) the inter-pass factor tables of a transform of
// length N = R*C and returns pointers to them.
int get_twiddles(dmul_ctx* ctx, const PlanDev& pl, TwiddleSet* tw) {
  if (find_twiddles(ctx, pl, tw)) return DMUL_OK;
  const int lb = pass_split_bits(pl.logC, pl.rad3);
  std::vector<uint64_t> h(pass_words(pl.N, lb));
  PassTables pt;
  fill_pass_tables(pl.N, lb, h.data(), pt.scale);
  hipError_t e = hipMalloc(&pt.dev, h.size() * sizeof(uint64_t));
  if (e != hipSuccess) return from_hip(e);
  e = hipMemcpy(pt.dev, h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(pt.dev);
    return from_hip(e);
  }
  auto it = ctx->pass.emplace(pl.N, pt).first;
  set_twiddles(ctx, pl, it->second, tw);
  return DMUL_OK;
}

// Workspace of at least `words` 64-bit words (waits for queued work before
// replacing a smaller one).
int ensure_workspace(dmul_ctx* ctx, size_t words) {
  if (ctx->ws_words >= words) return DMUL_OK;
  if (ctx->budget && words * sizeof(uint64_t) > ctx->budget) return DMUL_ENOMEM;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return from_hip(e);
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_words = 0;
  e = hipMalloc(&ctx->ws, words * sizeof(uint64_t));
  if (e != hipSuccess) return from_hip(e);
  ctx->ws_words = words;
  return DMUL_OK;
}

// Status words allocated with a context: the single product's and 4096 batch products'.
constexpr size_t kStatusWords = 4097;

int ensure_status(dmul_ctx* ctx, size_t n) {
  if (ctx->status_cap >= n) return DMUL_OK;
  // grow by doubling, from room for a 4096-product batch: a larger array
  // costs a free of the old one, which waits for the whole device
  size_t cap = ctx->status_cap ? 2 * ctx->status_cap : kStatusWords;
  while (cap < n) cap *= 2;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return from_hip(e);
  int* d = nullptr;
  e = hipMalloc(&d, cap * sizeof(int));
  if (e != hipSuccess) return from_hip(e);
  e = hipMemsetAsync(d, 0, cap * sizeof(int), ctx->stream);
  // the words in use (the single product's and those of batches not yet
  // synchronised, whose work is complete after the wait above) carry over
  if (e == hipSuccess && ctx->d_status)
    e = hipMemcpyAsync(d, ctx->d_status, ctx->status_used * sizeof(int), hipMemcpyDeviceToDevice,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return from_hip(e);
  }
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  ctx->d_status = d;
  ctx->status_cap = cap;
  return DMUL_OK;
}

// Recovery sync words (a counter and one map word per workgroup) for at
// least `words` words (one carry map per recovery block, rewritten by every launch).
int ensure_rec_sync(dmul_ctx* ctx, size_t words) {
  if (ctx->rec_sync_cap >= words) return DMUL_OK;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return from_hip(e);
  if (ctx->rec_sync) (void)hipFree(ctx->rec_sync);
  ctx->rec_sync = nullptr;
  ctx->rec_sync_cap = 0;
  const size_t cap = words > 4096 ? words : 4096;
  e = hipMalloc(&ctx->rec_sync, cap * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(ctx->rec_sync, 0, cap * sizeof(uint32_t));
  if (e != hipSuccess) return from_hip(e);
  ctx->rec_sync_cap = cap;
  return DMUL_OK;
}

// N = 2^e (rad3 = 0) or 3 * 2^e (rad3 = 1), a length the planner can choose.
bool size_class(uint64_t N, int* rad3, int* e) {
  int r = 0;
  if (N % 3 == 0) { N /= 3; r = 1; }
  if (N == 0 || (N & (N - 1))) return false;
  int l = 0;
  while (((uint64_t)1 << l) < N) ++l;
  if (l > kMaxLogN || (r && (l < kMinLogN3 || l > kMaxLogR3 + kMaxLogC3))) return false;
  *rad3 = r;
  *e = l;
  return true;
}

int row_iters_for(const dmul_ctx* ctx, const PlanDev& pl) {
  const int v = ctx->tune.row_iters[pl.rad3 ? 1 : 0][pl.logN];
  return v > 0 ? v : 1;
}

bool use_small(const dmul_ctx* ctx, const PlanDev& pl, size_t count) {
  // a tuned path is a batch choice: launches of fewer products of the length
  // take the default rule
  const int path = count >= kSmallMinCount ? ctx->tune.path[pl.rad3 ? 1 : 0][pl.logN] : 0;
  if (path == 1) return pl.N <= kSmallMaxN;
  if (path == 2) return false;
  return small_fits(pl, count);
}

int side_streams_for(const dmul_ctx* ctx) {
  const int s = ctx->tune.streams;
  return s > 0 ? (s < kMaxSideStreams ? s : kMaxSideStreams) : kDefaultSideStreams;
}

static bool overlaps(const uint64_t* x, size_t nx, const uint64_t* y, size_t ny) {
  if (!nx || !ny) return false;
  const uintptr_t a0 = (uintptr_t)x, a1 = a0 + nx * 8, b0 = (uintptr_t)y, b1 = b0 + ny * 8;
  return a0 < b1 && b0 < a1;
}

int check_args(const uint64_t* a, size_t na, const uint64_t* b, size_t nb, const uint64_t* out) {
  if ((na && !a) || (nb && !b) || (na + nb && !out)) return DMUL_EINVAL;
  if (overlaps(out, na + nb, a, na) || overlaps(out, na + nb, b, nb)) return DMUL_EINVAL;
  return DMUL_OK;
}

// Enqueues one whole product; `status` is the device word its bad-limb
// check reports to.  With `residues` set, stops after the convolution and
// copies both residue vectors there instead of recovering the answer.
// The plan of a product whose operands may come as cached spectra: the plan
// of (na, nb) must have the k and transform length every given spectrum was
// made for (DMUL_EINVAL otherwise).
int spectrum_plan(int device, const dmul_spectrum* sa, size_t na, const dmul_spectrum* sb, size_t nb,
                  unsigned flags, PlanDev* pl) {
  if ((sa && sa->na != na) || (sb && sb->na != nb)) return DMUL_EINVAL;
  if ((sa && sa->device != device) || (sb && sb->device != device)) return DMUL_EINVAL;
  const int rc = make_plan(na, nb, flags, pl);
  if (rc) return rc;
  for (const dmul_spectrum* s : {sa, sb}) {
    if (s && (s->pl.k != pl->k || s->pl.N != pl->N || s->pl.logR != pl->logR || s->pl.rad3 != pl->rad3))
      return DMUL_EINVAL;
  }
  return DMUL_OK;
}

static int enqueue_one(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                       uint64_t* out, unsigned flags, int* status, uint64_t* residues,
                       const dmul_spectrum* sa, const dmul_spectrum* sb);

int enqueue_product(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                    uint64_t* out, unsigned flags, int* status, uint64_t* residues,
                    const dmul_spectrum* sa, const dmul_spectrum* sb) {
  if (ctx->timing) ctx->timing->start(ctx->stream);
  const int rc = enqueue_one(ctx, a, na, b, nb, out, flags, status, residues, sa, sb);
  if (!rc && ctx->timing) ctx->timing->done.push_back(ctx->timing->record(ctx->stream));
  return rc;
}

static int enqueue_one(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                       uint64_t* out, unsigned flags, int* status, uint64_t* residues,
                       const dmul_spectrum* sa, const dmul_spectrum* sb) {
  if (na == 0 || nb == 0) return from_hip(launch_zero(out, na + nb, ctx->stream));
  PlanDev pl;
  int rc = spectrum_plan(ctx->device, sa, na, sb, nb, flags, &pl);
  if (rc) return rc;
  TwiddleSet tw;
  rc = get_twiddles(ctx, pl, &tw);
  if (rc) return rc;
  rc = ensure_workspace(ctx, workspace_words(pl));
  if (rc) return rc;
  const bool rec_lean = recover_lean(pl);
  rc = ensure_rec_sync(ctx, recover_blocks(pl, rec_lean) + 1);
  if (rc) return rc;
  Work w{};
  ProdDesc& d = w.one;
  d.pl = pl;
  d.a = a;
  d.b = b;
  d.out = out;
  d.ws = ctx->ws;
  d.status = status;
  d.rec_sync = ctx->rec_sync;
  d.nblk = (uint32_t)recover_blocks(pl, rec_lean);
  d.square = (sa || sb) ? (sa == sb ? 1 : 0) : ((a == b && na == nb) ? 1 : 0);
  d.xs = sa ? sa->dev : nullptr;
  d.ys = sb ? sb->dev : nullptr;
  w.many = nullptr;
  w.count = 1;
  Shape sh{pl.logR, pl.logC, pl.rad3, d.square ? 0 : 1, row_iters_for(ctx, pl), d.nblk, rec_lean ? 1 : 0};
  if (ctx->poison) {
    hipError_t e = launch_fill32(ctx->ws, 2 * workspace_words(pl), kPoison, ctx->stream);
    if (e == hipSuccess) e = launch_fill32(ctx->rec_sync, d.nblk + 1, kPoison, ctx->stream);
    if (e != hipSuccess) return from_hip(e);
  }
  Marks* marks = ctx->prof;
  if (ctx->prof) ctx->prof->begin(ctx->stream);
  if (!residues && !sa && !sb && use_small(ctx, pl, 1))
    return from_hip(launch_small(w, sh, ctx->cs, tw, ctx->d_div, &ctx->h_div, ctx->stream, marks));
  hipError_t e;
  if (sa || sb) {
    e = launch_forward(w, sh, ctx->cs, tw, ctx->d_div, ctx->stream, marks);
    if (e == hipSuccess) e = launch_inverse(w, sh, ctx->cs, tw, ctx->stream, marks);
  } else {
    e = launch_fused(w, sh, ctx->cs, tw, ctx->d_div, ctx->stream, marks);
  }
  if (e != hipSuccess) return from_hip(e);
  if (residues) {
    e = hipMemcpyAsync(residues, ctx->ws, 2 * pl.N * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx->stream);
    return from_hip(e);
  }
  e = launch_recover(w, sh, ctx->cs, ctx->d_div, &ctx->h_div, ctx->stream, marks);
  return from_hip(e);
}

// The size-class tuning table: DMUL_TUNE_TABLE, else dmul_tune.txt next to
// the library.  Lines "N row_iters" ('#' starts a comment); missing or
// unreadable tables, and lines that name no size class, leave the defaults.
void load_tuning(TuneTable* t) {
  std::string path;
  if (const char* e = getenv("DMUL_TUNE_TABLE")) {
    path = e;
  } else {
    Dl_info info;
    if (dladdr((void*)&load_tuning, &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.rfind('/');
      path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/dmul_tune.txt";
    }
  }
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    unsigned long long n = 0;
    int iters = 0, path = 0, r3 = 0, e = 0, streams = 0;
    if (sscanf(line, "streams %d", &streams) == 1) {
      if (streams >= 1 && streams <= kMaxSideStreams) t->streams = streams;
      continue;
    }
    int queue = 0;
    if (sscanf(line, "queue %d", &queue) == 1) {
      if (queue == 0 || queue == 1) t->queue = queue;
      continue;
    }
    const int got = sscanf(line, "%llu %d %d", &n, &iters, &path);
    if (got >= 2 && size_class(n, &r3, &e) && iters > 0 && iters <= 64) {
      t->row_iters[r3][e] = iters;
      if (got == 3 && path >= 0 && path <= 2 && (path != 1 || n <= kSmallMaxN)) t->path[r3][e] = path;
    }
  }
  fclose(f);
}

}  // namespace dmi

namespace {
// The scratch memory of dmul_ex_noalloc: one product's workspace (4N words,
// N <= kStaticMaxN) followed by its recovery carry maps.  Every device the
// library runs on holds its own copy (64 MiB + 16 KiB) from the loading of
// this code object until the process ends.  Host code never uses this name
// as an address: scratch_address() asks the runtime for the current
// device's copy once per device and keeps it.
static __device__ __align__(256) uint64_t scratch[4 * kStaticMaxN + kStaticMapWords];

std::mutex g_scratch_mu;
std::map<int, uint64_t*> g_scratch;   // device -> its copy of scratch

// `device` must be the current device.
int scratch_address(int device, uint64_t** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return DMUL_EDEVICE;
    }
    it = g_scratch.emplace(device, (uint64_t*)p).first;
  }
  *out = it->second;
  return DMUL_OK;
}

std::mutex g_default_mu;
std::map<int, dmul_ctx*> g_default;

// A whole decimal number in [lo, hi] from the environment variable `name`:
// 1 with *v set, 0 when it is unset or empty, -1 when it is anything else.
int env_number(const char* name, unsigned long long lo, unsigned long long hi, unsigned long long* v) {
  const char* s = getenv(name);
  if (!s || !*s) return 0;
  unsigned long long x = 0;
  for (const char* q = s; *q; ++q) {
    if (*q < '0' || *q > '9' || x > (~0ULL - 9) / 10) return -1;
    x = 10 * x + (unsigned)(*q - '0');
  }
  if (x < lo || x > hi) return -1;
  *v = x;
  return 1;
}

// The flags a product of context c runs with: DMUL_FORCE_K fills in k
// where the caller's flags leave it to the library.
unsigned with_env_k(const dmul_ctx* c, unsigned flags) {
  return (flags & DMUL_FLAG_K_MASK) ? flags : (flags | c->env_k);
}

dmul_ctx* default_ctx(int device, int* rc) {
  std::lock_guard<std::mutex> lk(g_default_mu);
  auto it = g_default.find(device);
  if (it != g_default.end()) return it->second;
  dmul_ctx* c = nullptr;
  *rc = dmul_ctx_create(&c, device, 0);
  if (*rc) return nullptr;
  g_default[device] = c;
  return c;
}
}  // namespace

extern "C" {

const char* dmul_version(void) { return kLazy ? "dmul-gfx950 1.1 redundant-range" : "dmul-gfx950 1.1"; }

const char* dmul_strerror(int code) {
  switch (code) {
    case DMUL_OK: return "ok";
    case DMUL_EINVAL: return "invalid argument";
    case DMUL_EDIGIT: return "limb >= 10^19 in an operand";
    case DMUL_ERANGE: return "product outside the supported range";
    case DMUL_ENOMEM: return "workspace above budget or device allocation failed";
    case DMUL_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

void dmul_primes(uint64_t p[2], uint64_t g[2]) {
  p[0] = kP[0]; p[1] = kP[1];
  g[0] = kG[0]; g[1] = kG[1];
}

int dmul_plan(size_t na, size_t nb, unsigned flags, dmul_plan_info* info) {
  if (!info) return DMUL_EINVAL;
  PlanDev pl;
  const int rc = make_plan(na, nb, flags, &pl);
  if (rc) return rc;
  info->k = pl.k;
  info->log2_n = pl.logN;
  info->log2_rows = pl.logR;
  info->log2_cols = pl.logC;
  info->groups_a = pl.n;
  info->groups_b = pl.m;
  info->workspace_bytes = workspace_words(pl) * sizeof(uint64_t);
  info->transform_len = pl.N;
  info->factor = pl.rad3 ? 3 : 1;
  info->reserved = 0;
  return DMUL_OK;
}

size_t dmul_workspace_bytes(size_t na, size_t nb) {
  if (na == 0 || nb == 0) return 0;
  PlanDev pl;
  if (make_plan(na, nb, 0, &pl)) return 0;
  return workspace_words(pl) * sizeof(uint64_t);
}

int dmul_ctx_create(dmul_ctx** out, int device, size_t budget) {
  if (!out) return DMUL_EINVAL;
  *out = nullptr;
  // DMUL_HBM_BUDGET (bytes, 0 = no limit) stands in for a budget argument of 0;
  // DMUL_FORCE_K (kMinK..18) for the k field of flags that leave it 0
  unsigned long long env_budget = 0, env_k = 0;
  if (env_number("DMUL_HBM_BUDGET", 0, ~0ULL, &env_budget) < 0) return DMUL_EINVAL;
  if (env_number("DMUL_FORCE_K", kMinK, 18, &env_k) < 0) return DMUL_EINVAL;
  if (!check_field()) return DMUL_EDEVICE;
  const DivTable dt = make_div_table();
  if (!check_div_table(dt)) return DMUL_EDEVICE;
  DeviceGuard dg(device);
  if (!dg.ok()) return DMUL_EDEVICE;
  hipError_t e = hipSuccess;
  dmul_ctx* c = new (std::nothrow) dmul_ctx;
  if (!c) return DMUL_ENOMEM;
  c->device = device;
  c->budget = budget ? budget : (size_t)env_budget;
  c->env_k = (unsigned)env_k;
  if (const char* pv = getenv("DMUL_POISON")) c->poison = pv[0] && strcmp(pv, "0") != 0;
  c->h_div = dt;
  load_tuning(&c->tune);
  for (int i = 0; i < 2; ++i) {
    c->cs.P[i].p = kP[i];
    c->cs.P[i].p_hi = (uint32_t)(kP[i] >> 32);
  }
  c->cs.r_tilde = to_mont(inv_mod(kP[0] % kP[1], kP[1]), kP[1]);
  // root tables: for every length 2^l, l = 1..kMaxLogLen, and every stage b
  // of its butterflies, w^(i * 2^(l-1-b)) for i < 2^b (Montgomery form)
  std::vector<uint64_t> roots(4 * kRootWords);
  for (int i = 0; i < 2; ++i) {
    const uint64_t p = kP[i];
    for (int l = 1; l <= kMaxLogLen; ++l) {
      const uint64_t w = powmod(kG[i], (p - 1) >> l, p);
      const uint64_t wi = inv_mod(w, p);
      const size_t half = (size_t)1 << (l - 1);
      std::vector<uint64_t> fw(half), iw(half);    // w^e, w^-e for e < 2^(l-1)
      uint64_t x = 1, y = 1;
      for (size_t e = 0; e < half; ++e) {
        fw[e] = to_mont(x, p);
        iw[e] = to_mont(y, p);
        x = mulmod(x, w, p);
        y = mulmod(y, wi, p);
      }
      uint64_t* f = roots.data() + (size_t)(2 * i) * kRootWords + root_block_offset(l);
      uint64_t* g = roots.data() + (size_t)(2 * i + 1) * kRootWords + root_block_offset(l);
      for (int b = 0; b < l; ++b)
        for (size_t j = 0; j < ((size_t)1 << b); ++j) {
          f[root_stage_offset(b) + j] = fw[j << (l - 1 - b)];
          g[root_stage_offset(b) + j] = iw[j << (l - 1 - b)];
        }
    }
  }
  // radix-3 row tables: for every row length C = 3 * 2^l, l = 0..kMaxLogC3,
  // w_C^i (i < 2^(l+1)), forward and inverse; and the butterfly constant
  // kappa = (w - w^2) / 2 for the cube root of unity w of each direction.
  std::vector<uint64_t> r3(4 * kR3TableWords);
  for (int i = 0; i < 2; ++i) {
    const uint64_t p = kP[i];
    for (int l = 0; l <= kMaxLogC3; ++l) {
      const uint64_t w = powmod(kG[i], (p - 1) / ((uint64_t)3 << l), p);
      const uint64_t wi = inv_mod(w, p);
      uint64_t* f = r3.data() + (size_t)(2 * i) * kR3TableWords + r3_table_offset(l);
      uint64_t* g = r3.data() + (size_t)(2 * i + 1) * kR3TableWords + r3_table_offset(l);
      uint64_t x = 1, y = 1;
      for (size_t j = 0; j < ((size_t)2 << l); ++j) {
        f[j] = to_mont(x, p);
        g[j] = to_mont(y, p);
        x = mulmod(x, w, p);
        y = mulmod(y, wi, p);
      }
    }
    const uint64_t inv2 = (p + 1) / 2;
    const uint64_t w3 = powmod(kG[i], (p - 1) / 3, p);
    for (int dir = 0; dir < 2; ++dir) {
      const uint64_t w = dir ? inv_mod(w3, p) : w3;
      const uint64_t w2 = mulmod(w, w, p);
      c->cs.kappa[i][dir] = to_mont(mulmod((w + p - w2) % p, inv2, p), p);
    }
  }
  int rc = DMUL_OK;
  e = hipMalloc(&c->d_roots, roots.size() * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemcpy(c->d_roots, roots.data(), roots.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_r3, r3.size() * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemcpy(c->d_r3, r3.data(), r3.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_div, sizeof(DivTable));
  if (e == hipSuccess) e = hipMemcpy(c->d_div, &dt, sizeof(DivTable), hipMemcpyHostToDevice);
  if (e != hipSuccess) rc = from_hip(e);
  if (!rc) rc = ensure_status(c, 1);
  if (!rc) rc = prebuild_pass_tables(c);
  // without the static array's address only dmul_ex_noalloc is unavailable
  // (it then returns DMUL_EDEVICE); every other entry point works
  if (!rc && scratch_address(device, &c->scratch) != DMUL_OK) c->scratch = nullptr;

  if (rc) {
    dmul_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return DMUL_OK;
}

int dmul_ctx_destroy(dmul_ctx* c) {
  if (!c) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  (void)hipStreamSynchronize(c->stream);
  delete c->batch;
  delete c->prof;
  delete c->timing;
  for (auto& kv : c->pass)
    if (kv.second.owned) (void)hipFree(kv.second.dev);
  if (c->pass_block) (void)hipFree(c->pass_block);
  if (c->ws) (void)hipFree(c->ws);
  if (c->d_roots) (void)hipFree(c->d_roots);
  if (c->d_r3) (void)hipFree(c->d_r3);
  if (c->d_div) (void)hipFree(c->d_div);
  if (c->d_status) (void)hipFree(c->d_status);
  if (c->rec_sync) (void)hipFree(c->rec_sync);
  delete c;
  return DMUL_OK;
}

int dmul_ctx_set_stream(dmul_ctx* c, void* stream) {
  if (!c) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  if ((hipStream_t)stream == c->stream) return DMUL_OK;
  // work queued on the old stream uses the context's buffers and status
  // words: it completes before anything is enqueued on the new one
  if (hipStreamSynchronize(c->stream) != hipSuccess) return DMUL_EDEVICE;
  c->stream = (hipStream_t)stream;
  return DMUL_OK;
}

int dmul_ex(dmul_ctx* c, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
            uint64_t* out, unsigned flags) {
  if (!c) return DMUL_EINVAL;
  int rc = check_args(a, na, b, nb, out);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  rc = enqueue_product(c, a, na, b, nb, out, with_env_k(c, flags), c->d_status, nullptr);
  if (rc == DMUL_EDEVICE && c->pending == DMUL_OK) c->pending = rc;
  return rc;
}

int dmul_sync(dmul_ctx* c) {
  if (!c) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && c->prof) c->prof->collect();
  if (e == hipSuccess && c->timing) c->timing->collect();
  int rc = c->pending;
  c->pending = DMUL_OK;
  if (e != hipSuccess) rc = from_hip(e);
  const size_t n = c->status_used;
  std::vector<int> st(n, 0);
  e = hipMemcpy(st.data(), c->d_status, n * sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(c->d_status, 0, n * sizeof(int));
  if (e != hipSuccess) return from_hip(e);
  // status bit 1: a limb >= 10^19
  auto code = [](int w) { return (w & 1) ? DMUL_EDIGIT : DMUL_OK; };
  if (st[0] && rc == DMUL_OK) rc = code(st[0]);
  for (const auto& pb : c->batches) {
    for (size_t i = 0; i < pb.count; ++i)
      if (st[pb.off + i] && pb.host[i] == DMUL_OK) pb.host[i] = code(st[pb.off + i]);
  }
  c->batches.clear();
  c->status_used = 1;
  return rc;
}

int dmul(const uint64_t* a, size_t na, const uint64_t* b, size_t nb, uint64_t* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DMUL_EDEVICE;
  int rc = DMUL_OK;
  dmul_ctx* c = default_ctx(dev, &rc);
  if (!c) return rc;
  rc = dmul_ex(c, a, na, b, nb, out, 0);
  const int rs = dmul_sync(c);
  return rc ? rc : rs;
}

int dmul_host(int device, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
              uint64_t* out, unsigned flags) {
  if ((na && !a) || (nb && !b) || (na + nb && !out)) return DMUL_EINVAL;
  DeviceGuard dg(device);
  if (!dg.ok()) return DMUL_EDEVICE;
  int rc = DMUL_OK;
  dmul_ctx* c = default_ctx(device, &rc);
  if (!c) return rc;
  uint64_t *da = nullptr, *db = nullptr, *dz = nullptr;
  hipError_t e = hipMalloc(&da, (na + 1) * 8);
  if (e == hipSuccess) e = hipMalloc(&db, (nb + 1) * 8);
  if (e == hipSuccess) e = hipMalloc(&dz, (na + nb + 1) * 8);
  if (e == hipSuccess && na) e = hipMemcpy(da, a, na * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && nb) e = hipMemcpy(db, b, nb * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const bool same = (a == b && na == nb);
    rc = dmul_ex(c, da, na, same ? da : db, nb, dz, flags);
    const int rs = dmul_sync(c);
    if (!rc) rc = rs;
    if (!rc && na + nb) e = hipMemcpy(out, dz, (na + nb) * 8, hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess && !rc) rc = from_hip(e);
  if (da) (void)hipFree(da);
  if (db) (void)hipFree(db);
  if (dz) (void)hipFree(dz);
  return rc;
}

int dmul_debug_residues(dmul_ctx* c, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                        uint64_t* res, unsigned flags) {
  if (!c || !res || !na || !nb || !a || !b) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  int rc;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    // flags as given: the caller sized res from dmul_plan with the same flags
    rc = enqueue_product(c, a, na, b, nb, nullptr, flags, c->d_status, res);
  }
  const int rs = dmul_sync(c);
  return rc ? rc : rs;
}

int dmul_ex_noalloc(dmul_ctx* c, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                    uint64_t* out, unsigned flags) {
  if (!c) return DMUL_EINVAL;
  int rc = check_args(a, na, b, nb, out);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  if (na == 0 || nb == 0) return from_hip(launch_zero(out, na + nb, c->stream));
  PlanDev pl;
  rc = make_plan(na, nb, with_env_k(c, flags), &pl);
  if (rc) return rc;
  if (pl.N > kStaticMaxN) return DMUL_ENOMEM;      // beyond the static scratch
  TwiddleSet tw;
  if (!c->scratch || !find_twiddles(c, pl, &tw)) return DMUL_EDEVICE;   // built at creation
  Work w{};
  ProdDesc& d = w.one;
  d.pl = pl;
  d.a = a;
  d.b = b;
  d.out = out;
  d.ws = c->scratch;
  d.status = c->d_status;
  d.rec_sync = (uint32_t*)(c->scratch + 4 * kStaticMaxN);
  const bool rec_lean = recover_lean(pl);
  d.nblk = (uint32_t)recover_blocks(pl, rec_lean);
  d.square = (a == b && na == nb) ? 1 : 0;
  w.count = 1;
  const Shape sh{pl.logR, pl.logC, pl.rad3, d.square ? 0 : 1, row_iters_for(c, pl), d.nblk, rec_lean ? 1 : 0};
  hipError_t e = hipSuccess;
  if (c->poison) {
    e = launch_fill32(d.ws, 2 * workspace_words(pl), kPoison, c->stream);
    if (e == hipSuccess) e = launch_fill32(d.rec_sync, d.nblk + 1, kPoison, c->stream);
    if (e != hipSuccess) return from_hip(e);
  }
  if (use_small(c, pl, 1)) {
    e = launch_small(w, sh, c->cs, tw, c->d_div, &c->h_div, c->stream, nullptr);
  } else {
    e = launch_fused(w, sh, c->cs, tw, c->d_div, c->stream, nullptr);
    if (e == hipSuccess) e = launch_recover(w, sh, c->cs, c->d_div, &c->h_div, c->stream, nullptr);
  }
  rc = from_hip(e);
  if (rc == DMUL_EDEVICE && c->pending == DMUL_OK) c->pending = rc;
  return rc;
}

int dmul_ctx_tune(dmul_ctx* c, uint64_t transform_len, int row_iters) {
  int r3 = 0, e = 0;
  if (!c || !size_class(transform_len, &r3, &e) || row_iters < 0 || row_iters > 64) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.row_iters[r3][e] = row_iters;
  if (c->batch) c->batch->forget_graphs(c->stream);
  return DMUL_OK;
}

int dmul_ctx_tune_path(dmul_ctx* c, uint64_t transform_len, int path) {
  int r3 = 0, e = 0;
  if (!c || !size_class(transform_len, &r3, &e) || path < 0 || path > 2) return DMUL_EINVAL;
  if (path == 1 && transform_len > kSmallMaxN) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.path[r3][e] = path;
  if (c->batch) c->batch->forget_graphs(c->stream);
  return DMUL_OK;
}

int dmul_ctx_tune_streams(dmul_ctx* c, int streams) {
  if (!c || streams < 0 || streams > kMaxSideStreams) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.streams = streams;
  if (c->batch) c->batch->forget_graphs(c->stream);
  return DMUL_OK;
}

int dmul_ctx_tune_queue(dmul_ctx* c, int queue) {
  if (!c || (queue != 0 && queue != 1)) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.queue = queue;
  if (c->batch) c->batch->forget_graphs(c->stream);
  return DMUL_OK;
}

int dmul_ctx_profile(dmul_ctx* c, int enable) {
  if (!c) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  (void)hipStreamSynchronize(c->stream);
  delete c->prof;
  c->prof = nullptr;
  if (enable) {
    c->prof = new (std::nothrow) Profiler();
    if (!c->prof) return DMUL_ENOMEM;
  }
  return DMUL_OK;
}

int dmul_ctx_profile_read(dmul_ctx* c, double* total_ms, uint64_t* launches, int n) {
  if (!c || n < 0 || (n && (!total_ms || !launches))) return DMUL_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < n && i < kNumPhases; ++i) {
    total_ms[i] = c->prof ? c->prof->total_ms[i] : 0.0;
    launches[i] = c->prof ? c->prof->count[i] : 0;
  }
  return kNumPhases;
}

int dmul_ctx_profile_events(dmul_ctx* c, int32_t* phases, double* end_ms, int n) {
  if (!c || n < 0 || (n && (!phases || !end_ms))) return DMUL_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->prof) return 0;
  const int m = (int)c->prof->timeline.size();
  for (int i = 0; i < n && i < m; ++i) {
    phases[i] = c->prof->timeline[i].first;
    end_ms[i] = c->prof->timeline[i].second;
  }
  return m;
}

int dmul_ctx_timing(dmul_ctx* c, int enable) {
  if (!c) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  (void)hipStreamSynchronize(c->stream);
  delete c->timing;
  c->timing = nullptr;
  if (enable) {
    c->timing = new (std::nothrow) Timing();
    if (!c->timing) return DMUL_ENOMEM;
  }
  return DMUL_OK;
}

long dmul_ctx_timing_read(dmul_ctx* c, double* ms, size_t n) {
  if (!c || (n && !ms)) return DMUL_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->timing) return 0;
  const std::vector<double>& t = c->timing->last;
  for (size_t i = 0; i < n && i < t.size(); ++i) ms[i] = t[i];
  return (long)t.size();
}

const char* dmul_phase_name(int phase) {
  static const char* names[kNumPhases] = {"fwd_cols", "fwd_rows", "inv_rows", "inv_cols",
                                          "rec_crt", "rec_apply", "whole", "rows"};
  return (phase >= 0 && phase < kNumPhases) ? names[phase] : "unknown";
}

int dmul_batch_ex(dmul_ctx* c, size_t count, const uint64_t* const* a, const size_t* na,
                  const dmul_spectrum* const* sa, const uint64_t* const* b, const size_t* nb,
                  const dmul_spectrum* const* sb, uint64_t* const* out, int32_t* status,
                  unsigned flags) {
  if (!c || (count && (!a || !na || !b || !nb || !out || !status))) return DMUL_EINVAL;
  if (flags & ~(DMUL_FLAG_K_MASK | DMUL_FLAG_POW2 | DMUL_FLAG_GRAPH)) return DMUL_EINVAL;
  for (size_t i = 0; i < count; ++i) {
    const dmul_spectrum* si = sa ? sa[i] : nullptr;
    const dmul_spectrum* ti = sb ? sb[i] : nullptr;
    if ((si && si->na != na[i]) || (ti && ti->na != nb[i])) return DMUL_EINVAL;
    // an operand given by its spectrum needs no limbs
    const int rc = check_args(a[i], si ? 0 : na[i], b[i], ti ? 0 : nb[i], out[i]);
    if (rc) return rc;
    if ((si || ti) && !out[i]) return DMUL_EINVAL;
  }
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->batch) {
    c->batch = new (std::nothrow) BatchEngine();
    if (!c->batch) return DMUL_ENOMEM;
  }
  // this batch's status words follow those of the batches not yet synchronised
  const size_t off = c->status_used;
  int rc = ensure_status(c, off + count);
  if (rc) return rc;
  try {
    c->batches.push_back({status, off, count});
  } catch (const std::bad_alloc&) {
    return DMUL_ENOMEM;
  }
  c->status_used = off + count;
  for (size_t i = 0; i < count; ++i) status[i] = DMUL_OK;
  rc = c->batch->run(c, count, a, na, sa, b, nb, sb, out, status, with_env_k(c, flags), c->d_status + off);
  if (rc == DMUL_EDEVICE && c->pending == DMUL_OK) c->pending = rc;
  return rc;
}

int dmul_batch(dmul_ctx* c, size_t count, const uint64_t* const* a, const size_t* na,
               const uint64_t* const* b, const size_t* nb, uint64_t* const* out,
               int32_t* status, unsigned flags) {
  return dmul_batch_ex(c, count, a, na, nullptr, b, nb, nullptr, out, status, flags);
}

size_t dmul_spectrum_bytes(size_t na, size_t nb, unsigned flags) {
  PlanDev pl;
  if (na == 0 || nb == 0 || make_plan(na, nb, flags & (DMUL_FLAG_K_MASK | DMUL_FLAG_POW2), &pl)) return 0;
  return 2 * (size_t)pl.N * sizeof(uint64_t);
}

int dmul_spectrum_create(dmul_ctx* c, const uint64_t* a, size_t na, size_t nb, unsigned flags,
                         void* mem, size_t mem_bytes, dmul_spectrum** out) {
  if (!c || !out) return DMUL_EINVAL;
  *out = nullptr;
  if (!a || na == 0 || nb == 0) return DMUL_EINVAL;
  flags = with_env_k(c, flags);
  PlanDev pl;
  int rc = make_plan(na, nb, flags, &pl);
  if (rc) return rc;
  const size_t bytes = 2 * (size_t)pl.N * sizeof(uint64_t);
  if (mem && (mem_bytes < bytes || ((uintptr_t)mem & 7))) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  TwiddleSet tw;
  rc = get_twiddles(c, pl, &tw);
  if (rc) return rc;
  dmul_spectrum* s = new (std::nothrow) dmul_spectrum;
  if (!s) return DMUL_ENOMEM;
  s->device = c->device;
  s->na = na;
  s->flags = flags;
  s->pl = pl;
  hipError_t e = hipSuccess;
  if (mem) {
    s->dev = (uint64_t*)mem;
  } else {
    e = hipMalloc(&s->dev, bytes);
    s->owned = true;
  }
  if (e != hipSuccess) {
    delete s;
    return from_hip(e);
  }
  // the forward passes of a squared product transform one operand into the
  // first 2N words of the workspace: here, the spectrum's own buffer
  Work w{};
  ProdDesc& d = w.one;
  d.pl = pl;
  d.a = a;
  d.b = a;
  d.ws = s->dev;
  d.status = c->d_status;
  d.square = 1;
  w.count = 1;
  const Shape sh{pl.logR, pl.logC, pl.rad3, 0, row_iters_for(c, pl), 0, 0};
  e = launch_forward(w, sh, c->cs, tw, c->d_div, c->stream, nullptr);
  if (e != hipSuccess) {
    if (s->owned) (void)hipFree(s->dev);
    delete s;
    if (c->pending == DMUL_OK) c->pending = DMUL_EDEVICE;
    return from_hip(e);
  }
  *out = s;
  return DMUL_OK;
}

int dmul_spectrum_destroy(dmul_spectrum* s) {
  if (!s) return DMUL_EINVAL;
  DeviceGuard dg(s->device);
  if (s->dev && s->owned) (void)hipFree(s->dev);
  delete s;
  return DMUL_OK;
}

int dmul_spectrum_export(dmul_ctx* c, const dmul_spectrum* s, uint64_t* out) {
  if (!c || !s || !out || s->device != c->device) return DMUL_EINVAL;
  if (s->pl.rad3 || s->pl.logR < 5) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  const uint64_t N = s->pl.N;
  hipError_t e = hipMemcpyAsync(out, s->dev, 2 * N * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return from_hip(e);
  for (int pi = 0; pi < 2; ++pi) {
    const int rc = transpose_inplace(out + pi * N, (uint64_t)1 << s->pl.logR, (uint64_t)1 << s->pl.logC,
                                     true, c->stream);
    if (rc) return rc;
  }
  return DMUL_OK;
}

int dmul_debug_transpose(dmul_ctx* c, uint64_t* data, size_t rows, size_t cols) {
  if (!c || !data) return DMUL_EINVAL;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  return transpose_inplace(data, rows, cols, false, c->stream);
}

int dmul_ex_spectrum(dmul_ctx* c, const dmul_spectrum* sa, const uint64_t* b, size_t nb,
                     const dmul_spectrum* sb, uint64_t* out, unsigned flags) {
  if (!c || !sa || !out) return DMUL_EINVAL;
  if (sb) {
    if (b || nb != sb->na) return DMUL_EINVAL;
  } else {
    const int rc = check_args(nullptr, 0, b, nb, out);
    if (rc) return rc;
  }
  DeviceGuard dg(c->device);
  if (!dg.ok()) return DMUL_EDEVICE;
  std::lock_guard<std::mutex> lk(c->mu);
  const int rc = enqueue_product(c, nullptr, sa->na, b, nb, out, with_env_k(c, flags), c->d_status, nullptr, sa, sb);
  if (rc == DMUL_EDEVICE && c->pending == DMUL_OK) c->pending = rc;
  return rc;
}

}  // extern "C"
