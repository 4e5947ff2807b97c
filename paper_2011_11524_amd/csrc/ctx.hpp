// Context object shared by the host-side pieces of the library.
#pragma once
#include <map>
#include <mutex>
#include <vector>

#include <dmul.h>

#include "internal.hpp"

namespace dmi {
class BatchEngine;
// Launch parameters per transform length N = 2^e ([0][e]) or 3 * 2^e
// ([1][e]), and for batches, from the size-class tuner (a text table: lines
// "N row_iters [path]" and "streams S"), or defaults (0).
struct TuneTable {
  int row_iters[2][kMaxLogN + 1] = {};
  int path[2][kMaxLogN + 1] = {};   // 0 the default rule, 1 whole-product kernel, 2 pass kernels
  int streams = 0;                  // side streams of a batch's classes (0: kDefaultSideStreams)
  int queue = 0;                    // 1: whole-product classes of a batch share persistent launches
};
constexpr int kMaxSideStreams = 16;
constexpr int kDefaultSideStreams = 8;
struct PassTables {
  uint64_t scale[2] = {};     // R^2 N^-1 mod p per prime
  uint64_t* dev = nullptr;   // per prime: hi_fwd[N >> lb] lo_fwd[2^lb] hi_inv[N >> lb] lo_inv[2^lb]
  bool owned = true;         // dev is its own allocation (not part of the prebuilt block)
};

// Per-kernel event timing (dmul_ctx_profile): an event before the first
// kernel of a product and one after every kernel; durations are collected
// at dmul_sync.
struct Profiler : Marks {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  size_t last = 0;
  struct Span { int phase; size_t a, b; };
  std::vector<Span> spans;
  double total_ms[kNumPhases] = {};
  uint64_t count[kNumPhases] = {};

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(hipStream_t st) {
    last = used;
    hipEvent_t e = next();
    if (e) (void)hipEventRecord(e, st);
  }
  void mark(int phase, hipStream_t st) override {
    const size_t i = used;
    hipEvent_t e = next();
    if (!e) return;
    (void)hipEventRecord(e, st);
    spans.push_back({phase, last, i});
    last = i;
  }
  // (phase, end time in ms since the first event) of every kernel of the
  // work completed by the last dmul_sync
  std::vector<std::pair<int, double>> timeline;
  void collect() {
    timeline.clear();
    for (const Span& s : spans) {
      float ms = 0.f, t = 0.f;
      if (hipEventElapsedTime(&ms, pool[s.a], pool[s.b]) == hipSuccess) {
        total_ms[s.phase] += ms;
        count[s.phase] += 1;
      }
      if (hipEventElapsedTime(&t, pool[0], pool[s.b]) == hipSuccess) timeline.push_back({s.phase, t});
    }
    spans.clear();
    used = 0;
  }
  ~Profiler() override {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Completion timing (dmul_ctx_timing): one event when the first work after a
// dmul_sync is enqueued, and one event per completed unit of work -- after
// each dmul_ex product, and after each size class of a batch on the stream
// that class runs on -- so the per-product completion times describe the
// same concurrent schedule that runs without timing.
struct Timing {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<size_t> done;       // per product since the last sync: its completion event
  std::vector<double> last;       // ms after the start event, work completed by the last sync

  size_t record(hipStream_t st) {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return SIZE_MAX;
      pool.push_back(e);
    }
    if (hipEventRecord(pool[used], st) != hipSuccess) return SIZE_MAX;
    return used++;
  }
  // the start event, recorded before the first work since the last sync
  void start(hipStream_t st) {
    if (used == 0) (void)record(st);
  }
  void collect() {
    last.assign(done.size(), -1.0);
    for (size_t i = 0; i < done.size(); ++i) {
      float ms = 0.f;
      if (done[i] < used && hipEventElapsedTime(&ms, pool[0], pool[done[i]]) == hipSuccess) last[i] = ms;
    }
    done.clear();
    used = 0;
  }
  ~Timing() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
}  // namespace dmi

using dmi::Consts;
using dmi::DivTable;

struct dmul_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  Consts cs{};
  DivTable* d_div = nullptr;
  DivTable h_div{};                     // host copy of the power-of-ten reciprocals
  uint64_t* d_roots = nullptr;          // [prime][dir] regions of kRootWords words (per-stage root tables)
  uint64_t* d_r3 = nullptr;             // [prime][dir] blocks of kR3TableWords words
  std::map<uint64_t, dmi::PassTables> pass; // by N
  uint64_t* pass_block = nullptr;       // the tables of every length up to kStaticMaxN, built at creation
  uint64_t* scratch = nullptr;          // this device's static scratch array (dmul_ex_noalloc)
  uint64_t* ws = nullptr;
  size_t ws_words = 0;
  int* d_status = nullptr;              // [0]: dmul_ex; then one region per batch since dmul_sync
  size_t status_cap = 0;
  size_t status_used = 1;               // words in use: [0] and every pending batch's region
  int pending = DMUL_OK;
  // batches enqueued since the last dmul_sync: each reports to its own words
  // d_status[off .. off + count), copied into its host array at dmul_sync
  struct PendingBatch { int32_t* host; size_t off, count; };
  std::vector<PendingBatch> batches;
  dmi::BatchEngine* batch = nullptr;
  dmi::Profiler* prof = nullptr;
  dmi::Timing* timing = nullptr;
  uint32_t* rec_sync = nullptr;         // recovery: one carry map per block
  size_t rec_sync_cap = 0;
  dmi::TuneTable tune;                  // per transform length launch parameters
  bool poison = false;                  // DMUL_POISON: fill scratch with 0xff before every product
  unsigned env_k = 0;                   // DMUL_FORCE_K: k of products whose flags name none (0: choose)
  std::mutex mu;
};

// Cached forward transforms of one operand (both primes) for one plan.
struct dmul_spectrum {
  int device = 0;
  size_t na = 0;                 // limbs of the operand
  unsigned flags = 0;            // planning flags it was made with
  dmi::PlanDev pl{};             // the plan (k, N, layout) it is valid for
  uint64_t* dev = nullptr;       // 2N words: transform mod p1, then mod p2
  bool owned = false;            // dev is the library's allocation
};

namespace dmi {
// Makes `device` current for the scope of an entry point and gives the
// caller back its own current device afterwards: a context's work goes to
// the context's device whatever device the calling thread has selected.
class DeviceGuard {
 public:
  explicit DeviceGuard(int device) {
    if (hipGetDevice(&prev_) != hipSuccess) {
      err_ = hipErrorInvalidDevice;
      return;
    }
    if (prev_ != device) {
      err_ = hipSetDevice(device);
      changed_ = err_ == hipSuccess;
      // the failed call's error must not surface at the next launch check
      if (!changed_) (void)hipGetLastError();
    }
  }
  ~DeviceGuard() {
    if (changed_) (void)hipSetDevice(prev_);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
  bool ok() const { return err_ == hipSuccess; }

 private:
  int prev_ = 0;
  bool changed_ = false;
  hipError_t err_ = hipSuccess;
};

int make_plan(size_t na, size_t nb, unsigned flags, PlanDev* pl);
size_t workspace_words(const PlanDev& pl);
int get_twiddles(dmul_ctx* ctx, const PlanDev& pl, TwiddleSet* tw);
bool find_twiddles(const dmul_ctx* ctx, const PlanDev& pl, TwiddleSet* tw);
int prebuild_pass_tables(dmul_ctx* ctx);
int layout_logR(int e, int rad3);
// rows x cols -> cols x rows in place on `stream` (transpose.hip); with
// bitrev, the row order and the columns of every row bit-reversed first.
int transpose_inplace(uint64_t* data, uint64_t rows, uint64_t cols, bool bitrev, hipStream_t stream);
int ensure_workspace(dmul_ctx* ctx, size_t words);
int ensure_rec_sync(dmul_ctx* ctx, size_t words);
int row_iters_for(const dmul_ctx* ctx, const PlanDev& pl);
// Whether `count` products of plan pl launched together take the
// whole-product kernel: the tuned path of their length, else small_fits.
bool use_small(const dmul_ctx* ctx, const PlanDev& pl, size_t count);
int side_streams_for(const dmul_ctx* ctx);
bool size_class(uint64_t N, int* rad3, int* e);
int from_hip(hipError_t e);
int enqueue_product(dmul_ctx* ctx, const uint64_t* a, size_t na, const uint64_t* b, size_t nb,
                    uint64_t* out, unsigned flags, int* status, uint64_t* residues,
                    const dmul_spectrum* sa = nullptr, const dmul_spectrum* sb = nullptr);
// Plan of a product on `device` whose operands may be spectra: DMUL_EINVAL
// when a spectrum belongs to another device, length or plan.
int spectrum_plan(int device, const dmul_spectrum* sa, size_t na, const dmul_spectrum* sb, size_t nb,
                  unsigned flags, PlanDev* pl);
}  // namespace dmi
