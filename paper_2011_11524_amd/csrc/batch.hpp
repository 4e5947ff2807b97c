// Batched products (dmul_batch): products are grouped by transform length
// (a size class) and every phase of a class runs as one launch over all of
// its products, each workgroup finding its product by blockIdx.z.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <vector>

#include <dmul.h>

#include "internal.hpp"
#include "ctx.hpp"

struct dmul_ctx;

namespace dmi {

class BatchEngine {
 public:
  ~BatchEngine();
  // Enqueues `count` products on the context's stream; status_dev[i] is the
  // device word product i reports to.  Host-side errors go to status[i].
  // Captured graphs bake in launch parameters: drop them when those change
  // (after the work queued on st, which may still run them, is done).
  void forget_graphs(hipStream_t st) {
    (void)hipStreamSynchronize(st);
    drop_graphs();
  }
  int run(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
          const dmul_spectrum* const* sa, const uint64_t* const* b, const size_t* nb,
          const dmul_spectrum* const* sb, uint64_t* const* out, int32_t* status,
          unsigned flags, int* status_dev);

 private:
  int reserve(dmul_ctx* ctx, size_t ws_words, size_t sync_words, size_t ndesc);
  void drop_graphs();

  // Captured batches, by a hash of everything the launches depend on; a
  // replay also needs the whole key to match.
  struct Graph {
    hipGraphExec_t exec = nullptr;
    ProdDesc* descs = nullptr;      // the batch's own descriptor copy
    std::vector<uint64_t> key;
  };
  std::map<uint64_t, Graph> graphs_;

  // Side streams: the size classes of a batch are independent (own
  // workspaces, descriptors and status words), so they are dealt to these
  // streams, forked from and joined back to the context stream by events,
  // and run concurrently instead of one after another.  How many are used
  // is a tuned parameter (default 8: a class of a few short products is a
  // chain of small, latency-bound launches).
  static constexpr int kSideStreams = kMaxSideStreams;
  int ensure_side_streams();
  hipStream_t side_[kSideStreams] = {};
  hipEvent_t fork_ = nullptr;
  hipEvent_t join_[kSideStreams] = {};

  uint64_t* ws_ = nullptr;          // per-product workspaces, back to back
  size_t ws_words_ = 0;
  uint32_t* sync_ = nullptr;        // per-product recovery carry maps
  size_t sync_words_ = 0;
  ProdDesc* d_desc_ = nullptr;      // descriptors on the device
  ProdDesc* h_desc_ = nullptr;      // pinned staging copy
  size_t desc_cap_ = 0;
  hipEvent_t copied_ = nullptr;     // the staging copy has been consumed
  int device_ = -1;
};

}  // namespace dmi
