// Batched products (dmul_batch).
#pragma once
#include <stddef.h>
#include <stdint.h>

struct dmul_ctx;

namespace dmi {

class BatchEngine {
 public:
  // Enqueues `count` products on the context's stream; status_dev[i] is the
  // device word product i reports a bad limb to.
  int run(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
          const uint64_t* const* b, const size_t* nb, uint64_t* const* out, int32_t* status,
          unsigned flags, int* status_dev);
};

}  // namespace dmi
