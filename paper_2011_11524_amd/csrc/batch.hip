// Batched products: every product goes through the same kernels as a
// single product, one after another on the context's stream.
#include <dmul.h>

#include "batch.hpp"
#include "ctx.hpp"

namespace dmi {

int BatchEngine::run(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
                     const uint64_t* const* b, const size_t* nb, uint64_t* const* out,
                     int32_t* status, unsigned flags, int* status_dev) {
  for (size_t i = 0; i < count; ++i) {
    const int rc = enqueue_product(ctx, a[i], na[i], b[i], nb[i], out[i], flags, status_dev + i, nullptr);
    if (rc) status[i] = rc;
    if (rc == DMUL_EDEVICE) return rc;
  }
  return DMUL_OK;
}

}  // namespace dmi
