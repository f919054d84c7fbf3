// batch.hip -- uneven batch in one persistent launch (work in progress).
#include "corrx_internal.h"

struct corrx_batch {
  int n;
};

extern "C" {
int corr_batch_create(const corrx_desc*, int, int, const int*, corrx_batch_t* out) {
  if (out) *out = nullptr;
  return CORRX_EUNSUPPORTED;
}
int corr_batch_destroy(corrx_batch_t b) {
  delete b;
  return CORRX_OK;
}
int64_t corr_batch_items(corrx_batch_t b) { return b ? 0 : CORRX_EINVAL; }
int corr_batch_xmac(corrx_batch_t, const void* const*, void* const*, void*) { return CORRX_EUNSUPPORTED; }
}
