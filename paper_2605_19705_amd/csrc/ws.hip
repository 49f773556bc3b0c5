// Warm-start encoder-decoder x0 = y + W_phi(y) (placeholder).
#include "ctx.h"

struct idq_ws {
  int device = 0;
};

namespace idq {
int ws_forward_internal(idq_ws*, const void*, void*, int, int, int, int, int, hipStream_t) {
  return fail(IDQ_E_UNSUPPORTED, "warm start not built yet");
}
}  // namespace idq

extern "C" {
int idq_ws_create(idq_ws** out, const double*, long long, int) {
  if (out) *out = nullptr;
  return idq::fail(IDQ_E_UNSUPPORTED, "warm start not built yet");
}
int idq_ws_destroy(idq_ws*) { return IDQ_OK; }
long long idq_ws_num_params(void) { return 0; }
int idq_ws_get_params(idq_ws*, double*) { return IDQ_E_UNSUPPORTED; }
int idq_ws_set_params(idq_ws*, const double*) { return IDQ_E_UNSUPPORTED; }
int idq_ws_forward(idq_ws*, const void*, void*, int, int, int, int, int, void*) { return IDQ_E_UNSUPPORTED; }
int idq_ws_train_step(idq_ws*, const void*, const void*, int, int, int, int, int, double, double*, void*) {
  return IDQ_E_UNSUPPORTED;
}
int idq_ws_grad(idq_ws*, const void*, const void*, void*, int, int, int, int, int, double*, void*) {
  return IDQ_E_UNSUPPORTED;
}
}
