// Allocation-free variant of idq_grad_data for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// The two-pass blur gradient J_A^T (A(x) - y) stages its intermediate image
// (A x - y, or the tanh-weighted residual) in a scratch buffer.  Here that
// buffer is a fixed file-scope device array, one per GPU, held until the
// process ends.  Its device address is resolved once per device, with that
// device current, when a context is created there; host code passes that
// address, never the array's name, to the kernels.
#include <mutex>

#include "ctx.h"

namespace idq {

static __device__ __align__(256) unsigned char scratch[IDQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(IDQ_E_INVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[device]) return IDQ_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(IDQ_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return IDQ_OK;
}

namespace {
void* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

}  // namespace idq

using namespace idq;

extern "C" int idq_grad_data_noalloc(idq_ctx* ctx, const void* x, const void* y, void* grad,
                                     int n, int c, int h, int w, int dtype, void* stream) {
  try {
    if (!ctx || !x || !y || !grad) return fail(IDQ_E_INVAL, "null argument");
    if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
    IDQ_HIP(hipSetDevice(ctx->device));
    Geometry g;
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long cnt = static_cast<long long>(n) * g.per;
    if (ctx->op_kind == IDQ_OP_IDENTITY)  // grad f = x - y: no intermediate image
      return launch_axpbypcz(1.0, x, -1.0, y, 0.0, nullptr, grad, cnt, dtype, s);
    if (ctx->op_kind == IDQ_OP_INPAINT || ctx->op_kind == IDQ_OP_RICIAN) {  // pixelwise
      DatafitArgs d{};
      d.mode = ctx->op_kind == IDQ_OP_INPAINT ? D_MASK_GRAD : D_RICIAN_GRAD;
      d.count = cnt;
      d.plane = static_cast<long long>(h) * w;
      d.x = x;
      d.y = y;
      d.mask = ctx->mask_dev[dtype == IDQ_F64 ? 0 : 1];
      d.out = grad;
      d.inv_s2 = ctx->sigma > 0.0 ? 1.0 / (ctx->sigma * ctx->sigma) : 0.0;
      return launch_datafit(d, dtype, s);
    }
    if (ctx->op_kind != IDQ_OP_BLUR_CIRC && ctx->op_kind != IDQ_OP_TANH_BLUR)
      return fail(IDQ_E_UNSUPPORTED, "idq_grad_data_noalloc: operator without a stencil gradient");
    const size_t bytes = static_cast<size_t>(cnt) * elem_size(dtype);
    if (bytes > static_cast<size_t>(IDQ_NOALLOC_SCRATCH_BYTES))
      return fail(IDQ_E_INVAL, "idq_grad_data_noalloc: " + std::to_string(bytes) +
                                   " bytes of intermediate image exceed the fixed scratch of " +
                                   std::to_string(static_cast<long long>(IDQ_NOALLOC_SCRATCH_BYTES)) +
                                   " bytes");
    void* tmp = scratch_of(ctx->device);
    if (!tmp) {  // a context is created with its device current, which resolves it
      IDQ_TRY(noalloc_init_device(ctx->device));
      tmp = scratch_of(ctx->device);
    }
    StencilArgs a = stencil_base(ctx, g, nullptr);
    a.in0 = x;
    a.aux = y;
    a.out = tmp;
    a.mode = ctx->op_kind == IDQ_OP_BLUR_CIRC ? S_B_MINUS : S_TANH_WRES;
    IDQ_TRY(launch_stencil(a, ctx->taps.data(), dtype, s));
    StencilArgs b = stencil_base(ctx, g, nullptr);
    b.in0 = tmp;
    b.out = grad;
    b.mode = S_BT;
    return launch_stencil(b, ctx->taps.data(), dtype, s);
  } catch (...) {
    return fail(IDQ_E_INVAL, "unexpected exception");
  }
}
