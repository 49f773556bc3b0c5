// Internal context of the i-DEQ library: network, operator, packed weights and
// a grow-only device workspace.
#pragma once

#include <vector>

#include "kernels.h"

namespace idq {

// Workspace slots.  Each slot is one device allocation that only grows.
enum Slot {
  W_X0, W_X1, W_Z, W_GF, W_S, W_Q, W_R, W_RD, W_T, W_HG, W_HF, W_V, W_W, W_U, W_UP, W_UN,
  W_PART, W_STATE, W_GATE, W_BETA, W_SCAL, W_WGPART, W_TMP0, W_TMP1, W_HIST, W_ZSUM, W_XHAT,
  W_CPLX, W_ATY, W_PROX,             // FFT work buffer, A^T y, proximal-step output
  W_PW, W_TRV, W_TRD,                // adjoint J_P w; training: dL/dx_hat, x_hat - x*
  W_H0,                              // W_H0 + l     : h_{l+1}         (l < L-1)
  W_HD0 = W_H0 + IDQ_MAX_LAYERS,     // W_HD0 + l    : h'_{l+1}
  W_DL0 = W_HD0 + IDQ_MAX_LAYERS,    // W_DL0 + l    : delta_{l+1}
  W_DDL0 = W_DL0 + IDQ_MAX_LAYERS,   // W_DDL0 + l   : delta'_{l+1}
  W_NSLOTS = W_DDL0 + IDQ_MAX_LAYERS
};

struct Workspace {
  void* ptr[W_NSLOTS] = {};
  size_t cap[W_NSLOTS] = {};
  int get(int slot, size_t bytes, void** out);
  void release();
};

struct LayerW {
  int ci = 0, co = 0;
  // per precision (IDQ_F64/F32/BF16/BF16X3): direct forward and transposed
  // weights [co][ci][9] / [ci][co][9] in the math type, bias [co], MFMA-packed
  // copies (BF16X3: MFMA copies and bias only).
  void* fwd[kNumPrec] = {};
  void* tr[kNumPrec] = {};
  void* bias[kNumPrec] = {};
  void* fwd_mfma[kNumPrec] = {};
  void* tr_mfma[kNumPrec] = {};
};

// Optional device-time accounting of kernel classes (HIP events around launches).
enum ProfClass { PC_CONV_WIDE_BF16 = 0, PC_CONV_WIDE_F32 = 1, PC_CONV_OTHER = 2, PC_STENCIL = 3,
                 PC_UPDATE = 4, PC_WARMSTART = 5,
                 PC_CONV_WIDE_SPLIT = 6, PC_COUNT = 7 };
struct ProfRec {
  int cls;
  hipEvent_t e0, e1;
};
struct Profiler {
  bool on = false;
  unsigned mask = 0;   // classes timed while on (bit cls)
  bool timed(int cls) const { return on && ((mask >> cls) & 1u); }
  int every = 1;                   // time one launch in `every` of each class
  long long seen[PC_COUNT] = {};   // launches of each class since the enable
  bool sample(int cls) { return timed(cls) && (seen[cls]++ % every) == 0; }
  std::vector<hipEvent_t> pool;
  std::vector<ProfRec> pending;
  double ms[PC_COUNT] = {};
  long long launches[PC_COUNT] = {};
  unsigned long long* dev_px = nullptr;  // device counters, one per class
  int take(int cls, ProfRec* r);                   // events only
  int begin(int cls, hipStream_t s, ProfRec* r);   // take + record the start
  int end(ProfRec& r, hipStream_t s);
  int flush();
  void release();
};

struct Geometry {
  int n, c, h, w;      // solver images
  int NI, img_div;     // net images and the net-image -> image divisor
  long long per;       // c * h * w
  long long pix() const { return static_cast<long long>(NI) * h * w; }
};

}  // namespace idq

struct idq_ctx {
  int device = 0;
  int L = 0, act = IDQ_ACT_SOFTPLUS;
  int ch[IDQ_MAX_LAYERS + 1] = {};
  std::vector<double> params;
  std::vector<idq::LayerW> layers;
  int op_kind = IDQ_OP_IDENTITY, kh = 0, kw = 0;
  double gain = 2.0;
  std::vector<double> taps;
  // pixel (inpainting) or k-space (MRI) mask, mh x mw, on the device in float64
  // [IDQ_F64] and float32 [IDQ_F32]; for MRI also the symmetrised mask M_s
  int mh = 0, mw = 0;
  void* mask_dev[2] = {};
  void* msym_dev[2] = {};
  double sigma = 0.0;          // Rician sigma_y
  // |k^|^2 of the blur on a spec_h x spec_w grid (Fourier proximal step)
  void* spec_dev[2] = {};
  int spec_h[2] = {}, spec_w[2] = {};
  idq::Workspace ws;
  hipStream_t gstream = nullptr;  // graph capture / replay (created on first use)
  hipEvent_t gev[2] = {};
  int* host_gate = nullptr;  // pinned, for polling
  int host_gate_cap = 0;
  idq::Profiler prof;
};

namespace idq {
// Shape check of an entry point's image tensors (api.hip).
int check_shape(const idq_ctx* ctx, int n, int c, int h, int w, Geometry* g);
// Stencil arguments of the context's forward operator for a geometry (api.hip).
StencilArgs stencil_base(const idq_ctx* ctx, const Geometry& g, const int* gate);
// Resolves the device address of the fixed scratch array of the
// allocation-free entry points on the current device (noalloc.hip).
int noalloc_init_device(int device);
// The solver, the backward, the weight packing and a float64 batch dot product
// (api.hip), for the training loop (train.hip).
int solve_internal(idq_ctx* ctx, const void* y, const void* x0, void* x_out, int n, int c, int h,
                   int w, int dtype, const idq_solve_opts* o, idq_solve_info* info,
                   hipStream_t s);
int backward_internal(idq_ctx* ctx, const void* xbar, const void* y, const void* v, void* dtheta,
                      double* dlambda, int n, int c, int h, int w, int dtype,
                      const idq_bwd_opts* o, idq_bwd_info* info, hipStream_t s);
int repack_weights(idq_ctx* ctx);
int dot_batch(idq_ctx* ctx, const void* a, const void* b, long long count, int dtype, double* out,
              hipStream_t s);
}  // namespace idq
