// Stateless fused LNCC cost and gradient (include/fa_lncc.h): the gradient
// kernel of the registration iteration in its gradient-only and loss-only
// modes, with its own control block, reduction buffers and padded copy of the
// moving image (fa_lncc_eval), or with those in a fixed device array of the
// library (fa_lncc_eval_noalloc).
#include <mutex>
#include <new>

#include "fa_host.h"
#include "fa_lncc.h"

using fa::fail;

// ---- allocation-free evaluation (fa_lncc_eval_noalloc) ----------------------
// Every buffer the evaluation needs besides the caller's inputs and outputs
// lives in this array: the control block, the loss partials of the gradient
// launch, the partials of the two mean reductions and the zero-bordered copy
// of the moving image.  Each GPU holds its own copy, at its own address, from
// the library's load until the process ends.  In host code the name is only a
// host-side stand-in for the symbol: kernels and copies take the device
// address kept in g_scratch_dev below, never the name.
static __device__ __align__(256) unsigned char scratch[FA_LNCC_NOALLOC_SCRATCH_BYTES];

struct fa_lncc_s {
  hipStream_t stream = nullptr;
  fa_shape shape{};
  int64_t n = 0;
  int window = 5;
  float eps = 1e-5f;
  fa::Tiling tg{};
  fa::Ctl* ctl = nullptr;
  double* partials = nullptr;   // one per workgroup of the gradient launch
  double* mean_partials = nullptr;  // kMeanBlocks doubles for the intensity means
  float* moving_pad = nullptr;  // the moving image with a zero border, refreshed per call
  float* moving_quad = nullptr; // the same as corner quads (NULL where quad_supported fails)
};

namespace {

void release(fa_lncc h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->ctl) (void)hipFree(h->ctl);
  if (h->partials) (void)hipFree(h->partials);
  if (h->mean_partials) (void)hipFree(h->mean_partials);
  if (h->moving_pad) (void)hipFree(h->moving_pad);
  if (h->moving_quad) (void)hipFree(h->moving_quad);
  delete h;
}

// Per-device address of `scratch` (fa_lncc_eval_noalloc).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device address of `scratch` on the current device, looked up once per device
// with that device current.
fa_status scratch_address(void** out) {
  int dev = -1;
  FA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FA_EHIP, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FA_OK;
}

}  // namespace

extern "C" {

fa_status fa_lncc_create(fa_shape shape, int window, float cc_eps, void* hip_stream, fa_lncc* out) {
  if (!out) return fail(FA_EINVAL, "out is NULL");
  *out = nullptr;
  FA_TRY(fa::check_shape(shape));
  if (window < 1 || window > fa::kMaxWindow || window % 2 == 0)
    return fail(FA_EINVAL, "window must be odd and in [1, 9]");
  if (!(cc_eps >= 0.0f) || !(cc_eps < 1e30f)) return fail(FA_EINVAL, "cc_eps must be finite and >= 0");
  fa_lncc h = new (std::nothrow) fa_lncc_s();
  if (!h) return fail(FA_ENOMEM, "host allocation failed");
  h->stream = (hipStream_t)hip_stream;
  h->shape = shape;
  h->n = fa::voxels(shape);
  h->window = window;
  h->eps = cc_eps;
  h->tg = fa::choose_tiling(shape, fa::KIND_GRAD, fa::Tuning(), fa::grad_cube_supported(window));
  const int nb = h->tg.blocks();
  if (hipMalloc((void**)&h->ctl, sizeof(fa::Ctl)) != hipSuccess ||
      hipMalloc((void**)&h->partials, (size_t)nb * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->mean_partials, (size_t)fa::kMeanBlocks * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->moving_pad, (size_t)fa::padded_voxels(shape.n0, shape.n1, shape.n2) * sizeof(float)) !=
          hipSuccess) {
    (void)hipGetLastError();
    release(h);
    return fail(FA_ENOMEM, "device allocation failed");
  }
  // the gradient kernel samples the corner quads (two 16-byte loads per
  // trilinear sample instead of eight 4-byte gathers) where they fit
  if (fa::quad_supported(shape.n0, shape.n1, shape.n2) &&
      hipMalloc((void**)&h->moving_quad,
                (size_t)4 * fa::padded_voxels(shape.n0, shape.n1, shape.n2) * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    release(h);
    return fail(FA_ENOMEM, "device allocation failed");
  }
  const hipError_t e = fa::launch_ctl_init(h->ctl, 0.9f, 0.999f, 0, 0, h->stream);
  if (e != hipSuccess) {
    release(h);
    return fail(FA_EHIP, std::string("launch_ctl_init: ") + hipGetErrorString(e));
  }
  *out = h;
  return FA_OK;
}

fa_status fa_lncc_eval(fa_lncc h, const float* fixed, const float* moving, const float* d,
                       float* loss_dev, float* grad_dev, const float* grad_scale_dev) {
  if (!h) return fail(FA_EINVAL, "evaluator is NULL");
  if (!fixed || !moving || !d) return fail(FA_EINVAL, "fixed, moving and d must not be NULL");
  if (!loss_dev && !grad_dev) return fail(FA_EINVAL, "loss_dev and grad_dev are both NULL");
  // global intensity means: LNCC is invariant to a global shift of either
  // image, and removing it keeps the fp32 window variances well conditioned
  FA_HIP(fa::launch_mean(fixed, h->n, h->mean_partials, &h->ctl->shift_i, h->stream));
  FA_HIP(fa::launch_mean(moving, h->n, h->mean_partials, &h->ctl->shift_j, h->stream));
  FA_HIP(fa::launch_pad(moving, h->moving_pad, h->shape.n0, h->shape.n1, h->shape.n2, h->stream));
  if (h->moving_quad)
    FA_HIP(fa::launch_pad_quad(h->moving_pad, h->moving_quad, h->shape.n0, h->shape.n1, h->shape.n2, h->stream));
  fa::GradArgs ga{};
  ga.fixed = fixed;
  ga.moving_pad = h->moving_pad;
  ga.moving_quad = h->moving_quad;
  ga.d = d;
  ga.out = grad_dev;
  ga.gscale = grad_scale_dev;
  ga.partials = h->partials;
  ga.ctl = h->ctl;
  ga.n0 = h->shape.n0;
  ga.n1 = h->shape.n1;
  ga.n2 = h->shape.n2;
  ga.zc = h->tg.zc;
  ga.tiles_y = h->tg.tiles_y;
  ga.tiles_x = h->tg.tiles_x;
  ga.eps_cc = h->eps;
  ga.inv_n = (float)(1.0 / (double)h->n);
  ga.mode = grad_dev ? 1 : 2;
  FA_HIP(fa::launch_grad(ga, h->window, h->tg, h->stream));
  if (loss_dev)
    FA_HIP(fa::launch_partials_ratio(h->partials, h->tg.blocks(), -(double)h->n, loss_dev, h->stream));
  return FA_OK;
}

void fa_lncc_destroy(fa_lncc h) { release(h); }

fa_status fa_lncc_eval_noalloc(fa_shape shape, int window, float cc_eps, const float* fixed, const float* moving,
                               const float* d, float* loss_dev, float* grad_dev, const float* grad_scale_dev,
                               void* hip_stream) {
  FA_TRY(fa::check_shape(shape));
  if (window < 1 || window > fa::kMaxWindow || window % 2 == 0)
    return fail(FA_EINVAL, "window must be odd and in [1, 9]");
  if (!(cc_eps >= 0.0f) || !(cc_eps < 1e30f)) return fail(FA_EINVAL, "cc_eps must be finite and >= 0");
  if (!fixed || !moving || !d) return fail(FA_EINVAL, "fixed, moving and d must not be NULL");
  if (!loss_dev && !grad_dev) return fail(FA_EINVAL, "loss_dev and grad_dev are both NULL");
  const int64_t n = fa::voxels(shape);
  const fa::Tiling tg = fa::choose_tiling(shape, fa::KIND_GRAD, fa::Tuning(), fa::grad_cube_supported(window));
  const int nb = tg.blocks();
  // layout of the scratch array: control block | loss partials | mean partials | padded moving image
  const size_t off_part = align256(sizeof(fa::Ctl));
  const size_t off_mean = off_part + align256((size_t)nb * sizeof(double));
  const size_t off_pad = off_mean + align256((size_t)fa::kMeanBlocks * sizeof(double));
  const size_t need = off_pad + (size_t)fa::padded_voxels(shape.n0, shape.n1, shape.n2) * sizeof(float);
  if (need > (size_t)FA_LNCC_NOALLOC_SCRATCH_BYTES)
    return fail(FA_EINVAL, "volume too large for the allocation-free evaluation: needs " + std::to_string(need) +
                               " bytes of scratch, the library holds " +
                               std::to_string((size_t)FA_LNCC_NOALLOC_SCRATCH_BYTES));
  void* base = nullptr;
  FA_TRY(scratch_address(&base));
  unsigned char* b = static_cast<unsigned char*>(base);
  fa::Ctl* ctl = reinterpret_cast<fa::Ctl*>(b);
  double* partials = reinterpret_cast<double*>(b + off_part);
  double* mean_partials = reinterpret_cast<double*>(b + off_mean);
  float* moving_pad = reinterpret_cast<float*>(b + off_pad);
  const hipStream_t st = (hipStream_t)hip_stream;
  // every scratch word the kernels read is written earlier in this call, on
  // this stream: the control block by its init kernel, the shifts by the
  // means, the padded image by the pad kernel, each partial by its workgroup
  FA_HIP(fa::launch_ctl_init(ctl, 0.9f, 0.999f, 0, 0, st));
  FA_HIP(fa::launch_mean(fixed, n, mean_partials, &ctl->shift_i, st));
  FA_HIP(fa::launch_mean(moving, n, mean_partials, &ctl->shift_j, st));
  FA_HIP(fa::launch_pad(moving, moving_pad, shape.n0, shape.n1, shape.n2, st));
  fa::GradArgs ga{};
  ga.fixed = fixed;
  ga.moving_pad = moving_pad;
  ga.d = d;
  ga.out = grad_dev;
  ga.gscale = grad_scale_dev;
  ga.partials = partials;
  ga.ctl = ctl;
  ga.n0 = shape.n0;
  ga.n1 = shape.n1;
  ga.n2 = shape.n2;
  ga.zc = tg.zc;
  ga.tiles_y = tg.tiles_y;
  ga.tiles_x = tg.tiles_x;
  ga.eps_cc = cc_eps;
  ga.inv_n = (float)(1.0 / (double)n);
  ga.mode = grad_dev ? 1 : 2;
  FA_HIP(fa::launch_grad(ga, window, tg, st));
  if (loss_dev) FA_HIP(fa::launch_partials_ratio(partials, nb, -(double)n, loss_dev, st));
  return FA_OK;
}

}  // extern "C"
