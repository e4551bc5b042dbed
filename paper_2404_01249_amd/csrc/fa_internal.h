// Internal declarations shared by the HIP kernels and the host runtime.
// Nothing here is part of the public C ABI (include/fa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fa {

// clamp(v, lo, hi) for lo <= hi as one v_med3_f32.  The median selects one of
// its three operands, so for every non-NaN v the result is fminf(fmaxf(v, lo),
// hi) bit for bit; that form costs a NaN-quieting max per operand on this
// target besides the max and the min.
__device__ __forceinline__ float clamp_med3(float v, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(v, lo, hi);
}

// Adam's direction m_hat / (sqrt(v_hat) + eps) from the updated moments and
// the reciprocal bias corrections 1 / (1 - beta^t).  The square root is the
// hardware's v_sqrt_f32: the correctly rounded sqrtf expands to about 15
// instructions per component here, and the direction needs no correctly
// rounded root (eps and the fp32 moments dominate its error).
__device__ __forceinline__ float adam_direction(float mm, float vv, float ibc1, float ibc2, float eps) {
  return (mm * ibc1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vv * ibc2) + eps);
}

// Per-pair control block in device memory.  Kernels of one iteration read
// and update it so that a whole iteration can be replayed (for example from a
// captured graph) without host involvement.
// M = max |s| lives in kMSlots slots kMStride words apart (one per XCD, each
// in its own 128-byte line): a workgroup's atomicMax goes to the slot of its
// XCD, and readers take the maximum of the slots.  One address for every
// workgroup serialises the atomics (about 10 ns each on this GPU, 10 us for
// a thousand workgroups).
constexpr int kMSlots = 8, kMStride = 32;

struct Ctl {
  int t;                 // Adam step count of the iteration in flight (1-based)
  int iter;              // schedule iterations completed (index of the next loss)
  float bc1, bc2;        // 1 - beta1^t, 1 - beta2^t (from bp1, bp2)
  float beta1, beta2;    // copies of the Adam constants for the t update
  float shift_i, shift_j;  // mean intensities of the fixed and moving inputs; LNCC
                           // is invariant to a global intensity shift, and
                           // removing the mean reduces fp32 cancellation in the
                           // window variances
  double bp1, bp2;       // beta1^t, beta2^t in double: pow at a level's start,
                         // then one product per iteration
  // bit patterns of M (non-negative floats, so unsigned order is float order)
  alignas(128) unsigned int mslot[kMSlots * kMStride];
};

// Tile geometry of one streaming launch: in-plane tile (TY x TX) along
// (n1, n2); the workgroup marches along n0 over a chunk of ZC planes.
// cube: the smoothing and composition kernels take whole TZ x TY x TX bricks
// (zc = TZ planes) and run their three passes in LDS instead of marching
// along n0 (small volumes, where the march's sequential plane steps dominate).
struct Tiling {
  int ty, tx, zc;
  int tiles_y, tiles_x, chunks;
  int variant = 0;   // gradient kernel: 2 = gathers issued after the LDS passes
  bool cube = false;
  int blocks() const { return tiles_y * tiles_x * chunks; }
};
constexpr int kCubeZ = 4, kCubeY = 8, kCubeX = 16;   // brick of a cube launch

// Which launch after the gradient kernel records an iteration's loss and
// advances its step count (its GaussArgs carry the loss partials): the warp
// smoothing (2) when it is a brick launch, else the composition (1).
inline int record_launch(const Tiling& warp_smoothing) { return warp_smoothing.cube ? 2 : 1; }

// ---- fused gradient (+ Adam) kernel -------------------------------------
struct GradArgs {
  const float* fixed;
  const float* moving_pad;   // moving image with a zero border of kPad voxels
  const float* moving_quad;  // the same as corner quads (launch_pad_quad), or NULL
  const float* d;        // [3][N]
  float* m;              // [3][N] (Adam mode)
  float* v;              // [3][N]
  float* out;            // [3][N]: Adam direction (mode 0) or gradient (mode 1)
  const float* gscale;   // mode 1: optional device scalar multiplying the gradient
  double* partials;      // per-workgroup sum of cc
  Ctl* ctl;
  int n0, n1, n2;
  int zc, tiles_y, tiles_x;
  float eps_cc;
  float beta1, beta2, adam_eps;
  float inv_n;
  int mode;              // 0: gradient + Adam; 1: gradient only; 2: loss only
};

// ---- streaming separable Gaussian on a 3-channel field ---------------------
// EPI_COMPOSE samples d with global gathers (any step length);
// EPI_COMPOSE_LDS stages three planes of d in LDS and needs |u| <= 1 voxel
// (eta <= 2, since max |u| = eta / 2).
// EPI_SMOOTH_MAX stores the smoothed field and takes M = max |s| in one pass.
enum GaussEpilogue {
  EPI_STORE = 0,
  EPI_MAXNORM = 1,
  EPI_COMPOSE = 2,
  EPI_COMPOSE_LDS = 4,
  EPI_SMOOTH_MAX = 5
};

struct GaussArgs {
  const float* in;       // [3][N]
  float* out;            // [3][N] (store / compose)
  const float* d;        // [3][N] displacement sampled by the composition
  const float* wts;      // 2R+1 normalised taps (device)
  Ctl* ctl;
  const double* partials;  // loss partials of the gradient kernel (final epilogue)
  float* loss_hist;
  int loss_cap;
  int n_partials;
  float inv_n;
  float eta;
  int n0, n1, n2;
  int zc, tiles_y, tiles_x;
  // radius above kMaxRadius only (launch_gauss): a [3][N] scratch field
  // distinct from in and out
  float* wide_tmp;
};

// ---- batched launches ----------------------------------------------------
// One registration's share of a batched launch: its arguments and its range
// [first, first + nblocks) of the launch's workgroups (tile order, after the
// XCD renumbering).  owner[g] (one int per workgroup) names the entry of
// workgroup g.  Every entry of one launch shares the kernel's template
// parameters (window or radius, tile shape, brick or march, epilogue).
template <class Args>
struct BatchEntry {
  Args a;
  int first;
  int nblocks;
};

// ---- launchers (fa_kernels.hip) -----------------------------------------
hipError_t launch_grad(const GradArgs& a, int window, const Tiling& t, hipStream_t s);
hipError_t launch_gauss(const GaussArgs& a, int radius, int epilogue, const Tiling& t, hipStream_t s);
// Batched forms: `total` workgroups over the entries E (device memory) with
// owner (device memory, `total` ints); t gives the template parameters only
// (tile shape, brick or march) and must be the tiling of every entry.
// quad: every entry's moving_quad is set (the corner-quad gathers).  adam:
// every entry's mode is 0 (gradient and Adam; a kernel specialised for it).
hipError_t launch_grad_batch(const BatchEntry<GradArgs>* E, const int* owner, int total, int window,
                             const Tiling& t, bool quad, bool adam, hipStream_t s);
hipError_t launch_gauss_batch(const BatchEntry<GaussArgs>* E, const int* owner, int total, int radius,
                              int epilogue, const Tiling& t, hipStream_t s);
// Whether a batched form exists for these parameters.
bool grad_batch_supported(int window, const Tiling& t);
bool gauss_batch_supported(int radius, int epilogue, const Tiling& t);
// use_jac: the Eulerian direction J(phi)^T g (J = I + grad d, central
// differences inside, one-sided on the faces), then Adam, in place over g in
// ga (which receives the Adam direction); also clears M for the iteration.
hipError_t launch_eulerian_adam(float* ga, const float* d, float* m, float* v, Ctl* ctl, int n0, int n1,
                                int n2, float beta1, float beta2, float adam_eps, hipStream_t s);
hipError_t launch_fill(float* p, float value, int64_t n, hipStream_t s);
// out = in with a zero border of kPad voxels (padded_voxels(n0, n1, n2) floats).
hipError_t launch_pad(const float* in, float* out, int n0, int n1, int n2, hipStream_t s);
// Corner quads of the padded image `pad` (padded_voxels(n0, n1, n2) float4s
// into quad, 16-byte aligned; quad_supported must hold).
hipError_t launch_pad_quad(const float* pad, float* quad, int n0, int n1, int n2, hipStream_t s);
hipError_t launch_blur_axis(const float* in, float* out, int n0, int n1, int n2, int axis,
                            const float* wts, int radius, hipStream_t s);
hipError_t launch_resample(const float* in, float* out, int nin0, int nin1, int nin2,
                           int nout0, int nout1, int nout2, int nch,
                           float rho0, float rho1, float rho2, hipStream_t s);
hipError_t launch_warp(const float* img, const float* d, float* out, int n0, int n1, int n2,
                       hipStream_t s);
hipError_t launch_soa_to_aos(const float* in, float* out, int64_t n, hipStream_t s);
// out = u + d(x + u) ([3][n] fields; out must not alias d).
hipError_t launch_compose_fields(const float* u, const float* d, float* out, int n0, int n1, int n2,
                                 hipStream_t s);
// Sets the Adam step count to t_done + 1 (bias corrections in double), clears
// M; iter >= 0 also resets the iteration counter.
hipError_t launch_ctl_init(Ctl* ctl, float beta1, float beta2, int t_done, int iter, hipStream_t s);
// Mean of x (n values) into *dst (device float), via `scratch` (kMeanBlocks doubles).
hipError_t launch_mean(const float* x, int64_t n, double* scratch, float* dst, hipStream_t s);
hipError_t launch_sum_partials(const double* partials, int n, double* dst, hipStream_t s);
// (float)(sum of n partials / denom) into *dst (device float).
hipError_t launch_partials_ratio(const double* partials, int n, double denom, float* dst, hipStream_t s);
// Workgroups of the mean's first pass: eight per CU, so that the strided loads
// of each thread (a few per thread at 160x192x224) are not latency-bound
// (256 workgroups took 33 us for 6.9 M values, 2048 take 9 us).
constexpr int kMeanBlocks = 2048;

bool grad_tile_supported(int ty, int tx);
bool gauss_tile_supported(int ty, int tx);
// Whether a brick (cube) launch exists for this radius and epilogue.
bool gauss_cube_supported(int radius, int epilogue);
bool grad_cube_supported(int window);
size_t grad_lds_bytes(int window, int ty, int tx);
size_t gauss_lds_bytes(int radius, int ty, int tx);

constexpr int kMaxWindow = 9;
// Zero border of the padded moving image the gradient kernel samples.
constexpr int kPad = 2;
inline int64_t padded_voxels(int n0, int n1, int n2) {
  return (int64_t)(n0 + 2 * kPad) * (n1 + 2 * kPad) * (n2 + 2 * kPad);
}
// Whether the corner-quad copy of a padded volume stays below 4 GiB (its
// gathers use 32-bit byte offsets).
inline bool quad_supported(int n0, int n1, int n2) {
  // 32-bit byte offsets; padded plane size and padded indices below 2^24
  // (the gathers multiply them in 24 bits)
  const uint64_t p0 = (uint64_t)n0 + 2 * kPad, p1 = (uint64_t)n1 + 2 * kPad, p2 = (uint64_t)n2 + 2 * kPad;
  return (uint64_t)padded_voxels(n0, n1, n2) * 16u < ((uint64_t)1 << 32) && p1 * p2 < ((uint64_t)1 << 24) &&
         p0 < ((uint64_t)1 << 24);
}
// Gaussian radii: the streaming and brick kernels take 0..kMaxRadius as a
// template parameter; launch_gauss runs radii up to kMaxWideRadius through
// separable passes with a run-time radius (GaussArgs::wide_tmp).
constexpr int kMaxRadius = 6;
constexpr int kMaxWideRadius = 24;

}  // namespace fa
