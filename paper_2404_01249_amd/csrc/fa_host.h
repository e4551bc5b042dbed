// Host-side helpers shared by the sources of the C ABI: error reporting,
// status macros, shape checks and the launch-shape heuristic of the
// streaming kernels.  Not part of the public interface.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "fa.h"
#include "fa_internal.h"

namespace fa {

// Records msg as the calling thread's last error (returned by fa_last_error)
// and returns s.
fa_status fail(fa_status s, const std::string& msg);

// Every dimension >= 2 and n0*n1*n2 < 2^29 (gathers address a volume with
// 32-bit signed byte offsets).
fa_status check_shape(const fa_shape& s);

inline int64_t voxels(const fa_shape& s) { return (int64_t)s.n0 * s.n1 * s.n2; }

// Launch-shape override of one streaming kernel kind (0 = auto).
struct Tuning {
  int ty = 0, tx = 0, zc = 0, variant = 0;
};

// The streaming kernels whose launch shape is chosen per level.
enum KernelKind { KIND_GRAD = 0, KIND_SMOOTH_MAX = 1, KIND_WARP_SMOOTH = 2, KIND_COMPOSE = 3 };

// In-plane tile and n0 chunking of one launch of kernel `kind` over a volume
// of shape s (tu overrides the automatic choice).  cube_ok: a brick launch
// exists for the kernel's radius and epilogue (smoothing and composition
// kinds only).
Tiling choose_tiling(const fa_shape& s, KernelKind kind, const Tuning& tu = Tuning(), bool cube_ok = false);

// Sampled Gaussian taps exp(-k^2 / 2 sigma^2), |k| <= ceil(3 sigma), normalised
// to sum 1 (in double); sigma <= 0 gives the single tap 1.  tap_radius: the
// number of taps on each side.
std::vector<float> gaussian_taps(float sigma);
int tap_radius(float sigma);
// Validates every field of fa_params (FA_EINVAL with a message).
fa_status check_params(const fa_params* p);
// Grid of a pyramid level: max(1, floor(n / scale + 1/2)) per axis.
fa_shape level_shape(const fa_shape& s, float scale);

// Chunk lengths of the march tilings ts (one per entry of a batched launch of
// kernel `kind`, volumes of n0s[i] planes along n0, `halo` planes recomputed
// per chunk) for the resident slots they share; entries with pinned[i] keep
// their chunk.  Brick tilings are left as they are.
void batch_chunks(KernelKind kind, int halo, const std::vector<Tiling*>& ts, const std::vector<int>& n0s,
                  const std::vector<char>& pinned);

}  // namespace fa

#define FA_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fa::fail(FA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define FA_TRY(call)                       \
  do {                                     \
    fa_status s_ = (call);                 \
    if (s_ != FA_OK) return s_;            \
  } while (0)
