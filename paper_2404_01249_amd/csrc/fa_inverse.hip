// The post hoc inverse of a warp (include/fa_inverse.h): psi = id + e fitted
// to minimise the mean of |psi(phi(x)) - x|^2 + |phi(psi(x)) - x|^2 (Section
// 4.4.3, "Alternative formulations for Eulerian differential") with
// Algorithm 1's loop.  Two kernels of this file form the direction; the
// smoothing, composition and loss record are the registration's kernels.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "fa.h"
#include "fa_host.h"
#include "fa_internal.h"
#include "fa_inverse.h"

using fa::clamp_med3;
using fa::Ctl;
using fa::fail;
using fa::Tiling;

namespace {

// The splat accumulates sum_x 2 r1(x) w_j(x + d(x)) in 64-bit integers, in
// units of 2^-32: integer addition is associative, so the sum does not depend
// on the order in which the atomics land.  Each term is clamped to 2^30 in
// magnitude (only non-finite or absurd displacements reach it).
constexpr double kFixScale = 4294967296.0;
constexpr double kFixUnit = 1.0 / 4294967296.0;
constexpr float kFixClamp = 1073741824.0f;
constexpr int kInvThreads = 256;
constexpr int kInvMaxBlocks = 4096;

// Trilinear cell of position p on an n0 x n1 x n2 grid: flat corner indices
// and weights in the order (b0, b1, b2) = 000, 001, ..., 111; corners off the
// grid have weight 0 and index 0 (zero extension).
struct Cell {
  int idx[8];
  float w[8];
  float t0, t1, t2;
  unsigned ok;
};

__device__ __forceinline__ Cell cell_of(float p0, float p1, float p2, int n0, int n1, int n2) {
  Cell c;
  const float f0 = floorf(p0), f1 = floorf(p1), f2 = floorf(p2);
  c.t0 = p0 - f0;
  c.t1 = p1 - f1;
  c.t2 = p2 - f2;
  // far outside, the clamp keeps the integers small; every corner is then off the grid anyway
  const int i0 = (int)clamp_med3(f0, -2.0f, (float)n0);
  const int i1 = (int)clamp_med3(f1, -2.0f, (float)n1);
  const int i2 = (int)clamp_med3(f2, -2.0f, (float)n2);
  c.ok = 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b0 = (k >> 2) & 1, b1 = (k >> 1) & 1, b2 = k & 1;
    const int z = i0 + b0, y = i1 + b1, x = i2 + b2;
    const bool in = z >= 0 && z < n0 && y >= 0 && y < n1 && x >= 0 && x < n2;
    c.idx[k] = in ? (z * n1 + y) * n2 + x : 0;
    c.w[k] = in ? (b0 ? c.t0 : 1.0f - c.t0) * (b1 ? c.t1 : 1.0f - c.t1) * (b2 ? c.t2 : 1.0f - c.t2) : 0.0f;
    c.ok |= in ? (1u << k) : 0u;
  }
  return c;
}

__device__ __forceinline__ float sample(const float* __restrict__ f, const Cell& c) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += ((c.ok >> k) & 1u) ? c.w[k] * f[c.idx[k]] : 0.0f;
  return s;
}

// Value and position derivative of the trilinear sample (the derivative from
// the right at an integer coordinate, as the cell is chosen by floor).
__device__ __forceinline__ float sample_grad(const float* __restrict__ f, const Cell& c, float& g0, float& g1,
                                             float& g2) {
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = ((c.ok >> k) & 1u) ? f[c.idx[k]] : 0.0f;
  const float dx00 = v[1] - v[0], dx01 = v[3] - v[2], dx10 = v[5] - v[4], dx11 = v[7] - v[6];
  const float e00 = v[0] + c.t2 * dx00, e01 = v[2] + c.t2 * dx01;
  const float e10 = v[4] + c.t2 * dx10, e11 = v[6] + c.t2 * dx11;
  const float dy0 = e01 - e00, dy1 = e11 - e10;
  const float f0 = e00 + c.t1 * dy0, f1 = e10 + c.t1 * dy1;
  const float dxy0 = dx00 + c.t1 * (dx01 - dx00), dxy1 = dx10 + c.t1 * (dx11 - dx10);
  g0 = f1 - f0;
  g1 = dy0 + c.t0 * (dy1 - dy0);
  g2 = dxy0 + c.t0 * (dxy1 - dxy0);
  return f0 + c.t0 * (f1 - f0);
}

__device__ __forceinline__ unsigned long long to_fixed(float v) {
  const float vc = clamp_med3(v, -kFixClamp, kFixClamp);
  return (unsigned long long)__double2ll_rn((double)vc * kFixScale);
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kInvThreads / 64; ++i) s += red[i];
  return s;
}

// r1(x) = d(x) + e(x + d(x)), the residual of psi o phi.  Its derivative in e
// is the splat of 2 r1 at x + d(x), accumulated in acc ([3][N], fixed point,
// zero on entry).  part[block] = -sum of |r1|^2 over the block's voxels.
__global__ void __launch_bounds__(kInvThreads)
k_inv_splat(const float* __restrict__ d, const float* __restrict__ e, unsigned long long* __restrict__ acc,
            double* __restrict__ part, int n0, int n1, int n2) {
  __shared__ double red[kInvThreads / 64];
  const int N = n0 * n1 * n2;
  double loss = 0.0;
  for (int i = blockIdx.x * kInvThreads + threadIdx.x; i < N; i += gridDim.x * kInvThreads) {
    const int x = i % n2, y = (i / n2) % n1, z = i / (n1 * n2);
    const float d0 = d[i], d1 = d[N + i], d2 = d[2 * N + i];
    const Cell c = cell_of((float)z + d0, (float)y + d1, (float)x + d2, n0, n1, n2);
    const float r0 = d0 + sample(e, c);
    const float r1 = d1 + sample(e + N, c);
    const float r2 = d2 + sample(e + 2 * N, c);
    loss += (double)(r0 * r0 + r1 * r1 + r2 * r2);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (((c.ok >> k) & 1u) && c.w[k] != 0.0f) {
        const float w2 = 2.0f * c.w[k];
        atomicAdd(&acc[c.idx[k]], to_fixed(w2 * r0));
        atomicAdd(&acc[N + c.idx[k]], to_fixed(w2 * r1));
        atomicAdd(&acc[2 * N + c.idx[k]], to_fixed(w2 * r2));
      }
    }
  }
  const double s = block_sum256(loss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = -s;
}

// The same splat by bricks of 4 x 8 x 16 voxels (two per thread).  A smooth
// warp sends a brick's samples into a box of nodes little larger than the
// brick: the workgroup sums its contributions there with LDS atomics (the
// same fixed-point integers, so the result is bitwise that of the direct
// form), then adds each non-zero box node to acc with one global atomic per
// component.  A brick whose box exceeds kBoxNodes (a folded or wildly varying
// warp) scatters directly.
constexpr int kBZ = 4, kBY = 8, kBX = 16;
constexpr int kBoxNodes = 2048;   // 3 x 2048 x 8 B = 48 KiB of LDS

__global__ void __launch_bounds__(kInvThreads)
k_inv_splat_lds(const float* __restrict__ d, const float* __restrict__ e, unsigned long long* __restrict__ acc,
                double* __restrict__ part, int n0, int n1, int n2) {
  __shared__ unsigned long long box[3 * kBoxNodes];
  __shared__ int bb[6];   // box: lo0, lo1, lo2, hi0, hi1, hi2 (inclusive)
  __shared__ double red[kInvThreads / 64];
  constexpr int VPT = kBZ * kBY * kBX / kInvThreads;
  const int N = n0 * n1 * n2;
  const int tz = (n0 + kBZ - 1) / kBZ, ty = (n1 + kBY - 1) / kBY, tx = (n2 + kBX - 1) / kBX;
  const int nbricks = tz * ty * tx;
  const int tid = threadIdx.x;
  double loss = 0.0;
  for (int b = blockIdx.x; b < nbricks; b += gridDim.x) {
    const int bx = b % tx, by = (b / tx) % ty, bz = b / (tx * ty);
    int cz[VPT], cy[VPT], cx[VPT];
    float t0[VPT], t1[VPT], t2[VPT], r[VPT][3];
    bool valid[VPT];
    int lo0 = 1 << 30, lo1 = 1 << 30, lo2 = 1 << 30, hi0 = -(1 << 30), hi1 = -(1 << 30), hi2 = -(1 << 30);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int l = tid + k * kInvThreads;
      const int z = bz * kBZ + l / (kBY * kBX), y = by * kBY + (l / kBX) % kBY, x = bx * kBX + l % kBX;
      valid[k] = z < n0 && y < n1 && x < n2;
      cz[k] = cy[k] = cx[k] = 0;
      t0[k] = t1[k] = t2[k] = 0.0f;
      r[k][0] = r[k][1] = r[k][2] = 0.0f;
      if (valid[k]) {
        const int i = (z * n1 + y) * n2 + x;
        const float d0 = d[i], d1 = d[N + i], d2 = d[2 * N + i];
        const Cell c = cell_of((float)z + d0, (float)y + d1, (float)x + d2, n0, n1, n2);
        r[k][0] = d0 + sample(e, c);
        r[k][1] = d1 + sample(e + N, c);
        r[k][2] = d2 + sample(e + 2 * N, c);
        loss += (double)(r[k][0] * r[k][0] + r[k][1] * r[k][1] + r[k][2] * r[k][2]);
        t0[k] = c.t0;
        t1[k] = c.t1;
        t2[k] = c.t2;
        // the cell's lower corner (clamped as in cell_of: off-grid corners are dropped below)
        cz[k] = (int)clamp_med3(floorf((float)z + d0), -2.0f, (float)n0);
        cy[k] = (int)clamp_med3(floorf((float)y + d1), -2.0f, (float)n1);
        cx[k] = (int)clamp_med3(floorf((float)x + d2), -2.0f, (float)n2);
        lo0 = min(lo0, cz[k]);
        lo1 = min(lo1, cy[k]);
        lo2 = min(lo2, cx[k]);
        hi0 = max(hi0, cz[k] + 1);
        hi1 = max(hi1, cy[k] + 1);
        hi2 = max(hi2, cx[k] + 1);
      }
    }
    if (tid == 0) {
      bb[0] = bb[1] = bb[2] = 1 << 30;
      bb[3] = bb[4] = bb[5] = -(1 << 30);
    }
    __syncthreads();
    atomicMin(&bb[0], lo0);
    atomicMin(&bb[1], lo1);
    atomicMin(&bb[2], lo2);
    atomicMax(&bb[3], hi0);
    atomicMax(&bb[4], hi1);
    atomicMax(&bb[5], hi2);
    __syncthreads();
    // the box clipped to the grid (nodes off the grid receive nothing)
    const int b0 = max(bb[0], 0), b1 = max(bb[1], 0), b2 = max(bb[2], 0);
    const int e0 = min(bb[3], n0 - 1), e1 = min(bb[4], n1 - 1), e2 = min(bb[5], n2 - 1);
    const int s0 = e0 - b0 + 1, s1 = e1 - b1 + 1, s2 = e2 - b2 + 1;
    const bool empty = s0 <= 0 || s1 <= 0 || s2 <= 0;
    const int nb = empty ? 0 : s0 * s1 * s2;
    if (nb <= kBoxNodes) {
      for (int q = tid; q < 3 * nb; q += kInvThreads) box[q] = 0ull;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        if (!valid[k]) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int o0 = (j >> 2) & 1, o1 = (j >> 1) & 1, o2 = j & 1;
          const int z = cz[k] + o0, y = cy[k] + o1, x = cx[k] + o2;
          if (z < 0 || z >= n0 || y < 0 || y >= n1 || x < 0 || x >= n2) continue;
          const float w = (o0 ? t0[k] : 1.0f - t0[k]) * (o1 ? t1[k] : 1.0f - t1[k]) * (o2 ? t2[k] : 1.0f - t2[k]);
          if (w == 0.0f) continue;
          const int q = ((z - b0) * s1 + (y - b1)) * s2 + (x - b2);
          const float w2 = 2.0f * w;
          atomicAdd(&box[q], to_fixed(w2 * r[k][0]));
          atomicAdd(&box[nb + q], to_fixed(w2 * r[k][1]));
          atomicAdd(&box[2 * nb + q], to_fixed(w2 * r[k][2]));
        }
      }
      __syncthreads();
      for (int q = tid; q < nb; q += kInvThreads) {
        const int x = b2 + q % s2, y = b1 + (q / s2) % s1, z = b0 + q / (s1 * s2);
        const int gi = (z * n1 + y) * n2 + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const unsigned long long v = box[c * nb + q];
          if (v != 0ull) atomicAdd(&acc[c * N + gi], v);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        if (!valid[k]) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int o0 = (j >> 2) & 1, o1 = (j >> 1) & 1, o2 = j & 1;
          const int z = cz[k] + o0, y = cy[k] + o1, x = cx[k] + o2;
          if (z < 0 || z >= n0 || y < 0 || y >= n1 || x < 0 || x >= n2) continue;
          const float w = (o0 ? t0[k] : 1.0f - t0[k]) * (o1 ? t1[k] : 1.0f - t1[k]) * (o2 ? t2[k] : 1.0f - t2[k]);
          if (w == 0.0f) continue;
          const int gi = (z * n1 + y) * n2 + x;
          const float w2 = 2.0f * w;
          atomicAdd(&acc[gi], to_fixed(w2 * r[k][0]));
          atomicAdd(&acc[N + gi], to_fixed(w2 * r[k][1]));
          atomicAdd(&acc[2 * N + gi], to_fixed(w2 * r[k][2]));
        }
      }
    }
    __syncthreads();   // box and bb are reused by the next brick
  }
  const double s = block_sum256(loss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = -s;
}

// r2(x) = e(x) + d(x + e(x)), the residual of phi o psi, whose derivative in
// e(x) is 2 (I + grad d)^T r2; with the splat's sum (acc, cleared here for the
// next iteration) and the 1/N of the mean this is dU/de.  grad_only: write it
// to out.  Otherwise Adam on it (moments m, v; bias corrections from ctl):
// out = the direction; block 0 also clears M for the iteration's smoothing.
// part[block] = -sum of |r2|^2.
__global__ void __launch_bounds__(kInvThreads)
k_inv_dir(const float* __restrict__ d, const float* __restrict__ e, unsigned long long* __restrict__ acc,
          float* __restrict__ m, float* __restrict__ v, float* __restrict__ out, Ctl* __restrict__ ctl,
          double* __restrict__ part, int n0, int n1, int n2, float inv_n, float beta1, float beta2,
          float adam_eps, int grad_only) {
  __shared__ double red[kInvThreads / 64];
  const int N = n0 * n1 * n2;
  if (!grad_only && blockIdx.x == 0 && threadIdx.x < fa::kMSlots) ctl->mslot[threadIdx.x * fa::kMStride] = 0u;
  const float ibc1 = grad_only ? 1.0f : 1.0f / ctl->bc1;
  const float ibc2 = grad_only ? 1.0f : 1.0f / ctl->bc2;
  double loss = 0.0;
  for (int i = blockIdx.x * kInvThreads + threadIdx.x; i < N; i += gridDim.x * kInvThreads) {
    const int x = i % n2, y = (i / n2) % n1, z = i / (n1 * n2);
    float s[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      s[q] = (float)((double)(long long)acc[q * N + i] * kFixUnit);
      acc[q * N + i] = 0ull;
    }
    const float e0 = e[i], e1 = e[N + i], e2 = e[2 * N + i];
    const Cell c = cell_of((float)z + e0, (float)y + e1, (float)x + e2, n0, n1, n2);
    float J[3][3];   // J[q][a] = d d_q / d p_a at x + e(x)
    const float v0 = sample_grad(d, c, J[0][0], J[0][1], J[0][2]);
    const float v1 = sample_grad(d + N, c, J[1][0], J[1][1], J[1][2]);
    const float v2 = sample_grad(d + 2 * N, c, J[2][0], J[2][1], J[2][2]);
    const float r[3] = {e0 + v0, e1 + v1, e2 + v2};
    loss += (double)(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float g = (s[a] + 2.0f * (r[a] + J[0][a] * r[0] + J[1][a] * r[1] + J[2][a] * r[2])) * inv_n;
      const int ia = a * N + i;
      if (grad_only) {
        out[ia] = g;
      } else {
        const float mm = beta1 * m[ia] + (1.0f - beta1) * g;
        const float vv = beta2 * v[ia] + (1.0f - beta2) * g * g;
        m[ia] = mm;
        v[ia] = vv;
        out[ia] = fa::adam_direction(mm, vv, ibc1, ibc2, adam_eps);
      }
    }
  }
  const double t = block_sum256(loss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = -t;
}

int inv_blocks(int64_t n) {
  return (int)std::min<int64_t>((n + kInvThreads - 1) / kInvThreads, kInvMaxBlocks);
}

template <typename T>
fa_status ialloc(T** out, size_t count, const char* what) {
  *out = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc((void**)out, count * sizeof(T));
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(FA_ENOMEM, std::string("hipMalloc failed for ") + what + " (" + std::to_string(count * sizeof(T)) +
                               " bytes): " + hipGetErrorString(e));
  }
  return FA_OK;
}

struct ILevel {
  fa_shape shape{};
  int64_t n = 0;
  float scale = 1.0f;
  int iters = 0;
  float* d = nullptr;   // the warp's field on this grid (owned unless it aliases the input copy)
  bool owns = false;
  Tiling tsg{}, tsc{}, tsw{};
};

}  // namespace

struct fa_inverse_s {
  hipStream_t stream = nullptr;
  fa_shape shape{};
  int64_t n = 0;
  fa_params p{};
  float* in_d = nullptr;   // [3][n] copy of the input field
  std::vector<ILevel> levels;
  int64_t cap = 0;
  float* e = nullptr;      // psi - id at the current level, [3][n]
  float* m = nullptr;
  float* v = nullptr;
  float* a = nullptr;      // Adam direction
  float* tmp = nullptr;    // smoothed direction, then the composed field
  float* wide = nullptr;   // [3][cap] scratch of the smoothing passes with a radius above 6
  unsigned long long* acc = nullptr;   // splat accumulator [3][n], zero between iterations
  Ctl* ctl = nullptr;
  float* loss_hist = nullptr;
  int loss_cap = 0;
  double* partials = nullptr;
  float* scalar = nullptr;  // device float (eval_gradient's cost)
  float* wts = nullptr;
  int rg = 0, rw = 0, off_g = 0, off_w = 0, off_one = 0;
  int cur_level = 0, cur_iter = 0, t_done = 0, iters_done = 0;
  bool scheduled = false;
  bool splat_direct = false;   // the per-voxel global-atomic splat instead of the brick form
};

namespace {

void free_levels(fa_inverse H) {
  for (auto& L : H->levels)
    if (L.owns && L.d) (void)hipFree(L.d);
  H->levels.clear();
}

void free_all(fa_inverse H) {
  free_levels(H);
  float* fb[] = {H->in_d, H->e, H->m, H->v, H->a, H->tmp, H->wide, H->loss_hist, H->scalar, H->wts};
  for (float* b : fb)
    if (b) (void)hipFree(b);
  if (H->acc) (void)hipFree(H->acc);
  if (H->ctl) (void)hipFree(H->ctl);
  if (H->partials) (void)hipFree(H->partials);
}

// e scaled by rho, the Adam moments unscaled, trilinear at corner-aligned
// positions of the next (finer) grid.
fa_status transition(fa_inverse H) {
  const ILevel& C = H->levels[H->cur_level];
  const ILevel& F = H->levels[H->cur_level + 1];
  auto rho = [](int nf, int nc) { return nc > 1 ? (float)((double)(nf - 1) / (double)(nc - 1)) : 1.0f; };
  const fa_shape& c = C.shape;
  const fa_shape& f = F.shape;
  FA_HIP(fa::launch_resample(H->e, H->tmp, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, rho(f.n0, c.n0),
                             rho(f.n1, c.n1), rho(f.n2, c.n2), H->stream));
  FA_HIP(fa::launch_resample(H->m, H->a, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, 1.f, 1.f, 1.f, H->stream));
  FA_HIP(fa::launch_resample(H->v, H->m, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, 1.f, 1.f, 1.f, H->stream));
  // the fine e, m, v now sit in tmp, a, m; the coarse e and v buffers are free
  float* old_e = H->e;
  float* old_m = H->m;
  float* old_v = H->v;
  float* old_a = H->a;
  float* old_t = H->tmp;
  H->e = old_t;
  H->m = old_a;
  H->v = old_m;
  H->a = old_e;
  H->tmp = old_v;
  return FA_OK;
}

bool schedule_done(const fa_inverse H) {
  return H->cur_level == (int)H->levels.size() - 1 && H->cur_iter >= H->levels.back().iters;
}

fa_status launch_direction(fa_inverse H, const ILevel& L, float* out, int grad_only) {
  const fa_shape& s = L.shape;
  const int b = inv_blocks(L.n);
  if (H->splat_direct) {
    hipLaunchKernelGGL(k_inv_splat, dim3(b), dim3(kInvThreads), 0, H->stream, L.d, H->e, H->acc, H->partials,
                       s.n0, s.n1, s.n2);
  } else {
    hipLaunchKernelGGL(k_inv_splat_lds, dim3(b), dim3(kInvThreads), 0, H->stream, L.d, H->e, H->acc,
                       H->partials, s.n0, s.n1, s.n2);
  }
  FA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_inv_dir, dim3(b), dim3(kInvThreads), 0, H->stream, L.d, H->e, H->acc, H->m, H->v, out,
                     H->ctl, H->partials + b, s.n0, s.n1, s.n2, (float)(1.0 / (double)L.n), H->p.adam_beta1,
                     H->p.adam_beta2, H->p.adam_eps, grad_only);
  FA_HIP(hipGetLastError());
  return FA_OK;
}

fa_status launch_iteration(fa_inverse H, const ILevel& L) {
  FA_TRY(launch_direction(H, L, H->a, 0));
  fa::GaussArgs gs{};
  gs.ctl = H->ctl;
  gs.n0 = L.shape.n0;
  gs.n1 = L.shape.n1;
  gs.n2 = L.shape.n2;
  gs.eta = H->p.eta;
  gs.inv_n = (float)(1.0 / (double)L.n);

  fa::GaussArgs g1 = gs;   // s = G * a, M = max |s|
  g1.in = H->a;
  g1.out = H->tmp;
  g1.wts = H->wts + H->off_g;
  g1.wide_tmp = H->wide;
  g1.zc = L.tsg.zc;
  g1.tiles_y = L.tsg.tiles_y;
  g1.tiles_x = L.tsg.tiles_x;
  FA_HIP(fa::launch_gauss(g1, H->rg, fa::EPI_SMOOTH_MAX, L.tsg, H->stream));

  fa::GaussArgs g2 = gs;   // e' = u + e(x + u), u = -eta s / (2M), in place over s
  g2.in = H->tmp;
  g2.out = H->tmp;
  g2.d = H->e;
  g2.wts = H->wts + H->off_one;
  g2.zc = L.tsc.zc;
  g2.tiles_y = L.tsc.tiles_y;
  g2.tiles_x = L.tsc.tiles_x;

  fa::GaussArgs g3 = gs;   // e = G * e'
  g3.in = H->tmp;
  g3.out = H->e;
  g3.wts = H->wts + H->off_w;
  g3.wide_tmp = H->wide;
  g3.zc = L.tsw.zc;
  g3.tiles_y = L.tsw.tiles_y;
  g3.tiles_x = L.tsw.tiles_x;

  // the cost record and step count, in the launch the registration uses
  fa::GaussArgs& gr = fa::record_launch(L.tsw) == 2 ? g3 : g2;
  gr.partials = H->partials;
  gr.n_partials = 2 * inv_blocks(L.n);
  gr.loss_hist = H->loss_hist;
  gr.loss_cap = H->loss_cap;

  FA_HIP(fa::launch_gauss(g2, 0, H->p.eta <= 2.0f ? fa::EPI_COMPOSE_LDS : fa::EPI_COMPOSE, L.tsc, H->stream));

  FA_HIP(fa::launch_gauss(g3, H->rw, fa::EPI_STORE, L.tsw, H->stream));
  return FA_OK;
}

}  // namespace

extern "C" {

fa_status fa_inverse_create(const float* d, fa_shape shape, const fa_params* params, void* stream,
                            fa_inverse* out) {
  if (!out) return fail(FA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(FA_EINVAL, "d must be a device pointer");
  FA_TRY(fa::check_shape(shape));
  FA_TRY(fa::check_params(params));
  fa_inverse H = new (std::nothrow) fa_inverse_s();
  if (!H) return fail(FA_ENOMEM, "host allocation failed");
  H->stream = (hipStream_t)stream;
  H->shape = shape;
  H->n = fa::voxels(shape);
  H->p = *params;
  fa_status st = FA_OK;
  if ((st = ialloc(&H->in_d, (size_t)(3 * H->n), "input field")) != FA_OK ||
      (st = ialloc(&H->ctl, 1, "control block")) != FA_OK || (st = ialloc(&H->scalar, 1, "scalar")) != FA_OK) {
    free_all(H);
    delete H;
    return st;
  }
  const hipError_t e = hipMemcpyAsync(H->in_d, d, (size_t)(3 * H->n) * sizeof(float), hipMemcpyDeviceToDevice,
                                      H->stream);
  if (e != hipSuccess) {
    free_all(H);
    delete H;
    return fail(FA_EHIP, std::string("copying the field: ") + hipGetErrorString(e));
  }
  *out = H;
  return FA_OK;
}

fa_status fa_inverse_set_schedule(fa_inverse H, int n_levels, const float* scales, const int* iters) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (n_levels < 1 || n_levels > 16) return fail(FA_EINVAL, "n_levels must be in [1, 16]");
  if (!scales || !iters) return fail(FA_EINVAL, "scales and iters must not be NULL");
  std::vector<ILevel> lv(n_levels);
  int64_t total = 0, nmax = 0;
  H->rg = fa::tap_radius(H->p.sigma_grad);
  H->rw = fa::tap_radius(H->p.sigma_warp);
  for (int i = 0; i < n_levels; ++i) {
    if (!(scales[i] >= 1.0f) || !(scales[i] <= 20.0f)) return fail(FA_EINVAL, "scales must be in [1, 20]");
    if (iters[i] < 0) return fail(FA_EINVAL, "iters must be >= 0");
    lv[i].scale = scales[i];
    lv[i].iters = iters[i];
    lv[i].shape = fa::level_shape(H->shape, scales[i]);
    lv[i].n = fa::voxels(lv[i].shape);
    if (lv[i].shape.n0 < 2 || lv[i].shape.n1 < 2 || lv[i].shape.n2 < 2)
      return fail(FA_ESHAPE, "level " + std::to_string(i) + " has a dimension < 2");
    lv[i].tsg = fa::choose_tiling(lv[i].shape, fa::KIND_SMOOTH_MAX, fa::Tuning(),
                                  fa::gauss_cube_supported(H->rg, fa::EPI_SMOOTH_MAX));
    lv[i].tsw = fa::choose_tiling(lv[i].shape, fa::KIND_WARP_SMOOTH, fa::Tuning(),
                                  fa::gauss_cube_supported(H->rw, fa::EPI_STORE));
    lv[i].tsc = fa::choose_tiling(lv[i].shape, fa::KIND_COMPOSE, fa::Tuning(),
                                  H->p.eta <= 2.0f && fa::gauss_cube_supported(0, fa::EPI_COMPOSE_LDS));
    total += iters[i];
    nmax = std::max(nmax, lv[i].n);
  }
  if (total > (int64_t)1 << 30) return fail(FA_EINVAL, "too many iterations");

  FA_HIP(hipStreamSynchronize(H->stream));
  free_levels(H);
  H->scheduled = false;

  // tap tables: sigma_grad, sigma_warp, the single tap, then one blur per level
  std::vector<float> host;
  auto push = [&](const std::vector<float>& t) {
    const int off = (int)host.size();
    host.insert(host.end(), t.begin(), t.end());
    while (host.size() % 16) host.push_back(0.0f);
    return off;
  };
  H->off_g = push(fa::gaussian_taps(H->p.sigma_grad));
  H->off_w = push(fa::gaussian_taps(H->p.sigma_warp));
  H->off_one = push(std::vector<float>{1.0f});
  std::vector<int> off_blur(n_levels);
  for (int i = 0; i < n_levels; ++i) off_blur[i] = push(fa::gaussian_taps(lv[i].scale / 2.0f));
  if (H->wts) (void)hipFree(H->wts);
  H->wts = nullptr;
  FA_TRY(ialloc(&H->wts, host.size(), "tap tables"));
  FA_HIP(hipMemcpyAsync(H->wts, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, H->stream));

  // state (sized for the largest level) and the splat accumulator
  const int64_t need = std::max(nmax, H->n);   // the blur scratch below spans 5 input-sized volumes
  const bool wide = H->rg > fa::kMaxRadius || H->rw > fa::kMaxRadius;
  if (need > H->cap || (wide && !H->wide)) {
    float** bufs[] = {&H->e, &H->m, &H->v, &H->a, &H->tmp, &H->wide};
    for (float** b : bufs) {
      if (*b) (void)hipFree(*b);
      *b = nullptr;
    }
    if (H->acc) (void)hipFree(H->acc);
    H->acc = nullptr;
    if (H->partials) (void)hipFree(H->partials);
    H->partials = nullptr;
    H->cap = 0;
    for (int k = 0; k < (wide ? 6 : 5); ++k) FA_TRY(ialloc(bufs[k], (size_t)(3 * need), "state"));
    FA_TRY(ialloc(&H->acc, (size_t)(3 * need), "splat accumulator"));
    FA_TRY(ialloc(&H->partials, (size_t)(2 * kInvMaxBlocks), "cost partials"));
    H->cap = need;
  }
  FA_HIP(hipMemsetAsync(H->acc, 0, (size_t)(3 * H->cap) * sizeof(unsigned long long), H->stream));
  if (total > H->loss_cap) {
    if (H->loss_hist) (void)hipFree(H->loss_hist);
    H->loss_hist = nullptr;
    H->loss_cap = 0;
    FA_TRY(ialloc(&H->loss_hist, (size_t)total, "loss history"));
    H->loss_cap = (int)total;
  }

  // pyramid of the warp's field; e, m, v, a serve as blur scratch before the state is set
  H->levels = lv;
  for (int i = 0; i < n_levels; ++i) {
    ILevel& L = H->levels[i];
    if (L.scale == 1.0f && L.shape.n0 == H->shape.n0 && L.shape.n1 == H->shape.n1 && L.shape.n2 == H->shape.n2) {
      L.d = H->in_d;
      L.owns = false;
      continue;
    }
    FA_TRY(ialloc(&L.d, (size_t)(3 * L.n), "level field"));
    L.owns = true;
    // blur scratch: two volumes in m, the blurred field in e (both hold 3 input-sized volumes)
    float* p0p1 = H->m;
    float* blurred = H->e;
    const fa_shape& s = H->shape;
    const int64_t n = H->n;
    const int rad = fa::tap_radius(L.scale / 2.0f);
    const float* w = H->wts + off_blur[i];
    for (int c = 0; c < 3; ++c) {
      FA_HIP(fa::launch_blur_axis(H->in_d + c * n, p0p1, s.n0, s.n1, s.n2, 0, w, rad, H->stream));
      FA_HIP(fa::launch_blur_axis(p0p1, p0p1 + n, s.n0, s.n1, s.n2, 1, w, rad, H->stream));
      FA_HIP(fa::launch_blur_axis(p0p1 + n, blurred + c * n, s.n0, s.n1, s.n2, 2, w, rad, H->stream));
    }
    auto inv_rho = [](int nf, int nc) { return nc > 1 ? (float)((double)(nc - 1) / (double)(nf - 1)) : 1.0f; };
    FA_HIP(fa::launch_resample(blurred, L.d, s.n0, s.n1, s.n2, L.shape.n0, L.shape.n1, L.shape.n2, 3,
                               inv_rho(s.n0, L.shape.n0), inv_rho(s.n1, L.shape.n1), inv_rho(s.n2, L.shape.n2),
                               H->stream));
  }

  // psi = id, m = v = 0, t = 0
  const int64_t n0 = H->levels[0].n;
  FA_HIP(fa::launch_fill(H->e, 0.0f, 3 * n0, H->stream));
  FA_HIP(fa::launch_fill(H->m, 0.0f, 3 * n0, H->stream));
  FA_HIP(fa::launch_fill(H->v, 0.0f, 3 * n0, H->stream));
  FA_HIP(fa::launch_fill(H->a, 0.0f, 3 * n0, H->stream));
  FA_HIP(fa::launch_ctl_init(H->ctl, H->p.adam_beta1, H->p.adam_beta2, 0, 0, H->stream));
  H->cur_level = 0;
  H->cur_iter = 0;
  H->t_done = 0;
  H->iters_done = 0;
  H->scheduled = true;
  return FA_OK;
}

fa_status fa_inverse_step(fa_inverse H, int max_iters, int* iters_done, int* finished) {
  if (iters_done) *iters_done = 0;
  if (finished) *finished = 0;
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!H->scheduled) return fail(FA_ESTATE, "fa_inverse_set_schedule has not been called");
  if (max_iters < 0) return fail(FA_EINVAL, "max_iters must be >= 0");
  int done = 0;
  while (done < max_iters) {
    while (H->cur_level + 1 < (int)H->levels.size() && H->cur_iter >= H->levels[H->cur_level].iters) {
      FA_TRY(transition(H));
      H->cur_level += 1;
      H->cur_iter = 0;
    }
    if (schedule_done(H)) break;
    FA_TRY(launch_iteration(H, H->levels[H->cur_level]));
    H->cur_iter += 1;
    H->t_done += 1;
    H->iters_done += 1;
    done += 1;
  }
  if (iters_done) *iters_done = done;
  if (finished) *finished = schedule_done(H) ? 1 : 0;
  return FA_OK;
}

fa_status fa_inverse_get_field(fa_inverse H, float* dev_out, int* level, fa_shape* shape) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!H->scheduled) return fail(FA_ESTATE, "fa_inverse_set_schedule has not been called");
  const ILevel& L = H->levels[H->cur_level];
  if (level) *level = H->cur_level;
  if (shape) *shape = L.shape;
  if (dev_out)
    FA_HIP(hipMemcpyAsync(dev_out, H->e, (size_t)(3 * L.n) * sizeof(float), hipMemcpyDeviceToDevice, H->stream));
  return FA_OK;
}

fa_status fa_inverse_get_loss(fa_inverse H, float* host_out, int capacity, int* n_written) {
  if (n_written) *n_written = 0;
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!host_out && capacity > 0) return fail(FA_EINVAL, "host_out is NULL");
  const int cnt = std::min(std::max(capacity, 0), H->scheduled ? std::min(H->iters_done, H->loss_cap) : 0);
  FA_HIP(hipStreamSynchronize(H->stream));
  if (cnt > 0) FA_HIP(hipMemcpy(host_out, H->loss_hist, (size_t)cnt * sizeof(float), hipMemcpyDeviceToHost));
  if (n_written) *n_written = cnt;
  return FA_OK;
}

fa_status fa_inverse_eval_gradient(fa_inverse H, float* g_dev, float* loss_host) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!g_dev) return fail(FA_EINVAL, "g_dev is NULL");
  if (!H->scheduled) return fail(FA_ESTATE, "fa_inverse_set_schedule has not been called");
  const ILevel& L = H->levels[H->cur_level];
  FA_TRY(launch_direction(H, L, g_dev, 1));
  FA_HIP(fa::launch_partials_ratio(H->partials, 2 * inv_blocks(L.n), -(double)L.n, H->scalar, H->stream));
  if (loss_host) {
    FA_HIP(hipMemcpyAsync(loss_host, H->scalar, sizeof(float), hipMemcpyDeviceToHost, H->stream));
    FA_HIP(hipStreamSynchronize(H->stream));
  }
  return FA_OK;
}

fa_status fa_inverse_set_splat(fa_inverse H, int direct) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (direct != 0 && direct != 1) return fail(FA_EINVAL, "direct must be 0 or 1");
  H->splat_direct = direct != 0;
  return FA_OK;
}

void fa_inverse_destroy(fa_inverse H) {
  if (!H) return;
  (void)hipStreamSynchronize(H->stream);
  free_all(H);
  delete H;
}

}  // extern "C"
