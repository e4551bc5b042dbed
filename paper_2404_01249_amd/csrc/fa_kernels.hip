// HIP kernels (gfx950) of the FireANTs dense matching step.
//
// One iteration of Algorithm 1 runs as four streaming launches:
//
//   grad   : warp J = I_m(x + d), LNCC window statistics, LNCC adjoint, the
//            Gateaux gradient g = dL/dJ * grad_p I_m (Jacobian-free Eulerian
//            descent, Section 4.4.2) and the Adam update (Section 4.4) ->
//            m, v, direction a; per-workgroup loss partials.
//   gauss  : s = G_sigma_grad * a stored, M = max |s|     (EPI_SMOOTH_MAX)
//   gauss  : single tap: u = -eta s / (2M) (Appendix E), d' = u + d(x + u)
//            (the retraction phi o (id + u) of Algorithm 1)  (EPI_COMPOSE_LDS)
//   gauss  : d = G_sigma_warp * d'                          (EPI_STORE)
// The first workgroup of the composition, or of the warp smoothing where that
// is a brick launch, also records the loss and advances the Adam step count.
//
// Every streaming kernel gives a workgroup an in-plane tile (TY x TX columns
// along n1, n2) and marches it along n0 over a chunk of planes.  Window sums
// and Gaussian taps along n0 come from per-column register rings; the in-plane
// parts are separable passes over halo tiles staged in LDS.  The path is a
// stencil-and-gather workload bound by HBM bandwidth; there is no dense
// contraction, so no MFMA.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "fa_internal.h"

namespace fa {
namespace {

__device__ __forceinline__ int vidx(int z, int y, int x, int n1, int n2) {
  return (z * n1 + y) * n2 + x;
}

// M = max |s| over the slots of Ctl::mslot: cleared by threads 0..kMSlots-1
// of one workgroup, raised with one atomicMax per workgroup on the slot of
// its XCD (workgroups go to the XCDs round robin by linear index), read as
// the largest slot.
__device__ __forceinline__ void m_clear(Ctl* c, int tid) {
  if (tid < kMSlots) c->mslot[tid * kMStride] = 0u;
}
__device__ __forceinline__ void m_raise(Ctl* c, float bm, unsigned linear_block) {
  atomicMax(&c->mslot[(linear_block % kMSlots) * kMStride], __float_as_uint(bm));
}
__device__ __forceinline__ float m_value(const Ctl* c) {
  unsigned m = c->mslot[0];
#pragma unroll
  for (int j = 1; j < kMSlots; ++j) m = max(m, c->mslot[j * kMStride]);
  return __uint_as_float(m);
}

// Cell index and fraction of a sample coordinate, plus whether the lower and
// upper corners lie on the grid.  Coordinates far outside are clamped first
// (all corners are then off the grid anyway), which also keeps the integer
// conversion defined.
__device__ __forceinline__ void cell(float p, int n, int& i, float& t, bool& lo, bool& hi) {
  p = clamp_med3(p, -2.0f, (float)n + 1.0f);
  const float f = floorf(p);
  i = (int)f;
  t = p - f;
  lo = (i >= 0) & (i < n);
  hi = (i >= -1) & (i + 1 < n);
}

// Load with per-corner zero padding; the address is always in bounds.
__device__ __forceinline__ float ldz(const float* __restrict__ f, int idx, bool ok) {
  const float v = f[ok ? idx : 0];
  return ok ? v : 0.0f;
}

// The same for a sample at grid point x displaced by dd.  The cell index is
// x + floor(dd) and the fraction dd - floor(dd), so no precision is lost to
// forming x + dd in fp32: the cell is exactly the cell of the exact position
// (the trilinear derivative jumps between cells, so the cell matters) and the
// fraction is exact up to at most half an ulp of 1.
__device__ __forceinline__ void cell_at(int x, float dd, int n, int& i, float& t, bool& lo, bool& hi) {
  dd = clamp_med3(dd, (float)(-x - 2), (float)(n + 1 - x));
  const float f = floorf(dd);
  i = x + (int)f;
  t = dd - f;
  lo = (i >= 0) & (i < n);
  hi = (i >= -1) & (i + 1 < n);
}

struct Corners {
  int base, s0, s1;
  bool a0, b0, a1, b1, a2, b2;
  float t0, t1, t2;
};

// Corners of the sample at grid point (z, y, x) + (d0, d1, d2).
__device__ __forceinline__ Corners corners_at(int n0, int n1, int n2, int z, int y, int x, float d0,
                                              float d1, float d2) {
  Corners c;
  int i0, i1, i2;
  cell_at(z, d0, n0, i0, c.t0, c.a0, c.b0);
  cell_at(y, d1, n1, i1, c.t1, c.a1, c.b1);
  cell_at(x, d2, n2, i2, c.t2, c.a2, c.b2);
  c.s1 = n2;
  c.s0 = n1 * n2;
  c.base = (i0 * n1 + i1) * n2 + i2;
  return c;
}

__device__ __forceinline__ Corners make_corners(int n0, int n1, int n2, float p0, float p1, float p2) {
  Corners c;
  int i0, i1, i2;
  cell(p0, n0, i0, c.t0, c.a0, c.b0);
  cell(p1, n1, i1, c.t1, c.a1, c.b1);
  cell(p2, n2, i2, c.t2, c.a2, c.b2);
  c.s1 = n2;
  c.s0 = n1 * n2;
  c.base = (i0 * n1 + i1) * n2 + i2;
  return c;
}

// Trilinear sample T(f, p), zero outside the grid (per corner).
__device__ __forceinline__ float tri(const float* __restrict__ f, const Corners& c) {
  const float c000 = ldz(f, c.base, c.a0 & c.a1 & c.a2);
  const float c001 = ldz(f, c.base + 1, c.a0 & c.a1 & c.b2);
  const float c010 = ldz(f, c.base + c.s1, c.a0 & c.b1 & c.a2);
  const float c011 = ldz(f, c.base + c.s1 + 1, c.a0 & c.b1 & c.b2);
  const float c100 = ldz(f, c.base + c.s0, c.b0 & c.a1 & c.a2);
  const float c101 = ldz(f, c.base + c.s0 + 1, c.b0 & c.a1 & c.b2);
  const float c110 = ldz(f, c.base + c.s0 + c.s1, c.b0 & c.b1 & c.a2);
  const float c111 = ldz(f, c.base + c.s0 + c.s1 + 1, c.b0 & c.b1 & c.b2);
  const float e00 = c000 + c.t2 * (c001 - c000);
  const float e01 = c010 + c.t2 * (c011 - c010);
  const float e10 = c100 + c.t2 * (c101 - c100);
  const float e11 = c110 + c.t2 * (c111 - c110);
  const float f0 = e00 + c.t1 * (e01 - e00);
  const float f1 = e10 + c.t1 * (e11 - e10);
  return f0 + c.t0 * (f1 - f0);
}

// T(f, p) and dT/dp (the trilinear weight along one axis replaced by -1/+1;
// at integer coordinates this is the derivative from the right).
__device__ __forceinline__ float tri_grad(const float* __restrict__ f, const Corners& c,
                                          float& g0, float& g1, float& g2) {
  const float c000 = ldz(f, c.base, c.a0 & c.a1 & c.a2);
  const float c001 = ldz(f, c.base + 1, c.a0 & c.a1 & c.b2);
  const float c010 = ldz(f, c.base + c.s1, c.a0 & c.b1 & c.a2);
  const float c011 = ldz(f, c.base + c.s1 + 1, c.a0 & c.b1 & c.b2);
  const float c100 = ldz(f, c.base + c.s0, c.b0 & c.a1 & c.a2);
  const float c101 = ldz(f, c.base + c.s0 + 1, c.b0 & c.a1 & c.b2);
  const float c110 = ldz(f, c.base + c.s0 + c.s1, c.b0 & c.b1 & c.a2);
  const float c111 = ldz(f, c.base + c.s0 + c.s1 + 1, c.b0 & c.b1 & c.b2);
  const float dx00 = c001 - c000, dx01 = c011 - c010, dx10 = c101 - c100, dx11 = c111 - c110;
  const float e00 = c000 + c.t2 * dx00;
  const float e01 = c010 + c.t2 * dx01;
  const float e10 = c100 + c.t2 * dx10;
  const float e11 = c110 + c.t2 * dx11;
  const float dy0 = e01 - e00, dy1 = e11 - e10;
  const float f0 = e00 + c.t1 * dy0;
  const float f1 = e10 + c.t1 * dy1;
  const float dxy0 = dx00 + c.t1 * (dx01 - dx00);
  const float dxy1 = dx10 + c.t1 * (dx11 - dx10);
  g0 = f1 - f0;
  g1 = dy0 + c.t0 * (dy1 - dy0);
  g2 = dxy0 + c.t0 * (dxy1 - dxy0);
  return f0 + c.t0 * (f1 - f0);
}

// Number of grid points of [i - r, i + r] inside [0, n).
__device__ __forceinline__ float clipped_count(int i, int n, int r) {
  return (float)(min(i + r, n - 1) - max(i - r, 0) + 1);
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, each i a compile-time
// constant in f's body.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Box sums of two neighbouring outputs along a row: out[0] = in[0] + ... +
// in[W-1] and out[1] = in[1] + ... + in[W], each added left to right as a
// single output would be.  W is odd and in and out are 8-byte aligned, so the
// W + 1 inputs arrive as (W + 1) / 2 pair reads and the outputs as one pair
// write.
template <int W>
__device__ __forceinline__ void box_pair_x(const float* in, float* out) {
  float v[W + 1];
#pragma unroll
  for (int k = 0; k < (W + 1) / 2; ++k) {
    const float2 t = reinterpret_cast<const float2*>(in)[k];
    v[2 * k] = t.x;
    v[2 * k + 1] = t.y;
  }
  float a = v[0], b = v[1];
#pragma unroll
  for (int k = 1; k < W; ++k) {
    a += v[k];
    b += v[k + 1];
  }
  reinterpret_cast<float2*>(out)[0] = make_float2(a, b);
}

// The same with tap weights w[0..L-1]: out[0] = sum_k w[k] in[k] and out[1]
// = sum_k w[k] in[k + 1], each accumulated from k = 0 upwards.
template <int L>
__device__ __forceinline__ void tap_pair_x(const float* in, float* out, const float* w) {
  float v[L + 1];
#pragma unroll
  for (int k = 0; k < (L + 1) / 2; ++k) {
    const float2 t = reinterpret_cast<const float2*>(in)[k];
    v[2 * k] = t.x;
    v[2 * k + 1] = t.y;
  }
  float a = w[0] * v[0], b = w[0] * v[1];
#pragma unroll
  for (int k = 1; k < L; ++k) {
    a += w[k] * v[k];
    b += w[k] * v[k + 1];
  }
  reinterpret_cast<float2*>(out)[0] = make_float2(a, b);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that every XCD works through a contiguous range of
// tiles: neighbouring tiles then share their halo reads in one L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  constexpr int X = 8;
  const int q = G / X, r = G % X;
  const int x = b % X, k = b / X;
  return x * q + min(x, r) + k;
}

template <int NT>
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  return s;  // meaningful on thread 0
}

template <int NT>
__device__ float block_max(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float s = 0.0f;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s = fmaxf(s, red[i]);
  }
  return s;
}

// ---------------------------------------------------------------------------
// Fused warp + LNCC + adjoint + Adam.
//
// Stage 1 (window statistics) runs on the tile plus a 2r halo: each column
// keeps the last W planes of I and J in registers, sums them along n0, and
// the in-plane box sums are two passes over LDS.  Stage 2 (adjoint box sums of
// the per-centre coefficients A, B, C) runs on the tile plus an r halo:
// in-plane passes first, then a register ring along n0.  The output plane
// lags the input plane by 2r.
//
// Every thread's first stage-1 column is its own output column, so the
// output stage finds I, J and grad_p I_m at its plane in the oldest ring
// entries instead of sampling the moving image a second time.  The loads and
// gathers of the next input plane, and the Adam moments of the next output
// plane, are issued before the current plane's LDS passes and consumed after
// them (a two-stage software pipeline across the barriers).
// ---------------------------------------------------------------------------

// Trilinear gathers as 32-bit byte offsets from a uniform base pointer (the
// global loads then take the scalar-base form, with no per-lane 64-bit address
// arithmetic).  Every offset stays inside the volume (an axis whose corner is
// off the grid contributes offset 0), and an 8-bit mask zeroes the off-grid
// corners when the values are consumed.
__device__ __forceinline__ float load_at(const float* __restrict__ base, unsigned byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (size_t)byte_off);
}

__device__ __forceinline__ void store_at(float* __restrict__ base, unsigned byte_off, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (size_t)byte_off) = v;
}

__device__ __forceinline__ void axis_offsets(int x, float dd, int n, int stride_bytes, unsigned& lo,
                                             unsigned& hi, bool& lo_ok, bool& hi_ok, float& t) {
  dd = clamp_med3(dd, (float)(-x - 2), (float)(n + 1 - x));
  const float f = floorf(dd);
  const int i = x + (int)f;
  t = dd - f;
  lo_ok = i >= 0 && i < n;
  hi_ok = i >= -1 && i + 1 < n;
  lo = lo_ok ? (unsigned)(i * stride_bytes) : 0u;
  hi = hi_ok ? (unsigned)((i + 1) * stride_bytes) : 0u;
}

// The 8 corner offsets, validity mask and fractions of the sample at grid
// point (z, y, x) displaced by (d0, d1, d2); the cell is x + floor(d) as in
// cell_at.
struct Cell8 {
  unsigned off[8];
  unsigned mask;
  float t0, t1, t2;
};

__device__ __forceinline__ Cell8 cell8_at(int n0, int n1, int n2, int z, int y, int x, float d0, float d1,
                                          float d2) {
  Cell8 c;
  unsigned l0, h0, l1, h1, l2, h2;
  bool a0, b0, a1, b1, a2, b2;
  axis_offsets(z, d0, n0, n1 * n2 * 4, l0, h0, a0, b0, c.t0);
  axis_offsets(y, d1, n1, n2 * 4, l1, h1, a1, b1, c.t1);
  axis_offsets(x, d2, n2, 4, l2, h2, a2, b2, c.t2);
  const unsigned a00 = l0 + l1, a01 = l0 + h1, a10 = h0 + l1, a11 = h0 + h1;
  c.off[0] = a00 + l2;
  c.off[1] = a00 + h2;
  c.off[2] = a01 + l2;
  c.off[3] = a01 + h2;
  c.off[4] = a10 + l2;
  c.off[5] = a10 + h2;
  c.off[6] = a11 + l2;
  c.off[7] = a11 + h2;
  const unsigned mz = (a0 ? 0x0Fu : 0u) | (b0 ? 0xF0u : 0u);
  const unsigned my = (a1 ? 0x33u : 0u) | (b1 ? 0xCCu : 0u);
  const unsigned mx = (a2 ? 0x55u : 0u) | (b2 ? 0xAAu : 0u);
  c.mask = mz & my & mx;
  return c;
}

// The same for a volume stored with a zero border of kPad voxels on every
// side (padded strides).  The cell is clamped to [-kPad, n], so every corner
// lies in the padded volume, and a corner off the grid reads a zero of the
// border: no mask is needed (the mask is constant, and the selects fold
// away).  A sample clamped this way lies wholly in the border, so its value
// and derivative are 0, as with the masked form.
__device__ __forceinline__ void axis_offsets_pad(int x, float dd, int n, int stride_bytes, unsigned& lo,
                                                 unsigned& hi, float& t) {
  dd = clamp_med3(dd, (float)(-x - kPad), (float)(n - x));
  const float f = floorf(dd);
  const int i = x + kPad + (int)f;   // padded index, in [0, n + kPad]
  t = dd - f;
  lo = (unsigned)(i * stride_bytes);
  hi = lo + (unsigned)stride_bytes;
}

__device__ __forceinline__ Cell8 cell8_pad(int n0, int n1, int n2, int z, int y, int x, float d0, float d1,
                                           float d2) {
  Cell8 c;
  const int p2 = n2 + 2 * kPad, p1 = n1 + 2 * kPad;
  unsigned l0, h0, l1, h1, l2, h2;
  axis_offsets_pad(z, d0, n0, p1 * p2 * 4, l0, h0, c.t0);
  axis_offsets_pad(y, d1, n1, p2 * 4, l1, h1, c.t1);
  axis_offsets_pad(x, d2, n2, 4, l2, h2, c.t2);
  const unsigned a00 = l0 + l1, a01 = l0 + h1, a10 = h0 + l1, a11 = h0 + h1;
  c.off[0] = a00 + l2;
  c.off[1] = a00 + h2;
  c.off[2] = a01 + l2;
  c.off[3] = a01 + h2;
  c.off[4] = a10 + l2;
  c.off[5] = a10 + h2;
  c.off[6] = a11 + l2;
  c.off[7] = a11 + h2;
  c.mask = 0xFFu;
  return c;
}

// Eight corner values of a trilinear sample (loaded; consumed later so that
// issuing the loads does not wait for them).
struct Gather {
  float c[8];
  unsigned mask;
  float t0, t1, t2;
};

__device__ __forceinline__ void gather_issue(const float* __restrict__ f, const Cell8& c, Gather& g) {
#pragma unroll
  for (int k = 0; k < 8; ++k) g.c[k] = load_at(f, c.off[k]);
  g.mask = c.mask;
  g.t0 = c.t0;
  g.t1 = c.t1;
  g.t2 = c.t2;
}

// The padded moving image stored as corner quads (launch_pad_quad): entry
// (z, y, x) of the padded grid holds the padded values at (z, y, x),
// (z, y, x+1), (z, y+1, x) and (z, y+1, x+1).  A trilinear sample then takes
// two aligned 16-byte loads (planes z and z+1 of its cell) instead of eight
// 4-byte ones, and the corners arrive in gather_issue's order, so the values
// and every result are the same.  Byte offsets are 32-bit unsigned (the quad
// array stays below 4 GiB), and the padded plane size and every padded index
// stay below 2^24, so the index products are full-rate 24-bit multiplies (the
// runtime checks both: quad_supported).
__device__ __forceinline__ void quad_axis(int x, float dd, int n, unsigned stride_quads, unsigned& lo, float& t) {
  dd = clamp_med3(dd, (float)(-x - kPad), (float)(n - x));
  const float f = floorf(dd);
  lo = __umul24((unsigned)(x + kPad + (int)f), stride_quads);   // padded index in [0, n + kPad]
  t = dd - f;
}

__device__ __forceinline__ void gather_issue_quad(const float* __restrict__ q, int n0, int n1, int n2, int z,
                                                  int y, int x, float d0, float d1, float d2, Gather& g) {
  const unsigned p2 = (unsigned)(n2 + 2 * kPad), p1 = (unsigned)(n1 + 2 * kPad);
  unsigned l0, l1, l2;
  quad_axis(z, d0, n0, p1 * p2, l0, g.t0);
  quad_axis(y, d1, n1, p2, l1, g.t1);
  quad_axis(x, d2, n2, 1u, l2, g.t2);
  const char* b = reinterpret_cast<const char*>(q);
  const unsigned off = (l0 + l1 + l2) * 16u;
  const float4 lo = *reinterpret_cast<const float4*>(b + (size_t)off);
  const float4 hi = *reinterpret_cast<const float4*>(b + (size_t)(off + p1 * p2 * 16u));
  g.c[0] = lo.x;
  g.c[1] = lo.y;
  g.c[2] = lo.z;
  g.c[3] = lo.w;
  g.c[4] = hi.x;
  g.c[5] = hi.y;
  g.c[6] = hi.z;
  g.c[7] = hi.w;
  g.mask = 0xFFu;
}

__device__ __forceinline__ float gather_value(const Gather& g) {
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = ((g.mask >> k) & 1u) ? g.c[k] : 0.0f;
  const float e00 = v[0] + g.t2 * (v[1] - v[0]);
  const float e01 = v[2] + g.t2 * (v[3] - v[2]);
  const float e10 = v[4] + g.t2 * (v[5] - v[4]);
  const float e11 = v[6] + g.t2 * (v[7] - v[6]);
  const float f0 = e00 + g.t1 * (e01 - e00);
  const float f1 = e10 + g.t1 * (e11 - e10);
  return f0 + g.t0 * (f1 - f0);
}

__device__ __forceinline__ float gather_value_grad(const Gather& g, float& g0, float& g1, float& g2) {
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = ((g.mask >> k) & 1u) ? g.c[k] : 0.0f;
  const float dx00 = v[1] - v[0], dx01 = v[3] - v[2], dx10 = v[5] - v[4], dx11 = v[7] - v[6];
  const float e00 = v[0] + g.t2 * dx00;
  const float e01 = v[2] + g.t2 * dx01;
  const float e10 = v[4] + g.t2 * dx10;
  const float e11 = v[6] + g.t2 * dx11;
  const float dy0 = e01 - e00, dy1 = e11 - e10;
  const float f0 = e00 + g.t1 * dy0;
  const float f1 = e10 + g.t1 * dy1;
  const float dxy0 = dx00 + g.t1 * (dx01 - dx00);
  const float dxy1 = dx10 + g.t1 * (dx11 - dx10);
  g0 = f1 - f0;
  g1 = dy0 + g.t0 * (dy1 - dy0);
  g2 = dxy0 + g.t0 * (dxy1 - dxy0);
  return f0 + g.t0 * (f1 - f0);
}

// Stage-1 column `slot` of thread `tid` as (row, column) of the halo tile.
// Slot 0 is the thread's own output column; the remaining slots enumerate
// the halo bands (top, bottom, left, right).
template <int TY, int TX, int H>
__device__ __forceinline__ bool slot_coords(int tid, int slot, int& ey, int& ex) {
  constexpr int NT = TY * TX;
  constexpr int EX = TX + 2 * H;
  if (slot == 0) {
    ey = H + tid / TX;
    ex = H + tid % TX;
    return true;
  }
  if constexpr (H == 0) {
    ey = ex = 0;
    return false;
  } else {
  const int h = tid + (slot - 1) * NT;
  constexpr int TB = H * EX;       // one horizontal band
  constexpr int LB = TY * H;       // one vertical band
  if (h < TB) {
    ey = h / EX;
    ex = h % EX;
  } else if (h < 2 * TB) {
    ey = H + TY + (h - TB) / EX;
    ex = (h - TB) % EX;
  } else if (h < 2 * TB + LB) {
    ey = H + (h - 2 * TB) / H;
    ex = (h - 2 * TB) % H;
  } else if (h < 2 * TB + 2 * LB) {
    ey = H + (h - 2 * TB - LB) / H;
    ex = H + TX + (h - 2 * TB - LB) % H;
  } else {
    ey = ex = 0;
    return false;
  }
  return true;
  }
}

// MODE: A.mode fixed at compile time (0, 1 or 2), or -1 to read it at run time.
template <int W, int TY, int TX, bool PIPE, bool QUAD = false, int MODE = -1>
__device__ __forceinline__ void grad_body(const GradArgs& A, const int tile) {
  const int mode = MODE >= 0 ? MODE : A.mode;
  constexpr int R = W / 2;
  constexpr int NT = TY * TX;
  constexpr int E1Y = TY + 4 * R, E1X = TX + 4 * R, E1 = E1Y * E1X;
  constexpr int E2Y = TY + 2 * R, E2X = TX + 2 * R, E2 = E2Y * E2X;
  constexpr int XS1 = E1Y * E2X;
  constexpr int XS2 = E2Y * TX;
  constexpr int CPT1 = 1 + (E1 - NT + NT - 1) / NT;   // own column + halo columns
  // The in-plane x passes give each thread two neighbouring outputs (pair
  // reads along rows): every row length and array offset below is even.
  static_assert(TX % 2 == 0 && W % 2 == 1, "pairs need an even tile width and an odd window");
  extern __shared__ __attribute__((aligned(16))) float glds[];
  float* buf = glds;             // [5][E1], later [3][E2]
  float* bufx = glds + 5 * E1;   // [5][XS1], later [3][XS2]
  // grad_p I_m of the own column, delayed 2r planes from the input plane
  // to the output plane: a per-thread delay line of GS slots in LDS (slot
  // z mod GS).  Each thread touches only its own entries, so no barrier is
  // involved; with r > 0 a plane is stored after the output stage has read
  // the slot it replaces.
  constexpr int GS = (R == 0) ? 1 : 2 * R;
  // in LDS while the kernel's LDS stays within 64 KiB, else in registers
  constexpr bool GLDS = sizeof(float) * (5 * E1 + 5 * XS1 + 3 * GS * NT) <= 65536;
  float* gring = glds + 5 * E1 + 5 * XS1;   // [GS][3][NT] when GLDS
  float greg[3][GS];                       // when !GLDS: oldest entry first
#pragma unroll
  for (int j = 0; j < GS; ++j) greg[0][j] = greg[1][j] = greg[2][j] = 0.0f;

  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  int b = tile;
  const int bx = b % A.tiles_x;
  b /= A.tiles_x;
  const int by = b % A.tiles_y;
  b /= A.tiles_y;
  const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
  const int N = n0 * n1 * n2;
  const int z0 = b * A.zc;
  const int z1 = min(z0 + A.zc, n0);
  const int y0 = by * TY, x0 = bx * TX;

  int cy[CPT1], cx[CPT1], cl[CPT1];
  bool cin[CPT1], cuse[CPT1];
#pragma unroll
  for (int k = 0; k < CPT1; ++k) {
    int ey, ex;
    cuse[k] = slot_coords<TY, TX, 2 * R>(tid, k, ey, ex);
    cl[k] = ey * E1X + ex;
    cy[k] = y0 - 2 * R + ey;
    cx[k] = x0 - 2 * R + ex;
    cin[k] = cuse[k] && cy[k] >= 0 && cy[k] < n1 && cx[k] >= 0 && cx[k] < n2;
  }
  const int oy = tid / TX, ox = tid % TX;
  const int gy = y0 + oy, gx = x0 + ox;
  const bool out_col = gy < n1 && gx < n2;   // == cin[0]

  // per-thread entries of the window-statistics pass (tile + r halo): LDS
  // offset, in-plane window count (0 off the grid) and whether the entry is
  // a tile voxel whose cc enters the loss; fixed across planes
  constexpr int CPT2 = (E2 + NT - 1) / NT;
  int e2off[CPT2];
  float e2cnt[CPT2];
  bool e2own[CPT2];
#pragma unroll
  for (int k = 0; k < CPT2; ++k) {
    const int c = tid + k * NT;
    const int yo = c / E2X, xo = c - yo * E2X;
    const int yy = y0 - R + yo, xx = x0 - R + xo;
    e2off[k] = yo * E2X + xo;
    const bool ok = c < E2 && yy >= 0 && yy < n1 && xx >= 0 && xx < n2;
    e2cnt[k] = ok ? clipped_count(yy, n1, R) * clipped_count(xx, n2, R) : 0.0f;
    e2own[k] = ok && yo >= R && yo < R + TY && xo >= R && xo < R + TX;
  }

  float ringI[CPT1][W], ringJ[CPT1][W];
  float ringA[W], ringB[W], ringC[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
#pragma unroll
    for (int k = 0; k < CPT1; ++k) { ringI[k][j] = 0.0f; ringJ[k][j] = 0.0f; }
    ringA[j] = ringB[j] = ringC[j] = 0.0f;
  }

  const float ibc1 = 1.0f / A.ctl->bc1, ibc2 = 1.0f / A.ctl->bc2;
  if (mode == 0 && tile == 0) m_clear(A.ctl, tid);  // M of this iteration
  const float si = A.ctl->shift_i, sj = A.ctl->shift_j;
  const float gsc = (mode == 1 && A.gscale) ? *A.gscale : 1.0f;
  float lacc = 0.0f;   // this thread's cc sum over at most 2 zc columns

  const int zs = z0 - 2 * R, ze = z1 + 2 * R;

  // pipeline registers: raw loads of plane z+1 and gathers in flight
  float nd0[CPT1], nd1[CPT1], nd2[CPT1], nf[CPT1];
  Gather gq[CPT1];
  float curI[CPT1], curJ[CPT1], curG0 = 0.f, curG1 = 0.f, curG2 = 0.f;
  float nxI[CPT1];
  bool gv[CPT1];
  auto store_g = [&](int z) {
    if constexpr (GLDS) {
      float* gs = gring + (((z % GS) + GS) % GS) * 3 * NT + tid;
      gs[0] = curG0;
      gs[NT] = curG1;
      gs[2 * NT] = curG2;
    } else {
#pragma unroll
      for (int j = 0; j < GS - 1; ++j) {
        greg[0][j] = greg[0][j + 1];
        greg[1][j] = greg[1][j + 1];
        greg[2][j] = greg[2][j + 1];
      }
      greg[0][GS - 1] = curG0;
      greg[1][GS - 1] = curG1;
      greg[2][GS - 1] = curG2;
    }
  };

  auto load_raw = [&](int z, int k) {
    if (z >= 0 && z < n0 && cin[k]) {
      // byte offsets from uniform bases (volumes hold < 2^29 voxels)
      const unsigned off = (unsigned)vidx(z, cy[k], cx[k], n1, n2) * 4u;
      nd0[k] = load_at(A.d, off);
      nd1[k] = load_at(A.d + N, off);
      nd2[k] = load_at(A.d + 2 * N, off);
      nf[k] = load_at(A.fixed, off);
    }
  };
  auto issue_gather = [&](int z, int k) {
    gv[k] = z >= 0 && z < n0 && cin[k];
    if (gv[k]) {
      if constexpr (QUAD) {
        gather_issue_quad(A.moving_quad, n0, n1, n2, z, cy[k], cx[k], nd0[k], nd1[k], nd2[k], gq[k]);
      } else {
        const Cell8 c = cell8_pad(n0, n1, n2, z, cy[k], cx[k], nd0[k], nd1[k], nd2[k]);
        gather_issue(A.moving_pad, c, gq[k]);
      }
      nxI[k] = nf[k] - si;
    }
  };
  auto finish_gather = [&](int k) {
    if (gv[k]) {
      if (k == 0) {
        curJ[0] = gather_value_grad(gq[0], curG0, curG1, curG2) - sj;
      } else {
        curJ[k] = gather_value(gq[k]) - sj;
      }
      curI[k] = nxI[k];
    } else {
      curJ[k] = 0.0f;
      curI[k] = 0.0f;
      if (k == 0) curG0 = curG1 = curG2 = 0.0f;
    }
  };

  // prologue: plane zs in registers, plane zs+1 raw loads in flight
#pragma unroll
  for (int k = 0; k < CPT1; ++k) {
    load_raw(zs, k);
    issue_gather(zs, k);
    finish_gather(k);
    load_raw(zs + 1, k);
  }
  float pm[3] = {0.f, 0.f, 0.f}, pv[3] = {0.f, 0.f, 0.f};
  bool mv_ready = false;

  // The register rings of I, J (per column) and of the stage-2 sums hold the
  // last W planes.  Narrow windows rotate them by moves each plane step.  The
  // wide windows (one workgroup per CU, registers to spare) unroll the march
  // by W instead: at phase ph of W the newest entry goes to slot ph (slot
  // (ph + 1) mod W for the stage-2 ring, which starts 2r planes later), so
  // the j-th oldest entry sits at a slot fixed at compile time and no entry
  // moves.  The sums still run oldest first; the compiler may form a ring
  // entry's square or product once for the W windows that hold it instead of
  // fusing it into each sum, which changes the last bits.
  constexpr int UNZ = (W >= 7 && TY == 16) ? W : 1;   // not the 8-row tiles of thin volumes
  auto step = [&](const int zin, auto PH) __attribute__((always_inline)) {
    constexpr int ph = decltype(PH)::value;
    constexpr int pha = (ph + 1) % W;
    // slot of the j-th oldest entry of the I/J rings and of the stage-2 ring
    auto ri = [](int j) constexpr { return UNZ == 1 ? j : (ph + 1 + j) % W; };
    auto ra = [](int j) constexpr { return UNZ == 1 ? j : (pha + 1 + j) % W; };
#pragma unroll
    for (int k = 0; k < CPT1; ++k) {
      if constexpr (UNZ == 1) {
#pragma unroll
        for (int j = 0; j < W - 1; ++j) {
          ringI[k][j] = ringI[k][j + 1];
          ringJ[k][j] = ringJ[k][j + 1];
        }
        ringI[k][W - 1] = curI[k];
        ringJ[k][W - 1] = curJ[k];
      } else {
        ringI[k][ph] = curI[k];
        ringJ[k][ph] = curJ[k];
      }
    }
    if (R == 0) store_g(zin);
    // next plane: gathers in flight during this plane's passes (PIPE), or
    // issued after them (fewer live registers)
    if (PIPE) {
      // raised wave priority while the next plane's loads go out: they then
      // leave ahead of other waves' LDS passes (2% at 160x192x224; raising it
      // over the output stage as well gave the gain back)
      __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int k = 0; k < CPT1; ++k) {
        issue_gather(zin + 1, k);
        load_raw(zin + 2, k);
      }
      __builtin_amdgcn_s_setprio(0);
    }

    if (zin >= z0) {
#pragma unroll
      for (int k = 0; k < CPT1; ++k) {
        if (cuse[k]) {
          // sums start from the first term: 0 + x is not foldable in IEEE
          // arithmetic (signed zero) and would cost an add per sum
          const float i0 = ringI[k][ri(0)], j0 = ringJ[k][ri(0)];
          float s0 = i0, s1 = j0, s2 = i0 * i0, s3 = j0 * j0, s4 = i0 * j0;
#pragma unroll
          for (int j = 1; j < W; ++j) {
            const float i_ = ringI[k][ri(j)], j_ = ringJ[k][ri(j)];
            s0 += i_;
            s1 += j_;
            s2 += i_ * i_;
            s3 += j_ * j_;
            s4 += i_ * j_;
          }
          const int c = cl[k];
          buf[c] = s0;
          buf[E1 + c] = s1;
          buf[2 * E1 + c] = s2;
          buf[3 * E1 + c] = s3;
          buf[4 * E1 + c] = s4;
        }
      }
      __syncthreads();
      {
        // one quantity at a time, in a rolled loop (unrolled over the five
        // quantities the pass measured slower, and it crowds the register
        // budget)
        constexpr int HX = E2X / 2, PX = E1Y * HX;
        for (int p = tid; p < PX; p += NT) {
          const int yy = p / HX, xo = 2 * (p - yy * HX);
          const float* src = buf + yy * E1X + xo;
          float* dst = bufx + yy * E2X + xo;
#pragma unroll 1
          for (int q = 0; q < 5; ++q) box_pair_x<W>(src + q * E1, dst + q * XS1);
        }
      }
      __syncthreads();
      const int zc1 = zin - R;
      const bool z1ok = zc1 >= 0 && zc1 < n0;
      const float cz = clipped_count(zc1, n0, R);
      const bool z1out = zc1 >= z0 && zc1 < z1;
#pragma unroll
      for (int k2 = 0; k2 < CPT2; ++k2) {
        const int c = tid + k2 * NT;
        if (c >= E2) break;
        const float* src = bufx + e2off[k2];
        float SI = src[0], SJ = src[XS1], SII = src[2 * XS1], SJJ = src[3 * XS1], SIJ = src[4 * XS1];
#pragma unroll
        for (int k = 1; k < W; ++k) {
          SI += src[k * E2X];
          SJ += src[XS1 + k * E2X];
          SII += src[2 * XS1 + k * E2X];
          SJJ += src[3 * XS1 + k * E2X];
          SIJ += src[4 * XS1 + k * E2X];
        }
        float ca = 0.f, cb = 0.f, cc_ = 0.f;
        // A one-voxel window has zero variance and zero covariance exactly, so
        // its correlation and every coefficient are 0 (W == 1 skips the
        // arithmetic that would leave rounding residue).
        if (W > 1 && z1ok && e2cnt[k2] > 0.0f) {
          const float icnt = __builtin_amdgcn_rcpf(cz * e2cnt[k2]);
          const float muI = SI * icnt, muJ = SJ * icnt;
          const float cross = SIJ - muI * SJ;
          const float vI = SII - muI * SI;
          const float vJ = SJJ - muJ * SJ;
          const float D = vI * vJ + A.eps_cc;
          if (D != 0.0f) {
            const float invD = __builtin_amdgcn_rcpf(D);
            const float cc = cross * cross * invD;
            ca = 2.0f * cross * invD;
            cb = -2.0f * cc * vI * invD;
            cc_ = ca * muI + cb * muJ;
            if (z1out && e2own[k2]) lacc += cc;
          }
        }
        buf[c] = ca;
        buf[E2 + c] = cb;
        buf[2 * E2 + c] = cc_;
      }
      __syncthreads();
      {
        constexpr int HX = TX / 2, PX = E2Y * HX;
        for (int p = tid; p < PX; p += NT) {
          const int yy = p / HX, xo = 2 * (p - yy * HX);
          const float* src = buf + yy * E2X + xo;
          float* dst = bufx + yy * TX + xo;
#pragma unroll
          for (int q = 0; q < 3; ++q) box_pair_x<W>(src + q * E2, dst + q * XS2);
        }
      }
      __syncthreads();
      {
        const float* src = bufx + oy * TX + ox;
        float sa = src[0], sb = src[XS2], sc = src[2 * XS2];
#pragma unroll
        for (int k = 1; k < W; ++k) {
          sa += src[k * TX];
          sb += src[XS2 + k * TX];
          sc += src[2 * XS2 + k * TX];
        }
        if constexpr (UNZ == 1) {
#pragma unroll
          for (int j = 0; j < W - 1; ++j) {
            ringA[j] = ringA[j + 1];
            ringB[j] = ringB[j + 1];
            ringC[j] = ringC[j + 1];
          }
          ringA[W - 1] = sa;
          ringB[W - 1] = sb;
          ringC[W - 1] = sc;
        } else {
          ringA[pha] = sa;
          ringB[pha] = sb;
          ringC[pha] = sc;
        }
      }
      const int zc2 = zc1 - R;
      if (zc2 >= z0 && out_col) {
        const unsigned off = (unsigned)vidx(zc2, gy, gx, n1, n2) * 4u;
        if (mode == 0 && !mv_ready) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            pm[q] = load_at(A.m + q * N, off);
            pv[q] = load_at(A.v + q * N, off);
          }
        }
        float SA = ringA[ra(0)], SB = ringB[ra(0)], SC = ringC[ra(0)];
#pragma unroll
        for (int j = 1; j < W; ++j) {
          SA += ringA[ra(j)];
          SB += ringB[ra(j)];
          SC += ringC[ra(j)];
        }
        // oldest ring entries of the own column hold plane zc2
        const float dl = -A.inv_n * (ringI[0][ri(0)] * SA + ringJ[0][ri(0)] * SB - SC);
        float g[3];
        if constexpr (GLDS) {
          const float* gs = gring + (((zc2 % GS) + GS) % GS) * 3 * NT + tid;
          g[0] = dl * gs[0];
          g[1] = dl * gs[NT];
          g[2] = dl * gs[2 * NT];
        } else {
          g[0] = dl * greg[0][0];
          g[1] = dl * greg[1][0];
          g[2] = dl * greg[2][0];
        }
        if (mode == 0) {
          const float b1 = A.beta1, b2 = A.beta2;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const float mm = b1 * pm[q] + (1.0f - b1) * g[q];
            const float vv = b2 * pv[q] + (1.0f - b2) * g[q] * g[q];
            store_at(A.m + q * N, off, mm);
            store_at(A.v + q * N, off, vv);
            store_at(A.out + q * N, off, adam_direction(mm, vv, ibc1, ibc2, A.adam_eps));
          }
          // Adam moments of the next output plane
          mv_ready = zc2 + 1 < z1;
          if (mv_ready) {
            const unsigned noff = off + (unsigned)(n1 * n2) * 4u;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              pm[q] = load_at(A.m + q * N, noff);
              pv[q] = load_at(A.v + q * N, noff);
            }
          }
        } else if (mode == 1) {
#pragma unroll
          for (int q = 0; q < 3; ++q) store_at(A.out + q * N, off, g[q] * gsc);
        }
      }
    }
    if (R > 0) store_g(zin);
    if (!PIPE) {
#pragma unroll
      for (int k = 0; k < CPT1; ++k) {
        issue_gather(zin + 1, k);
        load_raw(zin + 2, k);
      }
    }
#pragma unroll
    for (int k = 0; k < CPT1; ++k) finish_gather(k);
  };
  if constexpr (UNZ == 1) {
    for (int zin = zs; zin < ze; ++zin) step(zin, std::integral_constant<int, 0>{});
  } else {
    // the guard is uniform across the workgroup, so the barriers inside
    // are reached by every thread or by none
    for (int zb = zs; zb < ze; zb += UNZ)
      static_for<UNZ>([&](auto PH) __attribute__((always_inline)) {
        if (zb + decltype(PH)::value < ze) step(zb + decltype(PH)::value, PH);
      });
  }
  const double tot = block_sum<NT>((double)lacc, red);
  if (tid == 0) A.partials[tile] = tot;
}

template <int W, int TY, int TX, bool PIPE, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TY * TX) k_grad(const GradArgs A) {
  grad_body<W, TY, TX, PIPE, QUAD, MODE>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// The same kernel compiled for two workgroups per CU (at most 128 VGPRs);
// used where that fits without spilling.
template <int W, int TY, int TX, bool PIPE, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TY * TX) __attribute__((amdgpu_waves_per_eu(4))) k_grad_o4(const GradArgs A) {
  grad_body<W, TY, TX, PIPE, QUAD, MODE>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Separable Gaussian (replicate boundary) on a 3-channel field, streaming.
// In-plane passes over a clamped halo tile in LDS, then a register ring of
// 2R+1 planes per output column along n0.  The next plane's loads are issued
// before the current plane's passes; the composition epilogue issues its
// gathers of d in one plane step and consumes them in the next.
// ---------------------------------------------------------------------------
// The iteration's loss record and Adam step count, run before its own work by
// the first workgroup of one launch after the gradient kernel (the launch
// whose GaussArgs carry the partials): the composition, or the warp smoothing
// where that is a brick launch (it costs the brick composition 0.6 us and the
// brick smoothing 0.1 us).  The gradient kernel of the iteration has written
// every loss partial, and no launch reads t or the bias corrections before
// the next iteration's gradient kernel.  No other workgroup waits for it, and
// the first workgroup is dispatched first.  The streaming smoothing launches
// never take it: inlined there, its registers cost occupancy or load
// pipelining at some radii.  The composition has registers to spare.  The partials are summed as 64-element
// chunks, each by one wave with the same shuffle tree, and the chunk sums in
// order by one thread: the sum does not depend on the workgroup size.
template <int NT>
__device__ __forceinline__ void record_iteration(const GaussArgs& A) {
  static_assert(NT % 64 == 0, "whole waves");
  constexpr int NW = NT / 64;
  __shared__ double csum[64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int n = A.n_partials, nch = (n + 63) / 64;
  // the counters are fetched with the partials: one memory round trip
  Ctl* C = A.ctl;
  const int it = C->iter, t = C->t;
  const double bp1 = C->bp1, bp2 = C->bp2;
  const float b1 = C->beta1, b2 = C->beta2;
  double s = 0.0;
  for (int c0 = 0; c0 < nch; c0 += 64) {   // rounds of at most 64 chunks
    const int cend = min(nch, c0 + 64);
    for (int c = c0 + wid; c < cend; c += NW) {
      const int i = c * 64 + lane;
      double v = i < n ? A.partials[i] : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) csum[c - c0] = v;
    }
    __syncthreads();
    if (tid == 0)
      for (int c = c0; c < cend; ++c) s += csum[c - c0];
    __syncthreads();
  }
  if (tid == 0) {
    if (A.loss_hist && it >= 0 && it < A.loss_cap) A.loss_hist[it] = (float)(-s * (double)A.inv_n);
    C->iter = it + 1;
    C->t = t + 1;
    const double p1 = bp1 * (double)b1, p2 = bp2 * (double)b2;
    C->bp1 = p1;
    C->bp2 = p2;
    C->bc1 = (float)(1.0 - p1);
    C->bc2 = (float)(1.0 - p2);
  }
}

template <int R, int TY, int TX, int EPI>
__device__ __forceinline__ void gauss_body(const GaussArgs& A, const int tile, const int nblocks) {
  constexpr int L = 2 * R + 1;
  constexpr int NT = TY * TX;
  constexpr int EY = TY + 2 * R, EX = TX + 2 * R, E = EY * EX;
  constexpr int XS = EY * TX;
  constexpr int CPT = (E + NT - 1) / NT;
  constexpr int DY = TY + 2, DX = TX + 2, DE = DY * DX;  // staged d planes (EPI_COMPOSE_LDS)
  // stride of the staged planes and components: DE rounded up to a multiple
  // of the 32 LDS banks, so that lanes of one row whose samples fall in
  // different planes (the sign of u0 flips along the row) read different
  // banks for different columns
  constexpr int DEP = (DE + 31) / 32 * 32;
  constexpr int CPTD = (DE + NT - 1) / NT;
  // the x pass gives each thread two neighbouring outputs (pair reads along
  // rows): EX, E, XS and every row offset are even
  static_assert(TX % 2 == 0, "pairs need an even tile width");
  extern __shared__ __attribute__((aligned(16))) float glds[];
  float* buf = glds;           // [3][E]
  float* bufx = glds + 3 * E;  // [3][XS]
  float* dring = glds + 3 * E + 3 * XS;  // [3 planes][3][DEP] (EPI_COMPOSE_LDS)
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  // the first tile of the composition records the iteration before its own work
  if ((EPI == EPI_COMPOSE_LDS || EPI == EPI_COMPOSE) && A.partials && tile == 0) record_iteration<NT>(A);
  int b = tile;
  const int bx = b % A.tiles_x;
  b /= A.tiles_x;
  const int by = b % A.tiles_y;
  b /= A.tiles_y;
  const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
  const int N = n0 * n1 * n2;
  const int z0 = b * A.zc;
  const int z1 = min(z0 + A.zc, n0);
  const int y0 = by * TY, x0 = bx * TX;
  const int oy = tid / TX, ox = tid % TX;
  const int gy = y0 + oy, gx = x0 + ox;
  const bool out_col = gy < n1 && gx < n2;

  // clamped in-plane offsets of this thread's halo-tile columns
  int coff[CPT];
  bool cuse[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    cuse[k] = c < E;
    const int yy = min(max(y0 - R + c / EX, 0), n1 - 1);
    const int xx = min(max(x0 - R + c % EX, 0), n2 - 1);
    coff[k] = yy * n2 + xx;
  }

  float w[L];
#pragma unroll
  for (int k = 0; k < L; ++k) w[k] = A.wts[k];
  float ring[3][L];
#pragma unroll
  for (int k = 0; k < L; ++k) ring[0][k] = ring[1][k] = ring[2][k] = 0.0f;

  float scale = 0.0f;
  if (EPI == EPI_COMPOSE || EPI == EPI_COMPOSE_LDS) {
    const float M = m_value(A.ctl);
    scale = M > 0.0f ? -A.eta / (2.0f * M) : 0.0f;
  }
  float mx = 0.0f;

  const int plane = n1 * n2;
  float pre[CPT][3];
  auto load_plane = [&](int z) {
    const int base = min(max(z, 0), n0 - 1) * plane;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (cuse[k]) {
        // byte offsets from uniform bases (volumes hold < 2^29 voxels)
        const unsigned off = (unsigned)(base + coff[k]) * 4u;
        pre[k][0] = load_at(A.in, off);
        pre[k][1] = load_at(A.in + N, off);
        pre[k][2] = load_at(A.in + 2 * N, off);
      }
    }
  };

  // d planes for the LDS composition: plane p lives in slot p mod 3 and
  // covers the tile plus one voxel on each side, zero off the grid (the
  // zero extension of the trilinear sample)
  float pd[CPTD][3];
  auto load_dplane = [&](int pz) {
#pragma unroll
    for (int k = 0; k < CPTD; ++k) {
      const int c = tid + k * NT;
      const int yy = y0 - 1 + c / DX, xx = x0 - 1 + c % DX;
      const bool ok = c < DE && pz >= 0 && pz < n0 && yy >= 0 && yy < n1 && xx >= 0 && xx < n2;
      const unsigned off = ok ? (unsigned)((pz * n1 + yy) * n2 + xx) * 4u : 0u;
      pd[k][0] = ok ? load_at(A.d, off) : 0.0f;
      pd[k][1] = ok ? load_at(A.d + N, off) : 0.0f;
      pd[k][2] = ok ? load_at(A.d + 2 * N, off) : 0.0f;
    }
  };
  auto store_dplane = [&](int pz) {
    const int slot = ((pz % 3) + 3) % 3;
#pragma unroll
    for (int k = 0; k < CPTD; ++k) {
      const int c = tid + k * NT;
      if (c < DE) {
        dring[(slot * 3 + 0) * DEP + c] = pd[k][0];
        dring[(slot * 3 + 1) * DEP + c] = pd[k][1];
        dring[(slot * 3 + 2) * DEP + c] = pd[k][2];
      }
    }
  };
  if (EPI == EPI_COMPOSE_LDS) {
    const int p0 = z0 - 2 * R + 1;   // plane stored by the first step (zin - R + 1)
    load_dplane(p0 - 2);
    store_dplane(p0 - 2);
    load_dplane(p0 - 1);
    store_dplane(p0 - 1);
    load_dplane(p0);
  }

  // composition gathers in flight (EPI_COMPOSE)
  Gather cg[3];
  float cu[3] = {0.f, 0.f, 0.f};
  int cidx = -1;
  auto finish_compose = [&]() {
    if (cidx >= 0) {
      A.out[cidx] = cu[0] + gather_value(cg[0]);
      A.out[N + cidx] = cu[1] + gather_value(cg[1]);
      A.out[2 * N + cidx] = cu[2] + gather_value(cg[2]);
      cidx = -1;
    }
  };

  load_plane(z0 - R);
  for (int zin = z0 - R; zin < z1 + R; ++zin) {
    if constexpr (R == 0) {
      // a single tap: the thread's own column is the output; no LDS passes
      ring[0][0] = pre[0][0];
      ring[1][0] = pre[0][1];
      ring[2][0] = pre[0][2];
      if (zin + 1 < z1) load_plane(zin + 1);
      if (EPI == EPI_COMPOSE_LDS) {
        __syncthreads();   // the previous step's reads of the d ring are done
        store_dplane(zin + 1);
        if (zin + 1 < z1) load_dplane(zin + 2);
        __syncthreads();
      }
      if (EPI == EPI_COMPOSE) finish_compose();
    } else {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (cuse[k]) {
        const int c = tid + k * NT;
        buf[c] = pre[k][0];
        buf[E + c] = pre[k][1];
        buf[2 * E + c] = pre[k][2];
      }
    }
    if (zin + 1 < z1 + R) load_plane(zin + 1);
    __syncthreads();
    if (EPI == EPI_COMPOSE_LDS) {
      // plane zo + 1 joins the ring (slot of zo - 2, last read before the
      // barrier above); the next plane's loads go out now
      store_dplane(zin - R + 1);
      if (zin + 1 < z1 + R) load_dplane(zin - R + 2);
    }
    {
      constexpr int HX = TX / 2, PX = EY * HX;
      for (int p = tid; p < PX; p += NT) {
        const int yy = p / HX, xo = 2 * (p - yy * HX);
        const float* src = buf + yy * EX + xo;
        float* dst = bufx + yy * TX + xo;
#pragma unroll
        for (int q = 0; q < 3; ++q) tap_pair_x<L>(src + q * E, dst + q * XS, w);
      }
    }
    __syncthreads();
    if (EPI == EPI_COMPOSE) finish_compose();
    {
      const float* src = bufx + oy * TX + ox;
      float s0 = w[0] * src[0], s1 = w[0] * src[XS], s2 = w[0] * src[2 * XS];
#pragma unroll
      for (int k = 1; k < L; ++k) {
        s0 += w[k] * src[k * TX];
        s1 += w[k] * src[XS + k * TX];
        s2 += w[k] * src[2 * XS + k * TX];
      }
#pragma unroll
      for (int j = 0; j < L - 1; ++j) {
        ring[0][j] = ring[0][j + 1];
        ring[1][j] = ring[1][j + 1];
        ring[2][j] = ring[2][j + 1];
      }
      ring[0][L - 1] = s0;
      ring[1][L - 1] = s1;
      ring[2][L - 1] = s2;
    }
    }
    const int zo = zin - R;
    if (zo >= z0 && out_col) {
      float v0 = w[0] * ring[0][0], v1 = w[0] * ring[1][0], v2 = w[0] * ring[2][0];
#pragma unroll
      for (int j = 1; j < L; ++j) {
        v0 += w[j] * ring[0][j];
        v1 += w[j] * ring[1][j];
        v2 += w[j] * ring[2][j];
      }
      const int idx = vidx(zo, gy, gx, n1, n2);
      const unsigned off = (unsigned)idx * 4u;
      if (EPI == EPI_STORE) {
        store_at(A.out, off, v0);
        store_at(A.out + N, off, v1);
        store_at(A.out + 2 * N, off, v2);
      } else if (EPI == EPI_MAXNORM) {
        mx = fmaxf(mx, v0 * v0 + v1 * v1 + v2 * v2);
      } else if (EPI == EPI_SMOOTH_MAX) {
        store_at(A.out, off, v0);
        store_at(A.out + N, off, v1);
        store_at(A.out + 2 * N, off, v2);
        mx = fmaxf(mx, v0 * v0 + v1 * v1 + v2 * v2);
      } else if (EPI == EPI_COMPOSE_LDS) {
        // d' = u + d(x + u) from the staged planes zo - 1 .. zo + 1; the
        // cell offset floor(u) is -1 or 0 for |u| <= 1 (u = 1 exactly uses
        // offset 0 with fraction 1, which selects the same corner value)
        const float u0 = scale * v0, u1 = scale * v1, u2 = scale * v2;
        const float f0 = clamp_med3(floorf(u0), -1.0f, 0.0f);
        const float f1 = clamp_med3(floorf(u1), -1.0f, 0.0f);
        const float f2 = clamp_med3(floorf(u2), -1.0f, 0.0f);
        const float t0 = u0 - f0, t1 = u1 - f1, t2 = u2 - f2;
        const int sA = (((zo + (int)f0) % 3) + 3) % 3;
        const int sB = (sA + 1) % 3;
        const int cb = (oy + 1 + (int)f1) * DX + (ox + 1 + (int)f2);
        float res[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float* pa = dring + (sA * 3 + q) * DEP + cb;
          const float* pb = dring + (sB * 3 + q) * DEP + cb;
          const float e00 = pa[0] + t2 * (pa[1] - pa[0]);
          const float e01 = pa[DX] + t2 * (pa[DX + 1] - pa[DX]);
          const float e10 = pb[0] + t2 * (pb[1] - pb[0]);
          const float e11 = pb[DX] + t2 * (pb[DX + 1] - pb[DX]);
          const float g0 = e00 + t1 * (e01 - e00);
          const float g1 = e10 + t1 * (e11 - e10);
          res[q] = g0 + t0 * (g1 - g0);
        }
        store_at(A.out, off, u0 + res[0]);
        store_at(A.out + N, off, u1 + res[1]);
        store_at(A.out + 2 * N, off, u2 + res[2]);
      } else {  // EPI_COMPOSE: d' = u + d(x + u); finished next plane step
        cu[0] = scale * v0;
        cu[1] = scale * v1;
        cu[2] = scale * v2;
        const Cell8 c = cell8_at(n0, n1, n2, zo, gy, gx, cu[0], cu[1], cu[2]);
        gather_issue(A.d, c, cg[0]);
        gather_issue(A.d + N, c, cg[1]);
        gather_issue(A.d + 2 * N, c, cg[2]);
        cidx = idx;
      }
    }
  }
  if (EPI == EPI_COMPOSE) finish_compose();

  if (EPI == EPI_MAXNORM || EPI == EPI_SMOOTH_MAX) {
    const float bm = block_max<NT>(mx, reinterpret_cast<float*>(red));
    if (tid == 0) m_raise(A.ctl, sqrtf(bm), blockIdx.x);
  }
}

// ---------------------------------------------------------------------------
// Brick form of the gradient kernel for small volumes.  A workgroup takes a
// TZ x TY x TX brick: it loads I and J = I_m(x + d) on the brick plus a 2r
// halo into LDS, forms the window sums of I, J, I^2, J^2 and IJ with three
// separable passes (x, y, z), the per-centre coefficients A, B, C on the
// brick plus an r halo, their window sums with three more passes, and the
// output as in k_grad.  No plane-by-plane march: the launch is a short chain
// of dependent steps, which is what bounds small volumes.  The sums run in a
// different order from the streaming form (x, y, z instead of z, x, y), so
// the two agree to rounding, not bitwise.
// ---------------------------------------------------------------------------
template <int W, int TZ, int TY, int TX>
struct GradCubeShape {
  static constexpr int R = W / 2;
  static constexpr int QZ = TZ + 4 * R, QY = TY + 4 * R, QX = TX + 4 * R, NQ = QZ * QY * QX;  // I, J
  static constexpr int CZ = TZ + 2 * R, CY = TY + 2 * R, CX = TX + 2 * R, NC = CZ * CY * CX;  // centres
  static constexpr int NX1 = QZ * QY * CX;   // stage-1 sums after the x pass
  static constexpr int NY1 = QZ * CY * CX;   // ... after the y pass
  static constexpr int NX2 = CZ * CY * TX;   // stage-2 sums after the x pass
  static constexpr int NY2 = CZ * TY * TX;   // ... after the y pass
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int SA = cmax(2 * NQ, cmax(5 * NY1, 3 * NX2));   // I, J -> stage-1 y -> stage-2 x
  static constexpr int SB = cmax(5 * NX1, cmax(3 * NC, 3 * NY2));   // stage-1 x -> A, B, C -> stage-2 y
  static constexpr size_t lds_bytes = sizeof(float) * (size_t)(SA + SB);
};

// MODE as for grad_body: A.mode fixed at compile time, or -1 to read it.
template <int W, int TZ, int TY, int TX, bool QUAD = false, int MODE = -1>
__device__ __forceinline__ void grad_cube_body(const GradArgs& A, const int tile) {
  const int mode = MODE >= 0 ? MODE : A.mode;
  using S = GradCubeShape<W, TZ, TY, TX>;
  constexpr int R = S::R;
  constexpr int NT = TZ * TY * TX;
  constexpr int QY = S::QY, QX = S::QX, NQ = S::NQ;
  constexpr int CY = S::CY, CX = S::CX, NC = S::NC;
  constexpr int NX1 = S::NX1, NY1 = S::NY1, NX2 = S::NX2, NY2 = S::NY2;
  extern __shared__ float lds[];
  float* bufA = lds;
  float* bufB = lds + S::SA;
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  int b = tile;
  const int bx = b % A.tiles_x;
  b /= A.tiles_x;
  const int by = b % A.tiles_y;
  b /= A.tiles_y;
  const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
  const int N = n0 * n1 * n2;
  const int z0 = b * TZ, y0 = by * TY, x0 = bx * TX;
  const float si = A.ctl->shift_i, sj = A.ctl->shift_j;
  if (mode == 0 && tile == 0) m_clear(A.ctl, tid);  // M of this iteration

  // the thread's own output voxel: I, J and grad_p I_m, Adam moments
  const int tz = tid / (TY * TX), tr = tid - tz * (TY * TX);
  const int ty = tr / TX, tx = tr - ty * TX;
  const int oz = z0 + tz, oy = y0 + ty, ox = x0 + tx;
  const bool own = oz < n0 && oy < n1 && ox < n2;
  // byte offset of the own voxel from uniform bases (volumes hold < 2^29 voxels)
  const unsigned ooff = own ? (unsigned)vidx(oz, oy, ox, n1, n2) * 4u : 0u;
  float oI = 0.f, oJ = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  float pm[3] = {0.f, 0.f, 0.f}, pv[3] = {0.f, 0.f, 0.f};
  if (own) {
    Gather gq;
    if constexpr (QUAD) {
      gather_issue_quad(A.moving_quad, n0, n1, n2, oz, oy, ox, load_at(A.d, ooff), load_at(A.d + N, ooff),
                        load_at(A.d + 2 * N, ooff), gq);
    } else {
      const Cell8 c = cell8_pad(n0, n1, n2, oz, oy, ox, load_at(A.d, ooff), load_at(A.d + N, ooff),
                                load_at(A.d + 2 * N, ooff));
      gather_issue(A.moving_pad, c, gq);
    }
    oI = load_at(A.fixed, ooff) - si;
    if (mode == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        pm[q] = load_at(A.m + q * N, ooff);
        pv[q] = load_at(A.v + q * N, ooff);
      }
    }
    oJ = gather_value_grad(gq, g0, g1, g2) - sj;
  }

  // stage-1 inputs on the brick plus 2r (zero off the grid), in batches of
  // KB voxels per thread: the batch's loads of d, then its gathers, are all
  // in flight together instead of one voxel's dependent loads at a time
  constexpr int KQ = (NQ + NT - 1) / NT;   // voxels per thread
  constexpr int KB = 3;                    // batch
#pragma unroll 1
  for (int k0 = 0; k0 < KQ; k0 += KB) {
    bool qok[KB];
    float qd0[KB], qd1[KB], qd2[KB], qf[KB];
    __builtin_amdgcn_s_setprio(2);   // as in the march: the batch's loads leave first
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int c = tid + (k0 + j) * NT;
      const int qz = c / (QY * QX), r = c - qz * (QY * QX);
      const int qy = r / QX, qx = r - qy * QX;
      const int z = z0 - 2 * R + qz, y = y0 - 2 * R + qy, x = x0 - 2 * R + qx;
      qok[j] = k0 + j < KQ && c < NQ && z >= 0 && z < n0 && y >= 0 && y < n1 && x >= 0 && x < n2;
      const unsigned off = qok[j] ? (unsigned)vidx(z, y, x, n1, n2) * 4u : 0u;
      qd0[j] = qok[j] ? load_at(A.d, off) : 0.0f;
      qd1[j] = qok[j] ? load_at(A.d + N, off) : 0.0f;
      qd2[j] = qok[j] ? load_at(A.d + 2 * N, off) : 0.0f;
      qf[j] = qok[j] ? load_at(A.fixed, off) : 0.0f;
    }
    Gather gq[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int c = tid + (k0 + j) * NT;
      const int qz = c / (QY * QX), r = c - qz * (QY * QX);
      const int qy = r / QX, qx = r - qy * QX;
      if constexpr (QUAD) {
        gather_issue_quad(A.moving_quad, n0, n1, n2, z0 - 2 * R + qz, y0 - 2 * R + qy, x0 - 2 * R + qx, qd0[j],
                          qd1[j], qd2[j], gq[j]);
      } else {
        const Cell8 c8 = cell8_pad(n0, n1, n2, z0 - 2 * R + qz, y0 - 2 * R + qy, x0 - 2 * R + qx,
                                   qd0[j], qd1[j], qd2[j]);
        gather_issue(A.moving_pad, c8, gq[j]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int c = tid + (k0 + j) * NT;
      if (k0 + j < KQ && c < NQ) {
        bufA[c] = qok[j] ? qf[j] - si : 0.0f;
        bufA[NQ + c] = qok[j] ? gather_value(gq[j]) - sj : 0.0f;
      }
    }
  }
  __syncthreads();
  // stage 1, x: sums of I, J, I^2, J^2, IJ over w voxels
  for (int c = tid; c < NX1; c += NT) {
    const int row = c / CX, xo = c - row * CX;
    const float* pI = bufA + row * QX + xo;
    const float* pJ = pI + NQ;
    const float i0 = pI[0], j0 = pJ[0];
    float s0 = i0, s1 = j0, s2 = i0 * i0, s3 = j0 * j0, s4 = i0 * j0;
#pragma unroll
    for (int k = 1; k < W; ++k) {
      const float i_ = pI[k], j_ = pJ[k];
      s0 += i_;
      s1 += j_;
      s2 += i_ * i_;
      s3 += j_ * j_;
      s4 += i_ * j_;
    }
    bufB[c] = s0;
    bufB[NX1 + c] = s1;
    bufB[2 * NX1 + c] = s2;
    bufB[3 * NX1 + c] = s3;
    bufB[4 * NX1 + c] = s4;
  }
  __syncthreads();
  // stage 1, y
  for (int c = tid; c < NY1; c += NT) {
    const int zq = c / (CY * CX), r = c - zq * (CY * CX);
    const int yo = r / CX, xo = r - yo * CX;
    const float* src = bufB + (zq * QY + yo) * CX + xo;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const float* p = src + q * NX1;
      float sum = p[0];
#pragma unroll
      for (int k = 1; k < W; ++k) sum += p[k * CX];
      bufA[q * NY1 + c] = sum;
    }
  }
  __syncthreads();
  // stage 1, z, and the per-centre coefficients on the brick plus r
  float lacc = 0.0f;
  for (int c = tid; c < NC; c += NT) {
    const int cz = c / (CY * CX), r = c - cz * (CY * CX);
    const int cy = r / CX, cx = r - cy * CX;
    const float* src = bufA + (cz * CY + cy) * CX + cx;
    float St[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const float* p = src + q * NY1;
      float sum = p[0];
#pragma unroll
      for (int k = 1; k < W; ++k) sum += p[k * CY * CX];
      St[q] = sum;
    }
    const int z = z0 - R + cz, y = y0 - R + cy, x = x0 - R + cx;
    const bool ok = z >= 0 && z < n0 && y >= 0 && y < n1 && x >= 0 && x < n2;
    float ca = 0.f, cb = 0.f, cc_ = 0.f;
    // a one-voxel window has zero variance and covariance: every coefficient is 0
    if (W > 1 && ok) {
      const float cnt = clipped_count(z, n0, R) * (clipped_count(y, n1, R) * clipped_count(x, n2, R));
      const float icnt = __builtin_amdgcn_rcpf(cnt);
      const float muI = St[0] * icnt, muJ = St[1] * icnt;
      const float cross = St[4] - muI * St[1];
      const float vI = St[2] - muI * St[0];
      const float vJ = St[3] - muJ * St[1];
      const float D = vI * vJ + A.eps_cc;
      if (D != 0.0f) {
        const float invD = __builtin_amdgcn_rcpf(D);
        const float cc = cross * cross * invD;
        ca = 2.0f * cross * invD;
        cb = -2.0f * cc * vI * invD;
        cc_ = ca * muI + cb * muJ;
        if (cz >= R && cz < R + TZ && cy >= R && cy < R + TY && cx >= R && cx < R + TX) lacc += cc;
      }
    }
    bufB[c] = ca;
    bufB[NC + c] = cb;
    bufB[2 * NC + c] = cc_;
  }
  __syncthreads();
  // stage 2 (sums of A, B, C over the window around each brick voxel), x
  for (int c = tid; c < NX2; c += NT) {
    const int row = c / TX, xo = c - row * TX;
    const float* src = bufB + row * CX + xo;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float* p = src + q * NC;
      float sum = p[0];
#pragma unroll
      for (int k = 1; k < W; ++k) sum += p[k];
      bufA[q * NX2 + c] = sum;
    }
  }
  __syncthreads();
  // stage 2, y
  for (int c = tid; c < NY2; c += NT) {
    const int zc = c / (TY * TX), r = c - zc * (TY * TX);
    const int yo = r / TX, xo = r - yo * TX;
    const float* src = bufA + (zc * CY + yo) * TX + xo;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float* p = src + q * NX2;
      float sum = p[0];
#pragma unroll
      for (int k = 1; k < W; ++k) sum += p[k * TX];
      bufB[q * NY2 + c] = sum;
    }
  }
  __syncthreads();
  // stage 2, z, and the output
  if (own) {
    const float* src = bufB + (tz * TY + ty) * TX + tx;
    float SA = src[0], SB = src[NY2], SC = src[2 * NY2];
#pragma unroll
    for (int k = 1; k < W; ++k) {
      SA += src[k * TY * TX];
      SB += src[NY2 + k * TY * TX];
      SC += src[2 * NY2 + k * TY * TX];
    }
    const float dl = -A.inv_n * (oI * SA + oJ * SB - SC);
    const float g[3] = {dl * g0, dl * g1, dl * g2};
    if (mode == 0) {
      const float ibc1 = 1.0f / A.ctl->bc1, ibc2 = 1.0f / A.ctl->bc2;
      const float b1 = A.beta1, b2 = A.beta2;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float mm = b1 * pm[q] + (1.0f - b1) * g[q];
        const float vv = b2 * pv[q] + (1.0f - b2) * g[q] * g[q];
        store_at(A.m + q * N, ooff, mm);
        store_at(A.v + q * N, ooff, vv);
        store_at(A.out + q * N, ooff, adam_direction(mm, vv, ibc1, ibc2, A.adam_eps));
      }
    } else if (mode == 1) {
      const float gsc = A.gscale ? *A.gscale : 1.0f;
#pragma unroll
      for (int q = 0; q < 3; ++q) store_at(A.out + q * N, ooff, g[q] * gsc);
    }
  }
  const double tot = block_sum<NT>((double)lacc, red);
  if (tid == 0) A.partials[tile] = tot;
}

// ---------------------------------------------------------------------------
// Brick forms of the smoothing and composition kernels for small volumes.
// A workgroup takes a TZ x TY x TX brick, loads its clamped halo region into
// LDS and runs the three separable passes there (x, then y, then z, the
// order and summation of k_gauss, so the results are bitwise those of the
// streaming form).  With no march along n0, a launch is a few dependent
// steps long instead of one step per plane of a chunk plus its halo.
// ---------------------------------------------------------------------------
template <int R, int TZ, int TY, int TX, int EPI>
__device__ __forceinline__ void gauss_cube_body(const GaussArgs& A, const int tile, const int nblocks) {
  constexpr int L = 2 * R + 1;
  constexpr int NT = TZ * TY * TX;
  constexpr int RZ = TZ + 2 * R, RY = TY + 2 * R, RX = TX + 2 * R;
  constexpr int NR = RZ * RY * RX;   // halo region
  constexpr int NX = RZ * RY * TX;   // after the x-pass
  constexpr int NY = RZ * TY * TX;   // after the y-pass
  static_assert(NY <= NR, "y-pass output reuses the region buffer");
  extern __shared__ float lds[];
  float* reg = lds;            // [3][NR], later [3][NY]
  float* xo = lds + 3 * NR;    // [3][NX]
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  // the first brick of a warp smoothing that records the iteration does so first
  if (EPI == EPI_STORE && A.partials && tile == 0) record_iteration<NT>(A);
  int b = tile;
  const int bx = b % A.tiles_x;
  b /= A.tiles_x;
  const int by = b % A.tiles_y;
  b /= A.tiles_y;
  const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
  const int N = n0 * n1 * n2;
  const int z0 = b * TZ, y0 = by * TY, x0 = bx * TX;

  float w[L];
#pragma unroll
  for (int k = 0; k < L; ++k) w[k] = A.wts[k];

  // the region's loads are all issued before any is consumed
  constexpr int KR = (NR + NT - 1) / NT;
  float rv[KR][3];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int c = min(tid + k * NT, NR - 1);
    const int zz = c / (RY * RX), r = c - zz * (RY * RX);
    const int yy = r / RX, xx = r - yy * RX;
    const int gz = min(max(z0 - R + zz, 0), n0 - 1);
    const int gy = min(max(y0 - R + yy, 0), n1 - 1);
    const int gx = min(max(x0 - R + xx, 0), n2 - 1);
    const unsigned off = (unsigned)((gz * n1 + gy) * n2 + gx) * 4u;
    rv[k][0] = load_at(A.in, off);
    rv[k][1] = load_at(A.in + N, off);
    rv[k][2] = load_at(A.in + 2 * N, off);
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int c = tid + k * NT;
    if (c < NR) {
      reg[c] = rv[k][0];
      reg[NR + c] = rv[k][1];
      reg[2 * NR + c] = rv[k][2];
    }
  }
  __syncthreads();
  for (int c = tid; c < NX; c += NT) {
    const int row = c / TX, xx = c - row * TX;
    const float* src = reg + row * RX + xx;
    float s0 = w[0] * src[0], s1 = w[0] * src[NR], s2 = w[0] * src[2 * NR];
#pragma unroll
    for (int k = 1; k < L; ++k) {
      s0 += w[k] * src[k];
      s1 += w[k] * src[NR + k];
      s2 += w[k] * src[2 * NR + k];
    }
    xo[c] = s0;
    xo[NX + c] = s1;
    xo[2 * NX + c] = s2;
  }
  __syncthreads();
  for (int c = tid; c < NY; c += NT) {
    const int zz = c / (TY * TX), r = c - zz * (TY * TX);
    const int yy = r / TX, xx = r - yy * TX;
    const float* src = xo + (zz * RY + yy) * TX + xx;
    float s0 = w[0] * src[0], s1 = w[0] * src[NX], s2 = w[0] * src[2 * NX];
#pragma unroll
    for (int k = 1; k < L; ++k) {
      s0 += w[k] * src[k * TX];
      s1 += w[k] * src[NX + k * TX];
      s2 += w[k] * src[2 * NX + k * TX];
    }
    reg[c] = s0;
    reg[NY + c] = s1;
    reg[2 * NY + c] = s2;
  }
  __syncthreads();
  const int tz = tid / (TY * TX), r = tid - tz * (TY * TX);
  const int ty = r / TX, tx = r - ty * TX;
  const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
  float mx = 0.0f;
  if (gz < n0 && gy < n1 && gx < n2) {
    const float* src = reg + (tz * TY + ty) * TX + tx;
    float v0 = w[0] * src[0], v1 = w[0] * src[NY], v2 = w[0] * src[2 * NY];
#pragma unroll
    for (int j = 1; j < L; ++j) {
      v0 += w[j] * src[j * TY * TX];
      v1 += w[j] * src[NY + j * TY * TX];
      v2 += w[j] * src[2 * NY + j * TY * TX];
    }
    const unsigned off = (unsigned)vidx(gz, gy, gx, n1, n2) * 4u;
    store_at(A.out, off, v0);
    store_at(A.out + N, off, v1);
    store_at(A.out + 2 * N, off, v2);
    if (EPI == EPI_SMOOTH_MAX) mx = v0 * v0 + v1 * v1 + v2 * v2;
  }
  if (EPI == EPI_SMOOTH_MAX) {
    const float bm = block_max<NT>(mx, reinterpret_cast<float*>(red));
    if (tid == 0) m_raise(A.ctl, sqrtf(bm), blockIdx.x);
  }
}

// d' = u + d(x + u), u = -eta s / (2M), |u| <= 1 voxel, on a brick: d is
// staged in LDS on the brick plus one voxel (zero off the grid).  Runs in
// place over s: each thread reads s only at the voxel it writes.
template <int TZ, int TY, int TX>
__device__ __forceinline__ void compose_cube_body(const GaussArgs& A, const int tile) {
  constexpr int NT = TZ * TY * TX;
  constexpr int DZ = TZ + 2, DY = TY + 2, DX = TX + 2, DE = DZ * DY * DX;
  extern __shared__ float lds[];   // [3][DE]
  const int tid = threadIdx.x;
  // the first brick records the iteration before its own work
  if (A.partials && tile == 0) record_iteration<NT>(A);
  int b = tile;
  const int bx = b % A.tiles_x;
  b /= A.tiles_x;
  const int by = b % A.tiles_y;
  b /= A.tiles_y;
  const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
  const int N = n0 * n1 * n2;
  const int z0 = b * TZ, y0 = by * TY, x0 = bx * TX;
  constexpr int KD = (DE + NT - 1) / NT;
  float dv[KD][3];
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const int c = tid + k * NT;
    const int zz = c / (DY * DX), r = c - zz * (DY * DX);
    const int yy = r / DX, xx = r - yy * DX;
    const int gz = z0 - 1 + zz, gy = y0 - 1 + yy, gx = x0 - 1 + xx;
    const bool ok = c < DE && gz >= 0 && gz < n0 && gy >= 0 && gy < n1 && gx >= 0 && gx < n2;
    const unsigned off = ok ? (unsigned)((gz * n1 + gy) * n2 + gx) * 4u : 0u;
    dv[k][0] = ok ? load_at(A.d, off) : 0.0f;
    dv[k][1] = ok ? load_at(A.d + N, off) : 0.0f;
    dv[k][2] = ok ? load_at(A.d + 2 * N, off) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const int c = tid + k * NT;
    if (c < DE) {
      lds[c] = dv[k][0];
      lds[DE + c] = dv[k][1];
      lds[2 * DE + c] = dv[k][2];
    }
  }
  const float M = m_value(A.ctl);
  const float scale = M > 0.0f ? -A.eta / (2.0f * M) : 0.0f;
  const int tz = tid / (TY * TX), r = tid - tz * (TY * TX);
  const int ty = r / TX, tx = r - ty * TX;
  const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
  const bool own = gz < n0 && gy < n1 && gx < n2;
  const unsigned off = own ? (unsigned)vidx(gz, gy, gx, n1, n2) * 4u : 0u;
  float sv[3] = {0.f, 0.f, 0.f};
  if (own) {
    sv[0] = load_at(A.in, off);
    sv[1] = load_at(A.in + N, off);
    sv[2] = load_at(A.in + 2 * N, off);
  }
  __syncthreads();
  if (own) {
    // the arithmetic of k_gauss<0, EPI_COMPOSE_LDS>: floor(u) is -1 or 0
    const float u0 = scale * sv[0], u1 = scale * sv[1], u2 = scale * sv[2];
    const float f0 = clamp_med3(floorf(u0), -1.0f, 0.0f);
    const float f1 = clamp_med3(floorf(u1), -1.0f, 0.0f);
    const float f2 = clamp_med3(floorf(u2), -1.0f, 0.0f);
    const float t0 = u0 - f0, t1 = u1 - f1, t2 = u2 - f2;
    const int cb = ((tz + 1 + (int)f0) * DY + (ty + 1 + (int)f1)) * DX + (tx + 1 + (int)f2);
    float res[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float* pa = lds + q * DE + cb;
      const float* pb = pa + DY * DX;
      const float e00 = pa[0] + t2 * (pa[1] - pa[0]);
      const float e01 = pa[DX] + t2 * (pa[DX + 1] - pa[DX]);
      const float e10 = pb[0] + t2 * (pb[1] - pb[0]);
      const float e11 = pb[DX] + t2 * (pb[DX + 1] - pb[DX]);
      const float g0 = e00 + t1 * (e01 - e00);
      const float g1 = e10 + t1 * (e11 - e10);
      res[q] = g0 + t0 * (g1 - g0);
    }
    store_at(A.out, off, u0 + res[0]);
    store_at(A.out + N, off, u1 + res[1]);
    store_at(A.out + 2 * N, off, u2 + res[2]);
  }
}

// ---------------------------------------------------------------------------
// Kernels of the iteration, in two forms.  The plain form runs one
// registration, with its arguments in the kernel arguments.  The batch form
// runs several registrations in one launch: entry e of a table in device
// memory holds the arguments of one registration and its range of
// workgroups in the launch, and owner[g] names the entry of workgroup g
// (after the XCD renumbering, so each XCD takes a contiguous range of the
// batch's tiles).  A workgroup loads its entry's arguments once, with scalar
// loads, and then runs the same body as the plain form.
// ---------------------------------------------------------------------------
// A pointer loaded from memory is generic to the compiler, and accesses
// through it become flat instructions (which also count against the LDS
// wait counter, so every LDS wait would wait for them too).  Each pointer is
// rebuilt from its integer value as a global-address-space pointer, which
// tells the compiler what it knows for kernel arguments: the body then uses
// global instructions.  (A plain cast to the global space and back is folded
// away before the address spaces are inferred.)
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
  typedef __attribute__((address_space(1))) T GT;
  return (T*)(GT*)(uintptr_t)p;
}

__device__ __forceinline__ void load_args(const GradArgs* __restrict__ s, GradArgs& A) {
  A.fixed = as_global(s->fixed);
  A.moving_pad = as_global(s->moving_pad);
  A.moving_quad = as_global(s->moving_quad);
  A.d = as_global(s->d);
  A.m = as_global(s->m);
  A.v = as_global(s->v);
  A.out = as_global(s->out);
  A.gscale = as_global(s->gscale);
  A.partials = as_global(s->partials);
  A.ctl = as_global(s->ctl);
  A.n0 = s->n0;
  A.n1 = s->n1;
  A.n2 = s->n2;
  A.zc = s->zc;
  A.tiles_y = s->tiles_y;
  A.tiles_x = s->tiles_x;
  A.eps_cc = s->eps_cc;
  A.beta1 = s->beta1;
  A.beta2 = s->beta2;
  A.adam_eps = s->adam_eps;
  A.inv_n = s->inv_n;
  A.mode = s->mode;
}

__device__ __forceinline__ void load_args(const GaussArgs* __restrict__ s, GaussArgs& A) {
  A.in = as_global(s->in);
  A.out = as_global(s->out);
  A.d = as_global(s->d);
  A.wts = as_global(s->wts);
  A.ctl = as_global(s->ctl);
  A.partials = as_global(s->partials);
  A.loss_hist = as_global(s->loss_hist);
  A.loss_cap = s->loss_cap;
  A.n_partials = s->n_partials;
  A.inv_n = s->inv_n;
  A.eta = s->eta;
  A.n0 = s->n0;
  A.n1 = s->n1;
  A.n2 = s->n2;
  A.zc = s->zc;
  A.tiles_y = s->tiles_y;
  A.tiles_x = s->tiles_x;
}

template <class Args>
__device__ __forceinline__ int batch_entry(const BatchEntry<Args>* __restrict__ E, const int* __restrict__ owner,
                                           Args& A, int& nblocks) {
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const int e = owner[g];
  load_args(&E[e].a, A);
  nblocks = E[e].nblocks;
  return g - E[e].first;
}

template <int W, int TY, int TX, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TY * TX) k_grad_batch(const BatchEntry<GradArgs>* __restrict__ E,
                                                        const int* __restrict__ owner) {
  GradArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  grad_body<W, TY, TX, true, QUAD, MODE>(A, tile);
}

template <int W, int TY, int TX, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TY * TX) __attribute__((amdgpu_waves_per_eu(4)))
k_grad_o4_batch(const BatchEntry<GradArgs>* __restrict__ E, const int* __restrict__ owner) {
  GradArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  grad_body<W, TY, TX, true, QUAD, MODE>(A, tile);
}

template <int R, int TY, int TX, int EPI>
__global__ void __launch_bounds__(TY * TX) k_gauss(const GaussArgs A) {
  gauss_body<R, TY, TX, EPI>(A, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

template <int R, int TY, int TX, int EPI>
__global__ void __launch_bounds__(TY * TX) k_gauss_batch(const BatchEntry<GaussArgs>* __restrict__ E,
                                                         const int* __restrict__ owner) {
  GaussArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  gauss_body<R, TY, TX, EPI>(A, tile, nb);
}

template <int W, int TZ, int TY, int TX, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TZ * TY * TX) k_grad_cube(const GradArgs A) {
  grad_cube_body<W, TZ, TY, TX, QUAD, MODE>(A, xcd_tile(blockIdx.x, gridDim.x));
}

template <int W, int TZ, int TY, int TX, bool QUAD = false, int MODE = -1>
__global__ void __launch_bounds__(TZ * TY * TX) k_grad_cube_batch(const BatchEntry<GradArgs>* __restrict__ E,
                                                                  const int* __restrict__ owner) {
  GradArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  grad_cube_body<W, TZ, TY, TX, QUAD, MODE>(A, tile);
}

template <int R, int TZ, int TY, int TX, int EPI>
__global__ void __launch_bounds__(TZ * TY * TX) k_gauss_cube(const GaussArgs A) {
  gauss_cube_body<R, TZ, TY, TX, EPI>(A, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

template <int R, int TZ, int TY, int TX, int EPI>
__global__ void __launch_bounds__(TZ * TY * TX) k_gauss_cube_batch(const BatchEntry<GaussArgs>* __restrict__ E,
                                                                   const int* __restrict__ owner) {
  GaussArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  gauss_cube_body<R, TZ, TY, TX, EPI>(A, tile, nb);
}

template <int TZ, int TY, int TX>
__global__ void __launch_bounds__(TZ * TY * TX) k_compose_cube(const GaussArgs A) {
  compose_cube_body<TZ, TY, TX>(A, xcd_tile(blockIdx.x, gridDim.x));
}

template <int TZ, int TY, int TX>
__global__ void __launch_bounds__(TZ * TY * TX) k_compose_cube_batch(const BatchEntry<GaussArgs>* __restrict__ E,
                                                                     const int* __restrict__ owner) {
  GaussArgs A;
  int nb;
  const int tile = batch_entry(E, owner, A, nb);
  compose_cube_body<TZ, TY, TX>(A, tile);
}

// ---------------------------------------------------------------------------
// Off-loop kernels: pyramid blur and resampling, warp, fills, layout copies.
// ---------------------------------------------------------------------------
// Algorithm 1 with use_jac: the descent direction is J(phi)^T dU/dphi
// (Section 4.4.2, Eulerian descent), J(phi) = I + grad d; component a is
// g_a + sum_c (d d_c / d x_a) g_c, with grad d by central differences inside
// the grid and one-sided differences on its faces.  Adam follows, as in the
// gradient kernel's own epilogue.  In place: each thread reads g only at the
// voxel whose direction it writes.
__global__ void __launch_bounds__(256)
k_eulerian_adam(float* __restrict__ ga, const float* __restrict__ d, float* __restrict__ m,
                float* __restrict__ v, Ctl* ctl, int n0, int n1, int n2, float beta1, float beta2,
                float adam_eps) {
  const int N = n0 * n1 * n2;
  if (blockIdx.x == 0) m_clear(ctl, threadIdx.x);   // M of this iteration
  const float ibc1 = 1.0f / ctl->bc1, ibc2 = 1.0f / ctl->bc2;
  const int plane = n1 * n2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const int x2 = i % n2, t = i / n2;
    const int x1 = t % n1, x0 = t / n1;
    const int xs[3] = {x0, x1, x2}, ns[3] = {n0, n1, n2}, st[3] = {plane, n2, 1};
    float g[3], out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = ga[c * N + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const bool has_lo = xs[a] > 0, has_hi = xs[a] < ns[a] - 1;
      const int lo = has_lo ? i - st[a] : i, hi = has_hi ? i + st[a] : i;
      const float h = (has_lo && has_hi) ? 0.5f : 1.0f;
      float r = g[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) r += (d[c * N + hi] - d[c * N + lo]) * h * g[c];
      out[a] = r;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int iq = q * N + i;
      const float mm = beta1 * m[iq] + (1.0f - beta1) * out[q];
      const float vv = beta2 * v[iq] + (1.0f - beta2) * out[q] * out[q];
      m[iq] = mm;
      v[iq] = vv;
      ga[iq] = adam_direction(mm, vv, ibc1, ibc2, adam_eps);
    }
  }
}

// Copy of a volume with a zero border of kPad voxels on every side.
__global__ void k_pad(const float* __restrict__ in, float* __restrict__ out, int n0, int n1, int n2) {
  const int p0 = n0 + 2 * kPad, p1 = n1 + 2 * kPad, p2 = n2 + 2 * kPad;
  const int64_t total = (int64_t)p0 * p1 * p2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % p2) - kPad;
    const int64_t t = i / p2;
    const int y = (int)(t % p1) - kPad;
    const int z = (int)(t / p1) - kPad;
    const bool in_grid = z >= 0 && z < n0 && y >= 0 && y < n1 && x >= 0 && x < n2;
    out[i] = in_grid ? in[((int64_t)z * n1 + y) * n2 + x] : 0.0f;
  }
}

// Corner quads of the padded image (gather_issue_quad): quad[i] = (pad[i],
// pad[i+1], pad[i+p2], pad[i+p2+1]) over the padded grid, zero where a corner
// leaves it (the last padded row and column, never the low corner of a cell).
__global__ void k_pad_quad(const float* __restrict__ pad, float4* __restrict__ quad, int p0, int p1, int p2) {
  const int64_t n = (int64_t)p0 * p1 * p2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % p2);
  const int y = (int)((i / p2) % p1);
  const bool xo = x + 1 < p2, yo = y + 1 < p1;
  float4 q;
  q.x = pad[i];
  q.y = xo ? pad[i + 1] : 0.0f;
  q.z = yo ? pad[i + p2] : 0.0f;
  q.w = (xo && yo) ? pad[i + p2 + 1] : 0.0f;
  quad[i] = q;
}

__global__ void k_fill(float* __restrict__ p, float value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// ---- Gaussian smoothing of a field with a radius above kMaxRadius ----------
// One separable pass of a 3-component field [3][n0][n1][n2] along one axis:
// out_c(x) = sum_{k=-R..R} w[k+R] in_c(x + k e_axis), the index clamped to the
// grid (replicate), the taps summed in that order.  The radius is a run-time
// value up to kMaxWideRadius.  A workgroup stages its line segment (outputs
// plus R on each side) in LDS once and every output reads its 2R+1 taps from
// there.
//
// Along n2: a workgroup of 256 threads takes 256 consecutive voxels of one
// row (grid: ceil(n2/256), n1, n0).
__global__ void __launch_bounds__(256) k_field_wide_x(const float* __restrict__ in, float* __restrict__ out,
                                                      int n0, int n1, int n2, const float* __restrict__ w, int R) {
  extern __shared__ float wl[];   // [3][256 + 2R]
  const int L = 256 + 2 * R;
  const int x0 = blockIdx.x * 256, y = blockIdx.y, z = blockIdx.z;
  const int64_t N = (int64_t)n0 * n1 * n2;
  const int64_t row = ((int64_t)z * n1 + y) * n2;
  for (int c = 0; c < 3; ++c)
    for (int i = threadIdx.x; i < L; i += 256) {
      const int xx = min(max(x0 - R + i, 0), n2 - 1);
      wl[c * L + i] = in[c * N + row + xx];
    }
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= n2) return;
  for (int c = 0; c < 3; ++c) {
    const float* src = wl + c * L + threadIdx.x;
    float acc = w[0] * src[0];
    for (int k = 1; k <= 2 * R; ++k) acc += w[k] * src[k];
    out[c * N + row + x] = acc;
  }
}

// Along n1 (axis 1) or n0 (axis 0): a workgroup of 64 x 8 threads takes 64
// consecutive n2 columns and kWideRun consecutive positions along the axis
// (grid: ceil(n2/64), ceil(n_axis/kWideRun), the remaining axis); thread
// (lane, j) forms the 8 consecutive outputs 8j .. 8j+7 of its column from a
// sliding window of 8 registers: taps go in blocks of 8 (the tap tables are
// zero-padded to a multiple of 16, so the block past 2R + 1 adds exact
// zeros), and each staged input is read from LDS once per thread instead of
// once per tap.  One component is staged at a time.  The last pass (axis 0)
// also runs the smoothing's epilogue (EPI): the max norm M of the result
// (EPI_SMOOTH_MAX), as the streaming kernels do; E carries the control block.
// (64 positions: at radius 18 a run of 32 re-read 36 halo positions for
// every 32 outputs)
constexpr int kWideRun = 64, kWideThreads = 8 * kWideRun;
template <int AX, int EPI>
__global__ void __launch_bounds__(kWideThreads) k_field_wide_yz(const float* __restrict__ in, float* __restrict__ out,
                                                       int n0, int n1, int n2, const float* __restrict__ w, int R,
                                                       const GaussArgs E) {
  extern __shared__ float wl[];   // [kWideRun + L8][64], one component at a time
  __shared__ double red[kWideThreads / 64];
  const int L8 = (2 * R + 1 + 7) / 8 * 8;
  const int LS = kWideRun + L8;
  const int lane = threadIdx.x & 63, j0 = threadIdx.x >> 6;
  const int x = blockIdx.x * 64 + lane;
  const int a0 = blockIdx.y * kWideRun;
  const int na = AX == 0 ? n0 : n1;
  const int other = blockIdx.z;   // y for AX == 0, z for AX == 1
  const int64_t N = (int64_t)n0 * n1 * n2;
  const int64_t astride = AX == 0 ? (int64_t)n1 * n2 : (int64_t)n2;
  const int64_t base = AX == 0 ? (int64_t)other * n2 : (int64_t)other * n1 * n2;
  const bool xin = x < n2;
  const int bo = 8 * j0;          // this thread's outputs, relative to a0
  float v[3][8];
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();   // the previous component's reads are done
    for (int i = j0; i < LS; i += kWideThreads / 64) {
      const int aa = min(max(a0 - R + i, 0), na - 1);
      wl[i * 64 + lane] = xin ? in[c * N + base + aa * astride + x] : 0.0f;
    }
    __syncthreads();
    float acc[8], xr[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      acc[o] = 0.0f;
      xr[o] = wl[(bo + o) * 64 + lane];
    }
    for (int k = 0; k < L8; k += 8) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const float wk = w[k + m];
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[o] += wk * xr[(m + o) & 7];
        xr[m] = wl[(bo + k + m + 8) * 64 + lane];
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      v[c][o] = acc[o];
      if (xin && a0 + bo + o < na) out[c * N + base + (int64_t)(a0 + bo + o) * astride + x] = acc[o];
    }
  }
  float mx = 0.0f;
  if (EPI == EPI_SMOOTH_MAX && xin) {
#pragma unroll
    for (int o = 0; o < 8; ++o)
      if (a0 + bo + o < na) mx = fmaxf(mx, v[0][o] * v[0][o] + v[1][o] * v[1][o] + v[2][o] * v[2][o]);
  }
  if (EPI == EPI_SMOOTH_MAX) {
    const float bm = block_max<kWideThreads>(mx, reinterpret_cast<float*>(red));
    if (threadIdx.x == 0) m_raise(E.ctl, sqrtf(bm), blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
  }
}

__global__ void k_blur_axis(const float* __restrict__ in, float* __restrict__ out, int n0, int n1,
                            int n2, int axis, const float* __restrict__ w, int R) {
  const int N = n0 * n1 * n2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = i % n2, y = (i / n2) % n1, z = i / (n1 * n2);
  const int pos = axis == 0 ? z : (axis == 1 ? y : x);
  const int n = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
  const int stride = axis == 0 ? n1 * n2 : (axis == 1 ? n2 : 1);
  float s = 0.0f;
  for (int k = -R; k <= R; ++k) {
    const int q = min(max(pos + k, 0), n - 1);
    s += w[k + R] * in[i + (q - pos) * stride];
  }
  out[i] = s;
}

// The same blur along n0 or n1 with T consecutive outputs per thread: the
// T + 2R inputs of a run are loaded once into registers instead of 2R + 1
// times per output through the caches.  Consecutive threads take consecutive
// lines (x fastest), so every load is coalesced.  Each output sums the same
// taps in the same order as k_blur_axis, so the results are bitwise equal.
template <int R, int T>
__global__ void __launch_bounds__(256) k_blur_axis_run(const float* __restrict__ in, float* __restrict__ out,
                                                       int n0, int n1, int n2, int axis,
                                                       const float* __restrict__ w) {
  const int n = axis == 0 ? n0 : n1;
  const int stride = axis == 0 ? n1 * n2 : n2;
  const int lines = axis == 0 ? n1 * n2 : n0 * n2;
  const int runs = (n + T - 1) / T;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= lines * runs) return;
  const int l = t % lines, r = t / lines;
  const int base = axis == 0 ? l : (l / n2) * (n1 * n2) + l % n2;
  const int p0 = r * T;
  float wt[2 * R + 1];
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) wt[k] = w[k];
  float v[T + 2 * R];
#pragma unroll
  for (int j = 0; j < T + 2 * R; ++j) v[j] = in[base + min(max(p0 - R + j, 0), n - 1) * stride];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (p0 + j < n) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * R; ++k) s += wt[k] * v[j + k];
      out[base + (p0 + j) * stride] = s;
    }
  }
}

// The same blur along n2 on a (n2 / 256, n1, n0) grid: the voxel comes from
// the block indices, with none of the runtime integer divisions of the flat
// form, and each lane's 2R + 1 taps are neighbouring floats.  Same taps and
// order as k_blur_axis (bitwise equal).
template <int R>
__global__ void __launch_bounds__(256) k_blur_x(const float* __restrict__ in, float* __restrict__ out, int n2,
                                                const float* __restrict__ w) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= n2) return;
  const size_t row = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * (size_t)n2;
  float s = 0.0f;
#pragma unroll
  for (int k = -R; k <= R; ++k) s += w[k + R] * in[row + min(max(x + k, 0), n2 - 1)];
  out[row + x] = s;
}

// Voxel (z, y, x) and flat index i of this thread in an n0 x n1 x n2 launch:
// on a (n2 / blockDim, n1, n0) grid (G3) from the block indices, with no
// integer divisions; else from a flat index.  False past the end of a row or
// of the volume.
template <bool G3>
__device__ __forceinline__ bool grid_voxel(int n0, int n1, int n2, int& z, int& y, int& x, int& i) {
  if constexpr (G3) {
    x = blockIdx.x * blockDim.x + threadIdx.x;
    y = blockIdx.y;
    z = blockIdx.z;
    i = (z * n1 + y) * n2 + x;
    return x < n2;
  } else {
    i = blockIdx.x * blockDim.x + threadIdx.x;
    x = i % n2;
    y = (i / n2) % n1;
    z = i / (n1 * n2);
    return i < n0 * n1 * n2;
  }
}

__device__ __forceinline__ float aligned_pos(int i, int nin, int nout) {
  return nout > 1 ? (float)(i * (nin - 1)) / (float)(nout - 1) : 0.0f;
}

template <bool G3>
__global__ void k_resample(const float* __restrict__ in, float* __restrict__ out, int ni0, int ni1,
                           int ni2, int no0, int no1, int no2, int nch, float rho0, float rho1,
                           float rho2) {
  const int No = no0 * no1 * no2;
  const int Ni = ni0 * ni1 * ni2;
  int z, y, x, i;
  if (!grid_voxel<G3>(no0, no1, no2, z, y, x, i)) return;
  const Corners c = make_corners(ni0, ni1, ni2, aligned_pos(z, ni0, no0), aligned_pos(y, ni1, no1),
                                 aligned_pos(x, ni2, no2));
  out[i] = rho0 * tri(in, c);
  if (nch > 1) {
    out[No + i] = rho1 * tri(in + Ni, c);
    out[2 * No + i] = rho2 * tri(in + 2 * Ni, c);
  }
}

template <bool G3>
__global__ void k_warp(const float* __restrict__ img, const float* __restrict__ d,
                       float* __restrict__ out, int n0, int n1, int n2) {
  const int N = n0 * n1 * n2;
  int z, y, x, i;
  if (!grid_voxel<G3>(n0, n1, n2, z, y, x, i)) return;
  const Cell8 c = cell8_at(n0, n1, n2, z, y, x, d[i], d[N + i], d[2 * N + i]);
  Gather g;
  gather_issue(img, c, g);
  out[i] = gather_value(g);
}

// out = u + d(x + u): the displacement of phi o (id + u) for phi = id + d,
// with d sampled trilinearly per component (zero outside the grid).
__global__ void k_compose_fields(const float* __restrict__ u, const float* __restrict__ d,
                                 float* __restrict__ out, int n0, int n1, int n2) {
  const int N = n0 * n1 * n2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = i % n2, y = (i / n2) % n1, z = i / (n1 * n2);
  const float u0 = u[i], u1 = u[N + i], u2 = u[2 * N + i];
  const Cell8 c = cell8_at(n0, n1, n2, z, y, x, u0, u1, u2);
  Gather g0, g1, g2;
  gather_issue(d, c, g0);
  gather_issue(d + N, c, g1);
  gather_issue(d + 2 * N, c, g2);
  out[i] = u0 + gather_value(g0);
  out[N + i] = u1 + gather_value(g1);
  out[2 * N + i] = u2 + gather_value(g2);
}

__global__ void k_soa_to_aos(const float* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[3 * i] = in[i];
  out[3 * i + 1] = in[n + i];
  out[3 * i + 2] = in[2 * n + i];
}

__global__ void k_ctl_init(Ctl* ctl, float beta1, float beta2, int t_done, int iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int t = t_done + 1;
    ctl->t = t;
    if (iter >= 0) ctl->iter = iter;
    ctl->beta1 = beta1;
    ctl->beta2 = beta2;
    ctl->bp1 = pow((double)beta1, (double)t);
    ctl->bp2 = pow((double)beta2, (double)t);
    ctl->bc1 = (float)(1.0 - ctl->bp1);
    ctl->bc2 = (float)(1.0 - ctl->bp2);
    for (int j = 0; j < kMSlots; ++j) ctl->mslot[j * kMStride] = 0u;
  }
}

__global__ void k_sum_partial(const float* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_mean_final(const double* __restrict__ part, int np, double n, float* __restrict__ dst) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *dst = (float)(s / n);
}

__global__ void k_sum_final(const double* __restrict__ part, int np, double* __restrict__ dst) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *dst = s;
}

// ---------------------------------------------------------------------------
// Dispatch tables
// ---------------------------------------------------------------------------
template <int W, int TY, int TX>
constexpr size_t grad_lds() {
  constexpr int R = W / 2;
  constexpr int GS = (R == 0) ? 1 : 2 * R;
  constexpr size_t base = sizeof(float) * (5 * (TY + 4 * R) * (TX + 4 * R) + 5 * (TY + 4 * R) * (TX + 2 * R));
  constexpr size_t ring = sizeof(float) * 3 * GS * TY * TX;
  return base + ring <= 65536 ? base + ring : base;
}

template <int R, int TY, int TX>
constexpr size_t gauss_lds(bool staged_d) {
  return sizeof(float) * (3 * (TY + 2 * R) * (TX + 2 * R) + 3 * (TY + 2 * R) * TX +
                          (staged_d ? 9 * (((TY + 2) * (TX + 2) + 31) / 32 * 32) : 0));
}

template <int W, int TY, int TX>
hipError_t grad_launch_t(const GradArgs& a, const Tiling& t, hipStream_t s) {
  constexpr size_t sh = grad_lds<W, TY, TX>();
  static_assert(sh <= 65536, "gradient kernel LDS exceeds 64 KiB");
  // two workgroups per CU where 128 VGPRs hold the kernel without spills
  constexpr bool occ2 = (W <= 5) && TY == 16 && TX == 32;
  const dim3 g(t.blocks()), blk(TY * TX);
  if constexpr (occ2) {
    if (t.variant == 2) k_grad_o4<W, TY, TX, false><<<g, blk, sh, s>>>(a);
    else if (a.moving_quad && a.mode == 0) k_grad_o4<W, TY, TX, true, true, 0><<<g, blk, sh, s>>>(a);
    else if (a.moving_quad) k_grad_o4<W, TY, TX, true, true><<<g, blk, sh, s>>>(a);
    else k_grad_o4<W, TY, TX, true><<<g, blk, sh, s>>>(a);
  } else {
    if (t.variant == 2) k_grad<W, TY, TX, false><<<g, blk, sh, s>>>(a);
    else if (a.moving_quad && a.mode == 0) k_grad<W, TY, TX, true, true, 0><<<g, blk, sh, s>>>(a);
    else if (a.moving_quad) k_grad<W, TY, TX, true, true><<<g, blk, sh, s>>>(a);
    else k_grad<W, TY, TX, true><<<g, blk, sh, s>>>(a);
  }
  return hipGetLastError();
}

template <int TY, int TX>
hipError_t grad_launch_tile(const GradArgs& a, int window, const Tiling& t, hipStream_t s) {
  switch (window) {
    case 1: return grad_launch_t<1, TY, TX>(a, t, s);
    case 3: return grad_launch_t<3, TY, TX>(a, t, s);
    case 5: return grad_launch_t<5, TY, TX>(a, t, s);
    case 7: return grad_launch_t<7, TY, TX>(a, t, s);
    case 9: return grad_launch_t<9, TY, TX>(a, t, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R, int TY, int TX>
hipError_t gauss_launch_r(const GaussArgs& a, int epi, const Tiling& t, hipStream_t s) {
  const dim3 g(t.blocks()), blk(TY * TX);
  const size_t sh = gauss_lds<R, TY, TX>(epi == EPI_COMPOSE_LDS);
  switch (epi) {
    case EPI_STORE: k_gauss<R, TY, TX, EPI_STORE><<<g, blk, sh, s>>>(a); break;
    case EPI_MAXNORM: k_gauss<R, TY, TX, EPI_MAXNORM><<<g, blk, sh, s>>>(a); break;
    case EPI_COMPOSE: k_gauss<R, TY, TX, EPI_COMPOSE><<<g, blk, sh, s>>>(a); break;
    case EPI_COMPOSE_LDS: k_gauss<R, TY, TX, EPI_COMPOSE_LDS><<<g, blk, sh, s>>>(a); break;
    case EPI_SMOOTH_MAX: k_gauss<R, TY, TX, EPI_SMOOTH_MAX><<<g, blk, sh, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TY, int TX>
hipError_t gauss_launch_tile(const GaussArgs& a, int radius, int epi, const Tiling& t, hipStream_t s) {
  switch (radius) {
    case 0: return gauss_launch_r<0, TY, TX>(a, epi, t, s);
    case 1: return gauss_launch_r<1, TY, TX>(a, epi, t, s);
    case 2: return gauss_launch_r<2, TY, TX>(a, epi, t, s);
    case 3: return gauss_launch_r<3, TY, TX>(a, epi, t, s);
    case 4: return gauss_launch_r<4, TY, TX>(a, epi, t, s);
    case 5: return gauss_launch_r<5, TY, TX>(a, epi, t, s);
    case 6: return gauss_launch_r<6, TY, TX>(a, epi, t, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
hipError_t gauss_cube_r(const GaussArgs& a, int epi, const Tiling& t, hipStream_t s) {
  constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
  constexpr size_t sh = sizeof(float) * 3 *
                        ((TZ + 2 * R) * (TY + 2 * R) * (TX + 2 * R) + (TZ + 2 * R) * (TY + 2 * R) * TX);
  static_assert(sh <= 65536, "brick smoothing LDS exceeds 64 KiB");
  const dim3 g(t.blocks()), blk(TZ * TY * TX);
  switch (epi) {
    case EPI_SMOOTH_MAX: k_gauss_cube<R, TZ, TY, TX, EPI_SMOOTH_MAX><<<g, blk, sh, s>>>(a); break;
    case EPI_STORE: k_gauss_cube<R, TZ, TY, TX, EPI_STORE><<<g, blk, sh, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t gauss_launch_cube(const GaussArgs& a, int radius, int epi, const Tiling& t, hipStream_t s) {
  if (epi == EPI_COMPOSE_LDS) {
    if (radius != 0) return hipErrorInvalidValue;
    constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
    constexpr size_t sh = sizeof(float) * 3 * (TZ + 2) * (TY + 2) * (TX + 2);
    k_compose_cube<TZ, TY, TX><<<dim3(t.blocks()), dim3(TZ * TY * TX), sh, s>>>(a);
    return hipGetLastError();
  }
  switch (radius) {
    case 0: return gauss_cube_r<0>(a, epi, t, s);
    case 1: return gauss_cube_r<1>(a, epi, t, s);
    case 2: return gauss_cube_r<2>(a, epi, t, s);
    case 3: return gauss_cube_r<3>(a, epi, t, s);
    default: return hipErrorInvalidValue;
  }
}

template <int W, bool QUAD, int MODE = -1>
hipError_t grad_cube_wq(const GradArgs& a, const Tiling& t, hipStream_t s) {
  constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
  constexpr size_t sh = GradCubeShape<W, TZ, TY, TX>::lds_bytes;
  static_assert(sh <= 160 * 1024 - 1024, "brick gradient LDS exceeds the 160 KiB of a CU");
  static bool attr_set = false;   // raise the dynamic LDS limit once per process
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grad_cube<W, TZ, TY, TX, QUAD, MODE>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  k_grad_cube<W, TZ, TY, TX, QUAD, MODE><<<dim3(t.blocks()), dim3(TZ * TY * TX), sh, s>>>(a);
  return hipGetLastError();
}

template <int W>
hipError_t grad_cube_w(const GradArgs& a, const Tiling& t, hipStream_t s) {
  if (a.moving_quad && a.mode == 0) return grad_cube_wq<W, true, 0>(a, t, s);
  return a.moving_quad ? grad_cube_wq<W, true>(a, t, s) : grad_cube_wq<W, false>(a, t, s);
}

hipError_t grad_launch_cube(const GradArgs& a, int window, const Tiling& t, hipStream_t s) {
  switch (window) {
    case 1: return grad_cube_w<1>(a, t, s);
    case 3: return grad_cube_w<3>(a, t, s);
    case 5: return grad_cube_w<5>(a, t, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- batched launches ------------------------------------------------------
template <int W, int TY, int TX>
hipError_t grad_batch_t(const BatchEntry<GradArgs>* E, const int* owner, int total, bool quad, bool adam,
                        hipStream_t s) {
  constexpr size_t sh = grad_lds<W, TY, TX>();
  constexpr bool occ2 = (W <= 5) && TY == 16 && TX == 32;
  const dim3 g(total), blk(TY * TX);
  if constexpr (occ2) {
    if (quad && adam) k_grad_o4_batch<W, TY, TX, true, 0><<<g, blk, sh, s>>>(E, owner);
    else if (quad) k_grad_o4_batch<W, TY, TX, true><<<g, blk, sh, s>>>(E, owner);
    else k_grad_o4_batch<W, TY, TX><<<g, blk, sh, s>>>(E, owner);
  } else {
    if (quad && adam) k_grad_batch<W, TY, TX, true, 0><<<g, blk, sh, s>>>(E, owner);
    else if (quad) k_grad_batch<W, TY, TX, true><<<g, blk, sh, s>>>(E, owner);
    else k_grad_batch<W, TY, TX><<<g, blk, sh, s>>>(E, owner);
  }
  return hipGetLastError();
}

template <int TY, int TX>
hipError_t grad_batch_tile(const BatchEntry<GradArgs>* E, const int* owner, int total, int window, bool quad,
                           bool adam, hipStream_t s) {
  switch (window) {
    case 1: return grad_batch_t<1, TY, TX>(E, owner, total, quad, adam, s);
    case 3: return grad_batch_t<3, TY, TX>(E, owner, total, quad, adam, s);
    case 5: return grad_batch_t<5, TY, TX>(E, owner, total, quad, adam, s);
    case 7: return grad_batch_t<7, TY, TX>(E, owner, total, quad, adam, s);
    case 9: return grad_batch_t<9, TY, TX>(E, owner, total, quad, adam, s);
    default: return hipErrorInvalidValue;
  }
}

template <int W, bool QUAD, int MODE = -1>
hipError_t grad_cube_batch_wq(const BatchEntry<GradArgs>* E, const int* owner, int total, hipStream_t s) {
  constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
  constexpr size_t sh = GradCubeShape<W, TZ, TY, TX>::lds_bytes;
  static bool attr_set = false;   // raise the dynamic LDS limit once per process
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_grad_cube_batch<W, TZ, TY, TX, QUAD, MODE>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  k_grad_cube_batch<W, TZ, TY, TX, QUAD, MODE><<<dim3(total), dim3(TZ * TY * TX), sh, s>>>(E, owner);
  return hipGetLastError();
}

template <int W>
hipError_t grad_cube_batch_w(const BatchEntry<GradArgs>* E, const int* owner, int total, bool quad, bool adam,
                             hipStream_t s) {
  if (quad && adam) return grad_cube_batch_wq<W, true, 0>(E, owner, total, s);
  return quad ? grad_cube_batch_wq<W, true>(E, owner, total, s) : grad_cube_batch_wq<W, false>(E, owner, total, s);
}

template <int R, int TY, int TX>
hipError_t gauss_batch_r(const BatchEntry<GaussArgs>* E, const int* owner, int total, int epi, hipStream_t s) {
  const dim3 g(total), blk(TY * TX);
  const size_t sh = gauss_lds<R, TY, TX>(epi == EPI_COMPOSE_LDS);
  switch (epi) {
    case EPI_SMOOTH_MAX: k_gauss_batch<R, TY, TX, EPI_SMOOTH_MAX><<<g, blk, sh, s>>>(E, owner); break;
    case EPI_STORE: k_gauss_batch<R, TY, TX, EPI_STORE><<<g, blk, sh, s>>>(E, owner); break;
    case EPI_COMPOSE_LDS:
    case EPI_COMPOSE:
      // the composition runs with the single tap (radius 0) only
      if constexpr (R == 0) {
        if (epi == EPI_COMPOSE_LDS) k_gauss_batch<0, TY, TX, EPI_COMPOSE_LDS><<<g, blk, sh, s>>>(E, owner);
        else k_gauss_batch<0, TY, TX, EPI_COMPOSE><<<g, blk, sh, s>>>(E, owner);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TY, int TX>
hipError_t gauss_batch_tile(const BatchEntry<GaussArgs>* E, const int* owner, int total, int radius, int epi,
                            hipStream_t s) {
  switch (radius) {
    case 0: return gauss_batch_r<0, TY, TX>(E, owner, total, epi, s);
    case 1: return gauss_batch_r<1, TY, TX>(E, owner, total, epi, s);
    case 2: return gauss_batch_r<2, TY, TX>(E, owner, total, epi, s);
    case 3: return gauss_batch_r<3, TY, TX>(E, owner, total, epi, s);
    case 4: return gauss_batch_r<4, TY, TX>(E, owner, total, epi, s);
    case 5: return gauss_batch_r<5, TY, TX>(E, owner, total, epi, s);
    case 6: return gauss_batch_r<6, TY, TX>(E, owner, total, epi, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
hipError_t gauss_cube_batch_r(const BatchEntry<GaussArgs>* E, const int* owner, int total, int epi,
                              hipStream_t s) {
  constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
  constexpr size_t sh = sizeof(float) * 3 *
                        ((TZ + 2 * R) * (TY + 2 * R) * (TX + 2 * R) + (TZ + 2 * R) * (TY + 2 * R) * TX);
  const dim3 g(total), blk(TZ * TY * TX);
  switch (epi) {
    case EPI_SMOOTH_MAX: k_gauss_cube_batch<R, TZ, TY, TX, EPI_SMOOTH_MAX><<<g, blk, sh, s>>>(E, owner); break;
    case EPI_STORE: k_gauss_cube_batch<R, TZ, TY, TX, EPI_STORE><<<g, blk, sh, s>>>(E, owner); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t gauss_cube_batch(const BatchEntry<GaussArgs>* E, const int* owner, int total, int radius, int epi,
                            hipStream_t s) {
  if (epi == EPI_COMPOSE_LDS) {
    if (radius != 0) return hipErrorInvalidValue;
    constexpr int TZ = kCubeZ, TY = kCubeY, TX = kCubeX;
    constexpr size_t sh = sizeof(float) * 3 * (TZ + 2) * (TY + 2) * (TX + 2);
    k_compose_cube_batch<TZ, TY, TX><<<dim3(total), dim3(TZ * TY * TX), sh, s>>>(E, owner);
    return hipGetLastError();
  }
  switch (radius) {
    case 0: return gauss_cube_batch_r<0>(E, owner, total, epi, s);
    case 1: return gauss_cube_batch_r<1>(E, owner, total, epi, s);
    case 2: return gauss_cube_batch_r<2>(E, owner, total, epi, s);
    case 3: return gauss_cube_batch_r<3>(E, owner, total, epi, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool grad_tile_supported(int ty, int tx) { return (ty == 16 && tx == 32) || (ty == 8 && tx == 32); }
bool grad_cube_supported(int window) { return window == 1 || window == 3 || window == 5; }

bool gauss_cube_supported(int radius, int epilogue) {
  if (epilogue == EPI_COMPOSE_LDS) return radius == 0;
  return (epilogue == EPI_SMOOTH_MAX || epilogue == EPI_STORE) && radius >= 0 && radius <= 3;
}

bool gauss_tile_supported(int ty, int tx) {
  return (ty == 16 && tx == 32) || (ty == 8 && tx == 32) || (ty == 8 && tx == 64);
}

size_t grad_lds_bytes(int window, int ty, int tx) {
  const int R = window / 2;
  const int GS = (R == 0) ? 1 : 2 * R;
  const size_t base = sizeof(float) * (size_t)(5 * (ty + 4 * R) * (tx + 4 * R) + 5 * (ty + 4 * R) * (tx + 2 * R));
  const size_t ring = sizeof(float) * (size_t)(3 * GS * ty * tx);
  return base + ring <= 65536 ? base + ring : base;
}

size_t gauss_lds_bytes(int radius, int ty, int tx) {
  return sizeof(float) * (size_t)(3 * (ty + 2 * radius) * (tx + 2 * radius) + 3 * (ty + 2 * radius) * tx +
                                  9 * (((ty + 2) * (tx + 2) + 31) / 32 * 32));
}

hipError_t launch_grad(const GradArgs& a, int window, const Tiling& t, hipStream_t s) {
  if (t.cube) return grad_launch_cube(a, window, t, s);
  if (t.ty == 16 && t.tx == 32) return grad_launch_tile<16, 32>(a, window, t, s);
  if (t.ty == 8 && t.tx == 32) return grad_launch_tile<8, 32>(a, window, t, s);
  return hipErrorInvalidValue;
}

bool grad_batch_supported(int window, const Tiling& t) {
  if (t.cube) return grad_cube_supported(window);
  return grad_tile_supported(t.ty, t.tx) && window >= 1 && window <= kMaxWindow && window % 2 == 1;
}

bool gauss_batch_supported(int radius, int epilogue, const Tiling& t) {
  if (t.cube) return gauss_cube_supported(radius, epilogue);
  if (!gauss_tile_supported(t.ty, t.tx) || radius < 0 || radius > kMaxRadius) return false;
  if (epilogue == EPI_SMOOTH_MAX || epilogue == EPI_STORE) return true;
  return (epilogue == EPI_COMPOSE_LDS || epilogue == EPI_COMPOSE) && radius == 0;
}

hipError_t launch_grad_batch(const BatchEntry<GradArgs>* E, const int* owner, int total, int window,
                             const Tiling& t, bool quad, bool adam, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  if (t.cube) {
    switch (window) {
      case 1: return grad_cube_batch_w<1>(E, owner, total, quad, adam, s);
      case 3: return grad_cube_batch_w<3>(E, owner, total, quad, adam, s);
      case 5: return grad_cube_batch_w<5>(E, owner, total, quad, adam, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (t.ty == 16 && t.tx == 32) return grad_batch_tile<16, 32>(E, owner, total, window, quad, adam, s);
  if (t.ty == 8 && t.tx == 32) return grad_batch_tile<8, 32>(E, owner, total, window, quad, adam, s);
  return hipErrorInvalidValue;
}

hipError_t launch_gauss_batch(const BatchEntry<GaussArgs>* E, const int* owner, int total, int radius,
                              int epilogue, const Tiling& t, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  if (t.cube) return gauss_cube_batch(E, owner, total, radius, epilogue, s);
  if (t.ty == 16 && t.tx == 32) return gauss_batch_tile<16, 32>(E, owner, total, radius, epilogue, s);
  if (t.ty == 8 && t.tx == 32) return gauss_batch_tile<8, 32>(E, owner, total, radius, epilogue, s);
  if (t.ty == 8 && t.tx == 64) return gauss_batch_tile<8, 64>(E, owner, total, radius, epilogue, s);
  return hipErrorInvalidValue;
}

hipError_t launch_gauss_narrow(const GaussArgs& a, int radius, int epilogue, const Tiling& t, hipStream_t s) {
  if (t.cube) return gauss_launch_cube(a, radius, epilogue, t, s);
  if (t.ty == 16 && t.tx == 32) return gauss_launch_tile<16, 32>(a, radius, epilogue, t, s);
  if (t.ty == 8 && t.tx == 32) return gauss_launch_tile<8, 32>(a, radius, epilogue, t, s);
  if (t.ty == 8 && t.tx == 64) return gauss_launch_tile<8, 64>(a, radius, epilogue, t, s);
  return hipErrorInvalidValue;
}

// Radius above kMaxRadius (sigma_grad or sigma_warp or the inverse's widths
// above 2 voxels): three separable passes, the last with the epilogue (max
// norm, or a plain store):
//   in -> out (n2), out -> wide_tmp (n1), wide_tmp -> out (n0).
// Needs a.wide_tmp distinct from a.in and a.out, a.in != a.out, and a tap
// table a.wts of 2R + 1 taps followed by zeros up to a multiple of 16 (the
// runtime's tables are laid out so).
hipError_t launch_gauss_wide(const GaussArgs& a, int radius, int epilogue, const Tiling& t, hipStream_t s) {
  (void)t;
  if (radius > kMaxWideRadius || !a.wide_tmp || a.wide_tmp == a.in || a.wide_tmp == a.out || a.in == a.out ||
      (epilogue != EPI_SMOOTH_MAX && epilogue != EPI_STORE))
    return hipErrorInvalidValue;
  const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
  if (n0 > 65535 || n1 > 65535) return hipErrorInvalidValue;
  const int l8 = (2 * radius + 1 + 7) / 8 * 8;
  const size_t shx = sizeof(float) * 3 * (256 + 2 * radius);
  // one component staged at a time: the run plus the taps rounded up to 8
  const size_t shyz = sizeof(float) * (kWideRun + l8) * 64;
  k_field_wide_x<<<dim3((n2 + 255) / 256, n1, n0), dim3(256), shx, s>>>(a.in, a.out, n0, n1, n2, a.wts, radius);
  k_field_wide_yz<1, EPI_STORE><<<dim3((n2 + 63) / 64, (n1 + kWideRun - 1) / kWideRun, n0), dim3(kWideThreads), shyz, s>>>(
      a.out, a.wide_tmp, n0, n1, n2, a.wts, radius, a);
  const dim3 g0((n2 + 63) / 64, (n0 + kWideRun - 1) / kWideRun, n1);
  switch (epilogue) {
    case EPI_SMOOTH_MAX:
      k_field_wide_yz<0, EPI_SMOOTH_MAX><<<g0, dim3(kWideThreads), shyz, s>>>(a.wide_tmp, a.out, n0, n1, n2, a.wts,
                                                                           radius, a);
      break;
    default:
      k_field_wide_yz<0, EPI_STORE><<<g0, dim3(kWideThreads), shyz, s>>>(a.wide_tmp, a.out, n0, n1, n2, a.wts, radius,
                                                                      a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_gauss(const GaussArgs& a, int radius, int epilogue, const Tiling& t, hipStream_t s) {
  if (radius > kMaxRadius) return launch_gauss_wide(a, radius, epilogue, t, s);
  return launch_gauss_narrow(a, radius, epilogue, t, s);
}


static inline unsigned grid1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_eulerian_adam(float* ga, const float* d, float* m, float* v, Ctl* ctl, int n0, int n1,
                                int n2, float beta1, float beta2, float adam_eps, hipStream_t s) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_eulerian_adam, dim3(blocks), dim3(256), 0, s, ga, d, m, v, ctl, n0, n1, n2, beta1, beta2,
                     adam_eps);
  return hipGetLastError();
}

hipError_t launch_pad(const float* in, float* out, int n0, int n1, int n2, hipStream_t s) {
  const int64_t total = (int64_t)(n0 + 2 * kPad) * (n1 + 2 * kPad) * (n2 + 2 * kPad);
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad, dim3(blocks), dim3(256), 0, s, in, out, n0, n1, n2);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, float value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid1(n, 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

template <int R>
hipError_t blur_axis_run(const float* in, float* out, int n0, int n1, int n2, int axis, const float* wts,
                         hipStream_t s) {
  constexpr int T = 8;
  const int n = axis == 0 ? n0 : n1;
  const int64_t threads = (int64_t)n0 * n1 * n2 / n * ((n + T - 1) / T);
  hipLaunchKernelGGL((k_blur_axis_run<R, T>), dim3(grid1(threads, 256)), dim3(256), 0, s, in, out, n0, n1, n2,
                     axis, wts);
  return hipGetLastError();
}

template <int R>
hipError_t blur_x(const float* in, float* out, int n0, int n1, int n2, const float* wts, hipStream_t s) {
  hipLaunchKernelGGL((k_blur_x<R>), dim3(grid1(n2, 256), n1, n0), dim3(256), 0, s, in, out, n2, wts);
  return hipGetLastError();
}

hipError_t launch_pad_quad(const float* pad, float* quad, int n0, int n1, int n2, hipStream_t s) {
  const int p0 = n0 + 2 * kPad, p1 = n1 + 2 * kPad, p2 = n2 + 2 * kPad;
  const int64_t n = (int64_t)p0 * p1 * p2;
  hipLaunchKernelGGL(k_pad_quad, dim3(grid1(n, 256)), dim3(256), 0, s, pad, reinterpret_cast<float4*>(quad), p0,
                     p1, p2);
  return hipGetLastError();
}

hipError_t launch_blur_axis(const float* in, float* out, int n0, int n1, int n2, int axis,
                            const float* wts, int radius, hipStream_t s) {
  if (axis == 2 && n0 <= 65535 && n1 <= 65535) {   // grid y and z hold n1 and n0
    switch (radius) {
      case 1: return blur_x<1>(in, out, n0, n1, n2, wts, s);
      case 2: return blur_x<2>(in, out, n0, n1, n2, wts, s);
      case 3: return blur_x<3>(in, out, n0, n1, n2, wts, s);
      case 4: return blur_x<4>(in, out, n0, n1, n2, wts, s);
      case 5: return blur_x<5>(in, out, n0, n1, n2, wts, s);
      case 6: return blur_x<6>(in, out, n0, n1, n2, wts, s);
      default: break;
    }
  }
  if (axis != 2) {   // the run form for strided axes (radii of the pyramid's usual scales)
    switch (radius) {
      case 1: return blur_axis_run<1>(in, out, n0, n1, n2, axis, wts, s);
      case 2: return blur_axis_run<2>(in, out, n0, n1, n2, axis, wts, s);
      case 3: return blur_axis_run<3>(in, out, n0, n1, n2, axis, wts, s);
      case 4: return blur_axis_run<4>(in, out, n0, n1, n2, axis, wts, s);
      case 5: return blur_axis_run<5>(in, out, n0, n1, n2, axis, wts, s);
      case 6: return blur_axis_run<6>(in, out, n0, n1, n2, axis, wts, s);
      default: break;
    }
  }
  const int64_t n = (int64_t)n0 * n1 * n2;
  hipLaunchKernelGGL(k_blur_axis, dim3(grid1(n, 256)), dim3(256), 0, s, in, out, n0, n1, n2, axis, wts, radius);
  return hipGetLastError();
}

hipError_t launch_resample(const float* in, float* out, int nin0, int nin1, int nin2, int nout0,
                           int nout1, int nout2, int nch, float rho0, float rho1, float rho2,
                           hipStream_t s) {
  if (nout0 <= 65535 && nout1 <= 65535) {   // grid z and y hold n0 and n1
    hipLaunchKernelGGL(k_resample<true>, dim3(grid1(nout2, 256), nout1, nout0), dim3(256), 0, s, in, out, nin0,
                       nin1, nin2, nout0, nout1, nout2, nch, rho0, rho1, rho2);
  } else {
    const int64_t n = (int64_t)nout0 * nout1 * nout2;
    hipLaunchKernelGGL(k_resample<false>, dim3(grid1(n, 256)), dim3(256), 0, s, in, out, nin0, nin1, nin2,
                       nout0, nout1, nout2, nch, rho0, rho1, rho2);
  }
  return hipGetLastError();
}

hipError_t launch_warp(const float* img, const float* d, float* out, int n0, int n1, int n2, hipStream_t s) {
  if (n0 <= 65535 && n1 <= 65535) {
    hipLaunchKernelGGL(k_warp<true>, dim3(grid1(n2, 256), n1, n0), dim3(256), 0, s, img, d, out, n0, n1, n2);
  } else {
    const int64_t n = (int64_t)n0 * n1 * n2;
    hipLaunchKernelGGL(k_warp<false>, dim3(grid1(n, 256)), dim3(256), 0, s, img, d, out, n0, n1, n2);
  }
  return hipGetLastError();
}

hipError_t launch_compose_fields(const float* u, const float* d, float* out, int n0, int n1, int n2,
                                hipStream_t s) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  hipLaunchKernelGGL(k_compose_fields, dim3(grid1(n, 256)), dim3(256), 0, s, u, d, out, n0, n1, n2);
  return hipGetLastError();
}

hipError_t launch_soa_to_aos(const float* in, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_soa_to_aos, dim3(grid1(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_ctl_init(Ctl* ctl, float beta1, float beta2, int t_done, int iter, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, beta1, beta2, t_done, iter);
  return hipGetLastError();
}

hipError_t launch_mean(const float* x, int64_t n, double* scratch, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partial, dim3(kMeanBlocks), dim3(256), 0, s, x, n, scratch);
  hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(256), 0, s, scratch, kMeanBlocks, (double)n, dst);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int n, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partials, n, dst);
  return hipGetLastError();
}

hipError_t launch_partials_ratio(const double* partials, int n, double denom, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(256), 0, s, partials, n, denom, dst);
  return hipGetLastError();
}

}  // namespace fa
