// Evaluation of a registration result (include/fa_eval.h): label transfer by
// nearest neighbour, per-class overlap counts, and det(I + grad d).
//
// All three are single passes over the volume, bound by HBM bandwidth; they
// run once per registration, not per iteration.  Integer results are exact:
// the rounding of a sample position is decided from the fp32 displacement
// without rounding error, and the determinant is evaluated in double
// precision in a fixed order, without contraction into fused multiply-adds.
#include <algorithm>
#include <vector>

#include "fa_eval.h"
#include "fa_host.h"

using fa::fail;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;
constexpr int kMaxClasses = 127;

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxBlocks));
}

// round(x + d) along one axis, half up, decided exactly: with q = floor(d),
// d - q is exact in fp32, so the comparison with 1/2 carries no rounding.
__device__ __forceinline__ bool rounded_coord(int x, float dv, int n, int& p) {
  if (!(fabsf(dv) < 1.0e9f)) return false;   // also rejects NaN
  const float q = floorf(dv);
  const int r = (int)q + ((dv - q) >= 0.5f ? 1 : 0);
  p = x + r;
  return p >= 0 && p < n;
}

__global__ void __launch_bounds__(kThreads)
k_warp_labels(const int8_t* __restrict__ lab, const float* __restrict__ d, int8_t* __restrict__ out,
              int n0, int n1, int n2) {
  const int N = n0 * n1 * n2;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < N; i += gridDim.x * kThreads) {
    const int x2 = i % n2;
    const int t = i / n2;
    const int x1 = t % n1;
    const int x0 = t / n1;
    int p0 = 0, p1 = 0, p2 = 0;
    const bool ok = rounded_coord(x0, d[i], n0, p0) && rounded_coord(x1, d[N + i], n1, p1) &&
                    rounded_coord(x2, d[2 * N + i], n2, p2);
    out[i] = ok ? lab[(p0 * n1 + p1) * n2 + p2] : (int8_t)-1;
  }
}

// Per-workgroup class counts in LDS, written to part[block][3 * nc].
__global__ void __launch_bounds__(kThreads)
k_overlap_partial(const int8_t* __restrict__ a, const int8_t* __restrict__ b, int64_t n, int nc,
                  unsigned* __restrict__ part) {
  __shared__ unsigned cnt[3 * kMaxClasses];
  for (int j = threadIdx.x; j < 3 * nc; j += kThreads) cnt[j] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int va = a[i], vb = b[i];
    const bool ia = (unsigned)va < (unsigned)nc, ib = (unsigned)vb < (unsigned)nc;
    if (ia) atomicAdd(&cnt[3 * va], 1u);
    if (ib) atomicAdd(&cnt[3 * vb + 1], 1u);
    if (ia && va == vb) atomicAdd(&cnt[3 * va + 2], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < 3 * nc; j += kThreads) part[(size_t)blockIdx.x * 3 * nc + j] = cnt[j];
}

// One workgroup per counter: the sum over the workgroups' partial counts.
__global__ void __launch_bounds__(kThreads)
k_overlap_final(const unsigned* __restrict__ part, int nblocks, int nc, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[kThreads];
  const int j = blockIdx.x;
  unsigned long long s = 0ull;
  for (int k = threadIdx.x; k < nblocks; k += kThreads) s += part[(size_t)k * 3 * nc + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// det(I + grad d) by central differences at interior voxels, in double.
// The expression is the cofactor expansion along the first row, evaluated
// left to right with separate multiplies and adds.
__global__ void __launch_bounds__(kThreads)
k_jacdet(const float* __restrict__ d, int n0, int n1, int n2, double* __restrict__ det,
         unsigned* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ unsigned nonpos;
  if (threadIdx.x == 0) nonpos = 0u;
  __syncthreads();
  const int m0 = n0 - 2, m1 = n1 - 2, m2 = n2 - 2;
  const int M = m0 * m1 * m2;
  const int N = n0 * n1 * n2;
  const int s1 = n2, s0 = n1 * n2;
  unsigned mine = 0u;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < M; i += gridDim.x * kThreads) {
    const int k2 = i % m2;
    const int t = i / m2;
    const int k1 = t % m1;
    const int k0 = t / m1;
    const int c = ((k0 + 1) * n1 + (k1 + 1)) * n2 + (k2 + 1);
    double J[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float* f = d + (size_t)q * N;
      J[q][0] = 0.5 * ((double)f[c + s0] - (double)f[c - s0]);
      J[q][1] = 0.5 * ((double)f[c + s1] - (double)f[c - s1]);
      J[q][2] = 0.5 * ((double)f[c + 1] - (double)f[c - 1]);
      J[q][q] = J[q][q] + 1.0;
    }
    const double c0 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c1 = J[1][0] * J[2][2] - J[1][2] * J[2][0];
    const double c2 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double v = J[0][0] * c0 - J[0][1] * c1 + J[0][2] * c2;
    if (det) det[i] = v;
    mine += v <= 0.0 ? 1u : 0u;
  }
  if (mine) atomicAdd(&nonpos, mine);
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = nonpos;
}

__global__ void __launch_bounds__(kThreads)
k_count_final(const unsigned* __restrict__ part, int nblocks, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[kThreads];
  unsigned long long s = 0ull;
  for (int k = threadIdx.x; k < nblocks; k += kThreads) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Stream-ordered scratch freed on every return path.
struct Scratch {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~Scratch() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

}  // namespace

extern "C" {

fa_status fa_warp_labels(const int8_t* labels_dev, const float* d_dev, fa_shape shape, int8_t* out_dev,
                         void* hip_stream) {
  if (!labels_dev || !d_dev || !out_dev) return fail(FA_EINVAL, "labels, d and out must not be NULL");
  FA_TRY(fa::check_shape(shape));
  if ((const void*)labels_dev == (const void*)out_dev) return fail(FA_EINVAL, "out must not alias labels");
  const hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n = fa::voxels(shape);
  hipLaunchKernelGGL(k_warp_labels, dim3(grid_for(n)), dim3(kThreads), 0, s, labels_dev, d_dev, out_dev,
                     shape.n0, shape.n1, shape.n2);
  FA_HIP(hipGetLastError());
  return FA_OK;
}

fa_status fa_label_overlap(const int8_t* a_dev, const int8_t* b_dev, int64_t n, int n_classes,
                           int64_t* counts_host, void* hip_stream) {
  if (!counts_host) return fail(FA_EINVAL, "counts_host is NULL");
  if (n_classes < 1 || n_classes > kMaxClasses) return fail(FA_EINVAL, "n_classes must be in [1, 127]");
  if (n < 0) return fail(FA_EINVAL, "n must be >= 0");
  if (n > 0 && (!a_dev || !b_dev)) return fail(FA_EINVAL, "a and b must not be NULL");
  std::fill(counts_host, counts_host + 3 * n_classes, (int64_t)0);
  if (n == 0) return FA_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  const int nb = grid_for(n);
  const size_t part_bytes = ((size_t)nb * 3 * n_classes * sizeof(unsigned) + 255) & ~(size_t)255;
  Scratch sc;
  sc.s = s;
  FA_HIP(hipMallocAsync(&sc.p, part_bytes + 3 * kMaxClasses * sizeof(unsigned long long), s));
  unsigned* part = (unsigned*)sc.p;
  unsigned long long* tot = (unsigned long long*)((char*)sc.p + part_bytes);
  hipLaunchKernelGGL(k_overlap_partial, dim3(nb), dim3(kThreads), 0, s, a_dev, b_dev, n, n_classes, part);
  FA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_overlap_final, dim3(3 * n_classes), dim3(kThreads), 0, s, part, nb, n_classes, tot);
  FA_HIP(hipGetLastError());
  std::vector<unsigned long long> h((size_t)3 * n_classes);
  FA_HIP(hipMemcpyAsync(h.data(), tot, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  for (size_t j = 0; j < h.size(); ++j) counts_host[j] = (int64_t)h[j];
  return FA_OK;
}

fa_status fa_jacobian_det(const float* d_dev, fa_shape shape, double* det_dev, int64_t* n_nonpos_host,
                          int64_t* n_interior_host, void* hip_stream) {
  if (!d_dev) return fail(FA_EINVAL, "d must not be NULL");
  if (shape.n0 < 1 || shape.n1 < 1 || shape.n2 < 1) return fail(FA_ESHAPE, "every dimension must be >= 1");
  if ((double)shape.n0 * shape.n1 * shape.n2 > 536870911.0)
    return fail(FA_ESHAPE, "volume too large: n0*n1*n2 must be < 2^29");
  const int64_t m = shape.n0 < 3 || shape.n1 < 3 || shape.n2 < 3
                        ? 0
                        : (int64_t)(shape.n0 - 2) * (shape.n1 - 2) * (shape.n2 - 2);
  if (n_interior_host) *n_interior_host = m;
  if (n_nonpos_host) *n_nonpos_host = 0;
  if (m == 0) return FA_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  const int nb = grid_for(m);
  Scratch sc;
  sc.s = s;
  const size_t part_bytes = ((size_t)nb * sizeof(unsigned) + 255) & ~(size_t)255;
  FA_HIP(hipMallocAsync(&sc.p, part_bytes + sizeof(unsigned long long), s));
  unsigned* part = (unsigned*)sc.p;
  unsigned long long* tot = (unsigned long long*)((char*)sc.p + part_bytes);
  hipLaunchKernelGGL(k_jacdet, dim3(nb), dim3(kThreads), 0, s, d_dev, shape.n0, shape.n1, shape.n2, det_dev,
                     part);
  FA_HIP(hipGetLastError());
  if (!n_nonpos_host) return FA_OK;
  hipLaunchKernelGGL(k_count_final, dim3(1), dim3(kThreads), 0, s, part, nb, tot);
  FA_HIP(hipGetLastError());
  unsigned long long h = 0;
  FA_HIP(hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  *n_nonpos_host = (int64_t)h;
  return FA_OK;
}

fa_status fa_compose_fields(const float* u_dev, const float* d_dev, fa_shape shape, float* out_dev,
                            void* hip_stream) {
  if (!u_dev || !d_dev || !out_dev) return fail(FA_EINVAL, "u, d and out must not be NULL");
  if (out_dev == d_dev) return fail(FA_EINVAL, "out must not alias d");
  FA_TRY(fa::check_shape(shape));
  FA_HIP(fa::launch_compose_fields(u_dev, d_dev, out_dev, shape.n0, shape.n1, shape.n2, (hipStream_t)hip_stream));
  return FA_OK;
}

}  // extern "C"
