// Measurement probe (not part of the library): the cost of a grid-wide
// barrier inside one cooperative launch against the cost of a kernel boundary
// on the same stream, for launch shapes of the registration's kernels.
//
//   k_empty: back-to-back launches of a near-empty kernel (optionally writing
//            `words` floats per thread) -> microseconds per launch;
//   k_bar:   one cooperative launch running `rounds` grid barriers (one
//            agent-scope counter, generation flag) -> microseconds per round;
//   k_bar2:  the same with a two-level barrier (eight group counters, then
//            one), waiters sleeping 1 or 8 units between polls.
//
// Every wait is bounded: a spin limit sets an error flag and leaves the loop,
// so the launch always ends.  Cooperative launches fail instead of starting
// when the grid cannot be resident at once.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2404_01249_amd/probes/grid_barrier.hip -o grid_barrier && ./grid_barrier
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("%s: %s\n", #x, hipGetErrorString(e)); exit(1);} } while (0)

struct Bar { unsigned count; unsigned pad0[63]; unsigned gen; unsigned pad1[63]; };

__device__ __forceinline__ void grid_barrier(Bar* b, unsigned nblocks, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&b->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 24)) { atomicExch(err, 1); break; }
      }
    }
  }
  __syncthreads();
}

struct Bar2 { unsigned grp[8][64]; unsigned top; unsigned pad[63]; unsigned gen; unsigned pad2[63]; };

template <int SLEEP>
__device__ __forceinline__ void grid_barrier2(Bar2* b, unsigned nblocks, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned grp = blockIdx.x & 7u;
    const unsigned members = (nblocks >> 3) + ((grp < (nblocks & 7u)) ? 1u : 0u);
    const unsigned groups = nblocks < 8 ? nblocks : 8u;
    bool last = false;
    const unsigned a = __hip_atomic_fetch_add(&b->grp[grp][0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == members - 1) {
      __hip_atomic_store(&b->grp[grp][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned t = __hip_atomic_fetch_add(&b->top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (t == groups - 1) {
        __hip_atomic_store(&b->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&b->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      unsigned spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(SLEEP);
        if (++spins > (1u << 24)) { atomicExch(err, 1); break; }
      }
    }
  }
  __syncthreads();
}

template <int SLEEP>
__global__ void k_bar2(Bar2* b, int rounds, int words, float* out, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int r = 0; r < rounds; ++r) {
    if (words > 0) {
      const int j = ((blockIdx.x + 1) % gridDim.x) * blockDim.x + threadIdx.x;
      float v = (r > 0) ? out[j] : 0.f;
      for (int k = 0; k < words; ++k) out[(size_t)k * gridDim.x * blockDim.x + i] = v + 1.f;
    }
    grid_barrier2<SLEEP>(b, gridDim.x, err);
  }
}

__global__ void k_empty(float* out, int words) {
  extern __shared__ float lds[];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float v = 0.f;
  if (words > 0) {
    lds[threadIdx.x] = (float)i;
    __syncthreads();
    v = lds[(threadIdx.x + 1) % blockDim.x];
    for (int k = 0; k < words; ++k) out[(size_t)k * gridDim.x * blockDim.x + i] = v + k;
  } else if (threadIdx.x == 0) out[blockIdx.x] = 1.f;
}

__global__ void k_bar(Bar* b, int rounds, int words, float* out, int* err) {
  extern __shared__ float lds[];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int r = 0; r < rounds; ++r) {
    if (words > 0) {
      // read a neighbour block's data written in the previous round
      const int j = ((blockIdx.x + 1) % gridDim.x) * blockDim.x + threadIdx.x;
      float v = (r > 0) ? out[j] : 0.f;
      for (int k = 0; k < words; ++k) out[(size_t)k * gridDim.x * blockDim.x + i] = v + 1.f;
    }
    grid_barrier(b, gridDim.x, err);
  }
}

int main() {
  int dev = 0; CK(hipSetDevice(dev));
  hipDeviceProp_t pr; CK(hipGetDeviceProperties(&pr, dev));
  printf("device %s CUs %d\n", pr.gcnArchName, pr.multiProcessorCount);
  float* out; CK(hipMalloc(&out, (size_t)64 << 20));
  Bar* b; CK(hipMalloc(&b, sizeof(Bar))); CK(hipMemset(b, 0, sizeof(Bar)));
  Bar2* b2; CK(hipMalloc(&b2, sizeof(Bar2))); CK(hipMemset(b2, 0, sizeof(Bar2)));
  int* err; CK(hipMalloc(&err, sizeof(int))); CK(hipMemset(err, 0, sizeof(int)));
  hipEvent_t e0, e1; CK(hipEventCreate(&e0)); CK(hipEventCreate(&e1));
  struct Cfg { int grid, threads, lds, words; };
  std::vector<Cfg> cfgs = {{240, 512, 134 * 1024, 0}, {240, 512, 134 * 1024, 8}, {512, 256, 0, 0},
                           {512, 256, 0, 8}, {256, 1024, 64 * 1024, 0}, {1024, 256, 16 * 1024, 4}};
  for (auto c : cfgs) {
    // bounds: words * grid * threads floats must fit in 64 MiB
    if ((size_t)c.words * c.grid * c.threads * 4 > ((size_t)64 << 20)) { printf("skip\n"); continue; }
    CK(hipFuncSetAttribute((const void*)k_empty, hipFuncAttributeMaxDynamicSharedMemorySize, c.lds));
    CK(hipFuncSetAttribute((const void*)k_bar, hipFuncAttributeMaxDynamicSharedMemorySize, c.lds));
    int per_cu = 0;
    CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bar, c.threads, c.lds));
    const int reps = 2000;
    for (int w = 0; w < 2; ++w) {
      CK(hipEventRecord(e0));
      for (int r = 0; r < reps; ++r) k_empty<<<c.grid, c.threads, c.lds>>>(out, c.words);
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
    }
    float ms_k; CK(hipEventElapsedTime(&ms_k, e0, e1));
    float ms_b = -1.f;
    if (per_cu * pr.multiProcessorCount >= c.grid) {
      int rounds = reps;
      void* args[] = {&b, &rounds, &c.words, &out, &err};
      for (int w = 0; w < 2; ++w) {
        CK(hipEventRecord(e0));
        CK(hipLaunchCooperativeKernel((const void*)k_bar, dim3(c.grid), dim3(c.threads), args, c.lds, 0));
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
      }
      CK(hipEventElapsedTime(&ms_b, e0, e1));
    }
    float ms_h[2] = {-1.f, -1.f};
    if (per_cu * pr.multiProcessorCount >= c.grid) {
      int rounds = reps;
      void* args[] = {&b2, &rounds, &c.words, &out, &err};
      const void* fns[2] = {(const void*)k_bar2<1>, (const void*)k_bar2<8>};
      for (int f = 0; f < 2; ++f) {
        CK(hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize, c.lds));
        for (int w = 0; w < 2; ++w) {
          CK(hipEventRecord(e0));
          CK(hipLaunchCooperativeKernel(fns[f], dim3(c.grid), dim3(c.threads), args, c.lds, 0));
          CK(hipEventRecord(e1));
          CK(hipEventSynchronize(e1));
        }
        CK(hipEventElapsedTime(&ms_h[f], e0, e1));
      }
    }
    printf("   hierarchical barrier: sleep1 %.2f us/round, sleep8 %.2f us/round\n", 1000.f * ms_h[0] / reps, 1000.f * ms_h[1] / reps);
    int herr = 0; CK(hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost));
    printf("grid %4d threads %4d lds %6d words %d (resident/CU %d): kernel %.2f us/launch, barrier %.2f us/round, err %d\n",
           c.grid, c.threads, c.lds, c.words, per_cu, 1000.f * ms_k / reps, ms_b < 0 ? -1.f : 1000.f * ms_b / reps, herr);
  }
  return 0;
}
