// Measurement aid, not part of libgabp.so: the cost of random 16-byte
// gathers on one device, the access that bounds the sweep kernels on random
// graphs.  Built into libgabp_probe.so beside the library and driven by the
// benchmark's --gather-probe mode.
//
// One launch reads n int32 indices (a coalesced stream) and gathers the
// 16-byte record src[idx[i]] for each; every thread adds up what it gathered
// and writes one record, so the launch moves 4 B of index and one gathered
// record per element plus a small output.  Thread i of the grid handles
// elements i, i + stride, ...; workgroup b runs on XCD b mod 8 under the
// hardware's round-robin dispatch, which is what the XCD-window experiment
// relies on when it builds its indices.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlock = 256;

// The gathered load under a cache policy: 0 plain, 1 non-temporal, 2 and 3
// relaxed atomic loads of the two words at agent and at system scope (the
// memory model's coherent forms).
template <int POL>
__device__ __forceinline__ double2 gather_one(const double2* src, int32_t j) {
  if (POL == 0) return src[j];
  if (POL == 1) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v v = __builtin_nontemporal_load((const d2v*)(src + j));
    return double2{v.x, v.y};
  }
  const double* w = (const double*)(src + j);
  constexpr int scope = POL == 2 ? __HIP_MEMORY_SCOPE_AGENT : __HIP_MEMORY_SCOPE_SYSTEM;
  return double2{__hip_atomic_load(w, __ATOMIC_RELAXED, scope), __hip_atomic_load(w + 1, __ATOMIC_RELAXED, scope)};
}

template <int POL>
__global__ __launch_bounds__(kBlock) void k_gather16(const int32_t* __restrict__ idx, int64_t n,
                                                     const double2* __restrict__ src, int64_t nsrc,
                                                     double2* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double ax = 0.0, ay = 0.0;
  for (int64_t i = tid; i < n; i += stride) {
    const int32_t j = idx[i];
    if (j >= 0 && (int64_t)j < nsrc) {
      const double2 v = gather_one<POL>(src, j);
      ax += v.x;
      ay += v.y;
    }
  }
  out[tid] = double2{ax, ay};
}

}  // namespace

extern "C" {

// Times `reps` launches of the gather over device arrays idx[n] (int32) and
// src[nsrc] (16-byte records) with the gathered load under cache policy
// `policy` (0 plain, 1 non-temporal, 2 agent-scope and 3 system-scope relaxed
// atomic loads of the record's two words); out must hold grid * 256 records.
// Writes the best launch time in milliseconds to *best_ms.  Returns 0, or the
// HIP error (hipErrorInvalidValue for a bad argument).
int gabp_probe_gather16_policy(const int32_t* idx, int64_t n, const void* src, int64_t nsrc, void* out, int grid,
                               int reps, int policy, float* best_ms) {
  if (!idx || !src || !out || !best_ms || n < 0 || nsrc <= 0 || grid < 1 || reps < 1 || policy < 0 || policy > 3)
    return (int)hipErrorInvalidValue;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  const double2* sp = (const double2*)src;
  double2* op = (double2*)out;
  float best = 1e30f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, 0);
    if (e == hipSuccess) {
      switch (policy) {
        case 0: hipLaunchKernelGGL(k_gather16<0>, dim3(grid), dim3(kBlock), 0, 0, idx, n, sp, nsrc, op); break;
        case 1: hipLaunchKernelGGL(k_gather16<1>, dim3(grid), dim3(kBlock), 0, 0, idx, n, sp, nsrc, op); break;
        case 2: hipLaunchKernelGGL(k_gather16<2>, dim3(grid), dim3(kBlock), 0, 0, idx, n, sp, nsrc, op); break;
        default: hipLaunchKernelGGL(k_gather16<3>, dim3(grid), dim3(kBlock), 0, 0, idx, n, sp, nsrc, op); break;
      }
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return (int)e;
}

// The plain-load gather (policy 0).
int gabp_probe_gather16(const int32_t* idx, int64_t n, const void* src, int64_t nsrc, void* out, int grid,
                        int reps, float* best_ms) {
  return gabp_probe_gather16_policy(idx, n, src, nsrc, out, grid, reps, 0, best_ms);
}

}  // extern "C"
