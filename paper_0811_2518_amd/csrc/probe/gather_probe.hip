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

__global__ __launch_bounds__(kBlock) void k_gather16(const int32_t* __restrict__ idx, int64_t n,
                                                     const double2* __restrict__ src, int64_t nsrc,
                                                     double2* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double ax = 0.0, ay = 0.0;
  for (int64_t i = tid; i < n; i += stride) {
    const int32_t j = idx[i];
    if (j >= 0 && (int64_t)j < nsrc) {
      const double2 v = src[j];
      ax += v.x;
      ay += v.y;
    }
  }
  out[tid] = double2{ax, ay};
}

}  // namespace

extern "C" {

// Times `reps` launches of the gather over device arrays idx[n] (int32) and
// src[nsrc] (16-byte records); out must hold grid * 256 records.  Writes the
// best launch time in milliseconds to *best_ms.  Returns 0, or the HIP error.
int gabp_probe_gather16(const int32_t* idx, int64_t n, const void* src, int64_t nsrc, void* out, int grid,
                        int reps, float* best_ms) {
  if (!idx || !src || !out || !best_ms || n < 0 || nsrc <= 0 || grid < 1 || reps < 1) return (int)hipErrorInvalidValue;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  float best = 1e30f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, 0);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_gather16, dim3(grid), dim3(kBlock), 0, 0, idx, n, (const double2*)src, nsrc,
                         (double2*)out);
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

}  // extern "C"
