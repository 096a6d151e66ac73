// Diagonal loading for non-walk-summable systems (Ch. 5 Sec. 5.2).
//
// With A normalised to unit diagonal, J = I - R, the loaded matrix
// J + gamma I is walk-summable for gamma > rho(|R|) - 1.  rho(|R|) is
// estimated on the device by power iteration on M = |R| + I, where
// |R|_ij = |A_ij| / sqrt(|A_ii A_jj|): M is symmetric and nonnegative, so for a
// positive iterate v the Rayleigh quotient v^T M v / v^T v bounds rho(M) from
// below and max_i (M v)_i / v_i bounds it from above (Collatz-Wielandt); the
// shift by I keeps the Perron root strictly dominant.  The loading uses the
// upper bound: gamma = (1 + delta) * rho_hi - 1 (0 when rho_hi < 1), applied
// as Gamma = gamma * diag(A).
#include <algorithm>
#include <cmath>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kLB = 256;

struct WalkScalars {
  double scale;   // 1 / max(y) of the previous iterate
  double lo, hi;  // bounds on rho(|R|)
  double ymax;
};

__global__ void k_walk_weights(int32_t n, const int32_t* __restrict__ off_ptr, const int32_t* __restrict__ col,
                               const double* __restrict__ a, const double* __restrict__ d, double* __restrict__ w) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double sr = 1.0 / sqrt(fabs(d[r]));
  for (int32_t s = off_ptr[r]; s < off_ptr[r + 1]; ++s) w[s] = fabs(a[s]) * sr / sqrt(fabs(d[col[s]]));
}

__global__ void k_walk_init(int32_t n, double* y, WalkScalars* ws) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 1.0;
  if (i == 0) {
    ws->scale = 1.0;
    ws->lo = 0.0;
    ws->hi = 1e300;
    ws->ymax = 1.0;
  }
}

// One step y = M v with v = yin * scale; per-workgroup partial sums of v.y,
// v.v and the maxima of y_i / v_i and y_i.
__global__ __launch_bounds__(kLB) void k_walk_step(int32_t n, const int32_t* __restrict__ off_ptr,
                                                   const int32_t* __restrict__ col, const double* __restrict__ w,
                                                   const double* __restrict__ yin, double* __restrict__ yout,
                                                   const WalkScalars* ws, double4* partials) {
  __shared__ double4 s_p[kLB];
  const double scale = ws->scale;
  const int r = blockIdx.x * kLB + threadIdx.x;
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
  if (r < n) {
    const double v = yin[r] * scale;
    double y = v;
    for (int32_t s = off_ptr[r]; s < off_ptr[r + 1]; ++s) y += w[s] * (yin[col[s]] * scale);
    yout[r] = y;
    p.x = v * y;
    p.y = v * v;
    p.z = v > 0.0 ? y / v : 0.0;
    p.w = y;
  }
  s_p[threadIdx.x] = p;
  __syncthreads();
  for (int off = kLB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double4 q = s_p[threadIdx.x + off];
      double4& m = s_p[threadIdx.x];
      m.x += q.x;
      m.y += q.y;
      m.z = fmax(m.z, q.z);
      m.w = fmax(m.w, q.w);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s_p[0];
}

__global__ __launch_bounds__(kLB) void k_walk_finish(int nparts, const double4* partials, WalkScalars* ws) {
  __shared__ double4 s_p[kLB];
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
  for (int i = threadIdx.x; i < nparts; i += kLB) {
    const double4 q = partials[i];
    p.x += q.x;
    p.y += q.y;
    p.z = fmax(p.z, q.z);
    p.w = fmax(p.w, q.w);
  }
  s_p[threadIdx.x] = p;
  __syncthreads();
  for (int off = kLB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double4 q = s_p[threadIdx.x + off];
      double4& m = s_p[threadIdx.x];
      m.x += q.x;
      m.y += q.y;
      m.z = fmax(m.z, q.z);
      m.w = fmax(m.w, q.w);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double4 t = s_p[0];
    ws->lo = t.x / t.y - 1.0;
    ws->hi = t.z - 1.0;
    ws->ymax = t.w;
    ws->scale = t.w > 0.0 ? 1.0 / t.w : 1.0;
  }
}

}  // namespace

gabp_status estimate_walk_rho(Ctx* c, double* lo_out, double* hi_out, int max_iter, double rtol) {
  hipStream_t s = c->stream;
  const int32_t n = c->n;
  *lo_out = 0.0;
  *hi_out = 0.0;
  if (n == 0 || c->E == 0) return GABP_OK;
  const int nb = (n + kLB - 1) / kLB;
  double *w = nullptr, *y0 = nullptr, *y1 = nullptr;
  double4* parts = nullptr;
  WalkScalars* ws = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(w);
    (void)hipFree(y0);
    (void)hipFree(y1);
    (void)hipFree(parts);
    (void)hipFree(ws);
  };
  if (hipMalloc((void**)&w, sizeof(double) * c->E) != hipSuccess ||
      hipMalloc((void**)&y0, sizeof(double) * n) != hipSuccess ||
      hipMalloc((void**)&y1, sizeof(double) * n) != hipSuccess ||
      hipMalloc((void**)&parts, sizeof(double4) * nb) != hipSuccess ||
      hipMalloc((void**)&ws, sizeof(WalkScalars)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(c, GABP_E_OOM, "allocation for the loading estimate failed");
  }
  hipLaunchKernelGGL(k_walk_weights, dim3(nb), dim3(kLB), 0, s, n, c->off_ptr_d, c->off_col_d, c->a64_d, c->d64_d,
                     w);
  hipLaunchKernelGGL(k_walk_init, dim3(nb), dim3(kLB), 0, s, n, y0, ws);
  WalkScalars h{};
  double* ya = y0;
  double* yb = y1;
  gabp_status st = GABP_OK;
  for (int it = 1; it <= max_iter; ++it) {
    hipLaunchKernelGGL(k_walk_step, dim3(nb), dim3(kLB), 0, s, n, c->off_ptr_d, c->off_col_d, w, ya, yb, ws, parts);
    hipLaunchKernelGGL(k_walk_finish, dim3(1), dim3(kLB), 0, s, nb, parts, ws);
    std::swap(ya, yb);
    if (it % 25 == 0 || it == max_iter) {
      hipError_t e = hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        st = hip_fail(c, e, "loading estimate");
        break;
      }
      if (!std::isfinite(h.hi) || !std::isfinite(h.lo)) {
        st = fail(c, GABP_E_NONFINITE, "non-finite spectral estimate");
        break;
      }
      if (h.hi - h.lo <= rtol * std::max(1.0, h.hi)) break;
    }
  }
  if (st == GABP_OK) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(c, e, "loading estimate kernels");
  }
  cleanup();
  *lo_out = h.lo;
  *hi_out = h.hi;
  return st;
}

}  // namespace gabp
