// gabp_solve_noalloc: the plain FP64 solve of gabp_create + gabp_solve for a
// small system, allocating nothing.  For callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).
//
// Everything the call needs beyond the caller's inputs and outputs lives in
// one file-scope device array, `scratch`: the validation flags, the off-
// diagonal CSR split from the caller's full CSR (Alg. 2's neighbourhoods
// N(i), Ch. 3 Sec. 3.3) with the diagonal, the size E, and the solver status.
// The solve itself is the one-workgroup kernel of small.hip, whose messages
// stay in registers and aggregates in LDS.  Two launches (validate and split,
// then solve) and one copy of the status back to the host; no hipMalloc,
// hipFree or allocating library call.  Each device holds its own copy of the
// array; its address is looked up once per device with
// hipGetSymbolAddress and kept.  Calls that overlap on one device share that
// array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kNaRows = kSmallLanes;       // largest n
constexpr int kNaSlots = 4 * kSmallLanes;  // largest number of off-diagonal entries

constexpr int kNaArg = 1;
constexpr int kNaZeroDiag = 2;
constexpr int kNaAsym = 4;
constexpr int kNaNonfinite = 8;
constexpr int kNaTooLarge = 16;

struct NaHeader {
  DevStatus st;        // written by the solve kernel
  int32_t flags;       // kNa* bits of the validation
  int32_t gate;        // nonzero: the solve kernel returns at once
  int32_t E;           // off-diagonal entries
  int32_t pad;
};

struct NaScratch {
  NaHeader h;
  int32_t off_ptr[kNaRows + 1];
  int32_t off_col[kNaSlots];
  double a[kNaSlots];
  double d[kNaRows];
};

constexpr size_t kScratchBytes = (sizeof(NaScratch) + 255) / 256 * 256;

// Validation of the caller's full CSR (the checks of gabp_create) and the
// split into the off-diagonal CSR and the diagonal, by one workgroup: lane r
// takes row r.  The symmetry check runs only on a sound structure, so every
// search stays inside the split arrays.
__global__ __launch_bounds__(kNaRows) void k_na_ingest(int32_t n, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ vals, NaScratch* sc) {
  __shared__ int s_flags;
  __shared__ unsigned long long s_max;
  __shared__ int s_nnz;
  const int r = threadIdx.x;
  if (r == 0) {
    const int nnz = row_ptr[n];
    int f = 0;
    if (row_ptr[0] != 0 || nnz < n) f |= kNaArg;
    else if ((int64_t)nnz - n > kNaSlots) f |= kNaTooLarge;
    s_flags = f;
    s_max = 0ull;
    s_nnz = nnz;
  }
  __syncthreads();
  const int nnz = s_nnz;
  int flags = 0;
  double maxabs = 0.0;
  if (r < n && s_flags == 0) {
    int lo = row_ptr[r], hi = row_ptr[r + 1];
    if (lo < 0 || hi > nnz || hi < lo) {  // never read outside col / vals
      flags |= kNaArg;
      lo = hi = 0;
    }
    int prev = -1, ndiag = 0;
    double dv = 0.0;
    int k = lo - r;  // off-diagonal slot of the row's next off-diagonal entry
    for (int e = lo; e < hi; ++e) {
      const int c = col[e];
      const double v = vals[e];
      if (c < 0 || c >= n || c <= prev) flags |= kNaArg;
      prev = c;
      if (!isfinite(v)) flags |= kNaNonfinite;
      maxabs = fmax(maxabs, fabs(v));
      if (c == r) {
        ++ndiag;
        dv = v;
      } else {
        if (k >= 0 && k < kNaSlots) {
          sc->off_col[k] = c;
          sc->a[k] = v;
        }
        ++k;
      }
    }
    if (ndiag != 1 || dv == 0.0) flags |= kNaZeroDiag;
    sc->d[r] = dv;
    sc->off_ptr[r] = lo - r;
    if (r == n - 1) sc->off_ptr[n] = hi - n;
  }
  if (flags) atomicOr(&s_flags, flags);
  if (isfinite(maxabs) && maxabs > 0.0) atomicMax(&s_max, (unsigned long long)__double_as_longlong(maxabs));
  __syncthreads();
  if (s_flags == 0 && r < n) {
    // |A_ij - A_ji| <= 1e-12 max|A| and the mirror entry present: binary search
    // for column r in row c of the split arrays
    const double tolv = 1e-12 * __longlong_as_double((long long)s_max);
    int asym = 0;
    for (int s = sc->off_ptr[r]; s < sc->off_ptr[r + 1]; ++s) {
      const int c = sc->off_col[s];
      int lo = sc->off_ptr[c], hi = sc->off_ptr[c + 1] - 1, found = -1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = sc->off_col[mid];
        if (v == r) {
          found = mid;
          break;
        }
        if (v < r) lo = mid + 1;
        else hi = mid - 1;
      }
      if (found < 0 || fabs(sc->a[s] - sc->a[found]) > tolv) asym = 1;
    }
    if (asym) atomicOr(&s_flags, kNaAsym);
  }
  __syncthreads();
  if (r == 0) {
    sc->h.flags = s_flags;
    sc->h.gate = s_flags != 0;
    sc->h.E = s_flags ? 0 : nnz - n;
    sc->h.pad = 0;
  }
}

}  // namespace

}  // namespace gabp

// The library's static device buffer of the no-allocation entry point (one
// copy per device, held until the process ends).  Host code never uses this
// name as an address: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[gabp::kScratchBytes];

namespace gabp {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
gabp_status scratch_on_current_device(NaScratch** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, GABP_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, GABP_E_ARG, "device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(nullptr, GABP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = (NaScratch*)g_scratch_ptr[dev];
  return GABP_OK;
}

}  // namespace

}  // namespace gabp

extern "C" gabp_status gabp_solve_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                          const double* vals, const double* b, double* x, double* var, double tol,
                                          int32_t max_iter, hipStream_t stream, gabp_info* info) {
  using namespace gabp;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n < 0) return fail(nullptr, GABP_E_ARG, "n < 0");
  if (n > kNaRows)
    return fail(nullptr, GABP_E_ARG,
                "n = " + std::to_string(n) + " exceeds the no-allocation limit of " + std::to_string(kNaRows) +
                    " rows");
  if (max_iter < 0) return fail(nullptr, GABP_E_ARG, "max_iter < 0");
  if (std::isnan(tol)) return fail(nullptr, GABP_E_ARG, "tol is NaN");
  if (n == 0) {
    if (info) info->converged = 1;
    return GABP_OK;
  }
  if (!row_ptr || !col_idx || !vals || !b || !x) return fail(nullptr, GABP_E_ARG, "NULL argument");
  NaScratch* sc = nullptr;
  gabp_status r = scratch_on_current_device(&sc);
  if (r != GABP_OK) return r;

  hipLaunchKernelGGL(k_na_ingest, dim3(1), dim3(kNaRows), 0, stream, n, row_ptr, col_idx, vals, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, GABP_E_HIP, std::string("validation launch: ") + hipGetErrorString(e));
  SmallArgs a{};
  a.n = n;
  a.E = 0;
  a.E_dev = &sc->h.E;
  a.gate = &sc->h.gate;
  a.off_ptr = sc->off_ptr;
  a.col = sc->off_col;
  a.a = sc->a;
  a.diag = sc->d;
  a.rhs = b;
  a.rhs_norm = nullptr;
  a.tol = tol;
  a.max_iter = max_iter;
  a.check_every = 1;
  a.st = &sc->h.st;
  a.x_direct = x;
  a.var_direct = var;
  e = launch_small_k4(a, stream);
  if (e != hipSuccess) return fail(nullptr, GABP_E_HIP, std::string("solve launch: ") + hipGetErrorString(e));
  NaHeader h{};
  e = hipMemcpyAsync(&h, &sc->h, sizeof(h), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(nullptr, GABP_E_HIP, std::string("status copy: ") + hipGetErrorString(e));

  gabp_status st;
  if (h.flags & kNaArg)
    st = fail(nullptr, GABP_E_ARG,
              "CSR structure: row_ptr[0] != 0, row pointers decrease, columns unsorted/duplicated or out of range");
  else if (h.flags & kNaTooLarge)
    st = fail(nullptr, GABP_E_ARG,
              "the matrix has more than " + std::to_string(kNaSlots) +
                  " off-diagonal entries, the no-allocation limit (use gabp_create)");
  else if (h.flags & kNaNonfinite)
    st = fail(nullptr, GABP_E_NONFINITE, "non-finite matrix value");
  else if (h.flags & kNaZeroDiag)
    st = fail(nullptr, GABP_E_ZERO_DIAG, "a diagonal entry is missing or zero");
  else if (h.flags & kNaAsym)
    st = fail(nullptr, GABP_E_NOT_SYMMETRIC, "pattern or values of A are not symmetric");
  else if (h.st.error & kErrNonfinite)
    st = fail(nullptr, GABP_E_NONFINITE, "non-finite message (P~_i = P_ji or overflow)");
  else if (tol > 0.0 && (h.st.error & kErrDiverged))
    st = fail(nullptr, GABP_E_DIVERGED, "residual diverged");
  else
    st = (tol <= 0.0 || h.st.conv_round >= 0) ? GABP_OK : GABP_NOT_CONVERGED;
  if (info && h.flags == 0) {
    info->sweeps = h.st.conv_round >= 0 ? h.st.conv_round : max_iter;
    info->converged = h.st.conv_round >= 0 ? 1 : 0;
    info->rel_residual = h.st.last_rel;
  }
  if (info) info->status = st;
  return st;
}
