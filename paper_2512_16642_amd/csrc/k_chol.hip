// Penalty and Cholesky factorisation of every frequency block (of one or many
// surveys).
//
// Paper: Q = S S^T + mu I (Hessian definition); each Nr x Nr block Qhat(w) of the
// block-diagonal frequency system is inverted and stored (frequency-domain
// inversion; last step of the Fourier block-diagonal Hessian algorithm).  The
// inverse is applied through a Cholesky factor Qhat = L L^H computed once and
// kept resident.  One workgroup factors one frequency (right-looking, column by
// column, trailing update spread over the workgroup).
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

template <class R>
struct cplx;
template <>
struct cplx<double> {
  using T = double2;
  __device__ static T make(double a, double b) { return make_double2(a, b); }
};
template <>
struct cplx<float> {
  using T = float2;
  __device__ static T make(float a, float b) { return make_float2(a, b); }
};

// In-place lower Cholesky of A (n x n, row-major, complex).  Reads the lower
// triangle, leaves L there and zeros above.  status[f] = 0 on success, 1 if a
// pivot is not positive and finite.
template <class R>
__device__ void chol_inplace(typename cplx<R>::T* A, int n, int32_t* status_f) {
  using C = typename cplx<R>::T;
  __shared__ int bad;
  __shared__ R piv;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      R d = A[(size_t)k * n + k].x;
      if (!(d > R(0)) || !isfinite(d)) {
        bad = 1;
      } else {
        piv = sqrt(d);
        A[(size_t)k * n + k] = cplx<R>::make(piv, R(0));
      }
    }
    __syncthreads();
    if (bad) break;
    R inv = R(1) / piv;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
      C a = A[(size_t)i * n + k];
      A[(size_t)i * n + k] = cplx<R>::make(a.x * inv, a.y * inv);
    }
    __syncthreads();
    // trailing update of the lower triangle: A[i][j] -= A[i][k] conj(A[j][k]), k < j <= i
    const int m = n - k - 1;
    const int mm = m * m;
    for (int p = threadIdx.x; p < mm; p += blockDim.x) {
      int ii = p / m, jj = p % m;
      if (jj > ii) continue;
      int i = k + 1 + ii, j = k + 1 + jj;
      C lik = A[(size_t)i * n + k], ljk = A[(size_t)j * n + k];
      C a = A[(size_t)i * n + j];
      // lik * conj(ljk)
      R pr = lik.x * ljk.x + lik.y * ljk.y;
      R pim = lik.y * ljk.x - lik.x * ljk.y;
      A[(size_t)i * n + j] = cplx<R>::make(a.x - pr, a.y - pim);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *status_f = bad;
  __syncthreads();
  // zero the strict upper triangle
  for (long long e = threadIdx.x; e < (long long)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    if (j > i) A[e] = cplx<R>::make(R(0), R(0));
  }
}

// One job = one (survey, frequency): Qhat = Hhat + mu I, then the Cholesky
// factor in FP64 (kept in lfac, with a complex64 copy in l32) or, for the plain
// form, in FP32 directly in l32.  A workgroup per job; any mix of sizes and
// forms in one launch (the batched-survey factorisation).
__global__ void __launch_bounds__(256) k_factor_jobs(const FactorJob* __restrict__ jobs) {
  const FactorJob j = jobs[blockIdx.x];
  const int n = j.nr;
  const size_t nn = (size_t)n * n;
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x) {
    double2 v = j.hhat[e];
    if (e % (n + 1) == 0) v = make_double2(v.x + j.mu, 0.0);
    j.qhat[e] = v;
  }
  __syncthreads();
  if (j.fp64) {
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x) j.lfac[e] = j.qhat[e];
    __syncthreads();
    chol_inplace<double>(j.lfac, n, j.status);
    __syncthreads();
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x)
      j.l32[e] = make_float2((float)j.lfac[e].x, (float)j.lfac[e].y);
  } else {
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x)
      j.l32[e] = make_float2((float)j.qhat[e].x, (float)j.qhat[e].y);
    __syncthreads();
    chol_inplace<float>(j.l32, n, j.status);
  }
}

}  // namespace

hipError_t launch_factor_jobs(const FactorJob* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_jobs, dim3(njobs), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

}  // namespace ehi
