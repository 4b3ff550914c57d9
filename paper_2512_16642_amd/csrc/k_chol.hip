// Penalty and Cholesky factorisation of every frequency block.
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

__global__ void k_penalty(Geometry g, const double2* __restrict__ hhat, double mu,
                          double2* __restrict__ qhat) {
  const int f = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nr * g.nr) return;
  int i = e / g.nr, j = e % g.nr;
  size_t o = (size_t)f * g.nr * g.nr + e;
  double2 v = hhat[o];
  if (i == j) v = make_double2(v.x + mu, 0.0);
  qhat[o] = v;
}

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

__global__ void __launch_bounds__(256)
    k_potrf_f64(Geometry g, const double2* __restrict__ qhat, double2* __restrict__ lfac,
                float2* __restrict__ l32, int32_t* __restrict__ status) {
  const int f = blockIdx.x;
  const int n = g.nr;
  const size_t nn = (size_t)n * n;
  double2* A = lfac + f * nn;
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x) A[e] = qhat[f * nn + e];
  __syncthreads();
  chol_inplace<double>(A, n, status + f);
  __syncthreads();
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x)
    l32[f * nn + e] = make_float2((float)A[e].x, (float)A[e].y);
}

__global__ void __launch_bounds__(256)
    k_potrf_f32(Geometry g, const double2* __restrict__ qhat, float2* __restrict__ l32,
                int32_t* __restrict__ status) {
  const int f = blockIdx.x;
  const int n = g.nr;
  const size_t nn = (size_t)n * n;
  float2* A = l32 + f * nn;
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x)
    A[e] = make_float2((float)qhat[f * nn + e].x, (float)qhat[f * nn + e].y);
  __syncthreads();
  chol_inplace<float>(A, n, status + f);
}

}  // namespace

hipError_t launch_penalty(const Geometry& g, const double2* hhat, double mu, double2* qhat,
                          hipStream_t st) {
  dim3 grid(cdiv(g.nr * g.nr, 256), g.nf);
  hipLaunchKernelGGL(k_penalty, grid, dim3(256), 0, st, g, hhat, mu, qhat);
  return hipGetLastError();
}

hipError_t launch_potrf_f64(const Geometry& g, const double2* qhat, double2* lfac, float2* lfac32,
                            int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_potrf_f64, dim3(g.nf), dim3(256), 0, st, g, qhat, lfac, lfac32, status);
  return hipGetLastError();
}

hipError_t launch_potrf_f32(const Geometry& g, const double2* qhat, float2* lfac32,
                            int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_potrf_f32, dim3(g.nf), dim3(256), 0, st, g, qhat, lfac32, status);
  return hipGetLastError();
}

}  // namespace ehi
