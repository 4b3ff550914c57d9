// Penalty and Cholesky factorisation of every frequency block (of one or many
// surveys).
//
// Paper: Q = S S^T + mu I (Hessian definition); each Nr x Nr block Qhat(w) of the
// block-diagonal frequency system is inverted and stored (frequency-domain
// inversion; last step of the Fourier block-diagonal Hessian algorithm).  The
// inverse is applied through a Cholesky factor Qhat = L L^H computed once and
// kept resident.  One workgroup factors one frequency (left-looking, column by
// column, each row's new entry one dot product).
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
// Left-looking, one column at a time: row j's finished part L[j][0..j) is
// staged in LDS, the pivot is d = A[j][j] - sum_k |L[j][k]|^2 (a workgroup
// reduction), and every row i > j forms L[i][j] = (A[i][j] - sum_k L[i][k]
// conj(L[j][k])) / L[j][j] as one dot product over its own finished entries
// (one to eight lanes per row), so each column costs two barriers and no
// element is rewritten by later columns.
template <class R>
__device__ void chol_inplace(typename cplx<R>::T* A, int n, int32_t* status_f) {
  using C = typename cplx<R>::T;
  constexpr int kMaxN = 1024;  // the largest nr the descriptor accepts
  __shared__ C lj[kMaxN];
  __shared__ R red[256 / 64];
  __shared__ int bad;
  __shared__ R piv;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n && n <= kMaxN; ++j) {
    R part = R(0);
    for (int k = threadIdx.x; k < j; k += blockDim.x) {
      const C v = A[(size_t)j * n + k];
      lj[k] = v;
      part += v.x * v.x + v.y * v.y;
    }
    // workgroup sum of |L[j][k]|^2
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      R sum = R(0);
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
      const R d = A[(size_t)j * n + j].x - sum;
      if (!(d > R(0)) || !isfinite(d)) {
        bad = 1;
      } else {
        piv = sqrt(d);
        A[(size_t)j * n + j] = cplx<R>::make(piv, R(0));
      }
    }
    __syncthreads();
    if (bad) break;
    const R inv = R(1) / piv;
    // g lanes per row (more lanes as fewer rows remain, so the workgroup stays
    // busy through the long dot products of the last columns), each summing
    // every g-th k, then a butterfly over the g lanes
    const int rows = n - j - 1;
    const int g = rows <= 8 ? 32 : rows <= 16 ? 16 : rows <= 32 ? 8 : rows <= 64 ? 4 : rows <= 128 ? 2 : 1;
    const int rg = (int)threadIdx.x & (g - 1);
    for (int i0 = j + 1; i0 < n; i0 += (int)blockDim.x / g) {
      const int i = i0 + (int)threadIdx.x / g;
      const bool live = i < n;
      const C* Ai = A + (size_t)(live ? i : j) * n;
      R sr = R(0), si = R(0);
      for (int k = rg; k < j; k += g) {
        const C a = Ai[k], b = lj[k];
        // a * conj(b)
        sr += a.x * b.x + a.y * b.y;
        si += a.y * b.x - a.x * b.y;
      }
      for (int o = 1; o < g; o <<= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
      }
      if (live && rg == 0) {
        const C a = Ai[j];
        A[(size_t)i * n + j] = cplx<R>::make((a.x - sr) * inv, (a.y - si) * inv);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *status_f = (bad || n > kMaxN) ? 1 : 0;
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
