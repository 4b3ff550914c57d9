// Multi-source deblurring delta d^e(w) = Qhat(w)^{-1} delta d(w).
//
// Paper: the block-diagonal frequency system is solved separately per frequency
// for every source with the stored blocks (frequency-domain inversion; the
// per-source step of the multiplier-based algorithm computes delta d^e in the
// frequency domain).  The factor L (complex64 copy) drives forward and back
// substitution; in the split-BF16 precision mode two refinement steps compute
// the residual R - Qhat X in FP64 and correct X (accumulated in FP64).
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

// One thread per (source, frequency).  work[.][s][.] starts as a copy of the
// right-hand side and is overwritten by the solution of L L^H x = rhs.
__global__ void __launch_bounds__(64)
    k_trsm(Geometry g, const float2* __restrict__ l32, const float2* __restrict__ rhs, int rhs_ld,
           int rhs_off, float2* __restrict__ work, int work_ld, int work_off, int cnt, int mode,
           double2* __restrict__ x64) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (s >= cnt) return;
  const int n = g.nr;
  const float2* L = l32 + (size_t)f * n * n;
  const float2* b = rhs + ((size_t)f * rhs_ld + rhs_off + s) * n;
  float2* v = work + ((size_t)f * work_ld + work_off + s) * n;
  // forward: L y = b
  for (int i = 0; i < n; ++i) {
    float2 t = b[i];
    const float2* Li = L + (size_t)i * n;
    for (int k = 0; k < i; ++k) {
      float2 l = Li[k], y = v[k];
      t.x -= l.x * y.x - l.y * y.y;
      t.y -= l.x * y.y + l.y * y.x;
    }
    float inv = 1.f / Li[i].x;
    v[i] = make_float2(t.x * inv, t.y * inv);
  }
  // back: L^H x = y
  for (int i = n - 1; i >= 0; --i) {
    float2 t = v[i];
    for (int k = i + 1; k < n; ++k) {
      float2 l = L[(size_t)k * n + i], x = v[k];  // conj(l) * x
      t.x -= l.x * x.x + l.y * x.y;
      t.y -= l.x * x.y - l.y * x.x;
    }
    float inv = 1.f / L[(size_t)i * n + i].x;
    v[i] = make_float2(t.x * inv, t.y * inv);
  }
  if (mode == kTrsmStoreX64 || mode == kTrsmAddX64) {
    double2* x = x64 + ((size_t)f * g.max_ns + s) * n;
    for (int i = 0; i < n; ++i) {
      double2 d = make_double2((double)v[i].x, (double)v[i].y);
      if (mode == kTrsmAddX64) {
        double2 o = x[i];
        d.x += o.x;
        d.y += o.y;
      }
      x[i] = d;
    }
  }
}

// r32[f][s][i] = R[f][s0+s][i] - sum_j Qhat[f][i][j] x64[f][s][j], in FP64.
__global__ void __launch_bounds__(64)
    k_residual(Geometry g, const double2* __restrict__ qhat, const float2* __restrict__ resid,
               int resid_ns, int s0, const double2* __restrict__ x64, float2* __restrict__ r32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int f = blockIdx.z;
  const int n = g.nr;
  if (i >= n) return;
  const double2* Q = qhat + (size_t)f * n * n + (size_t)i * n;
  const double2* x = x64 + ((size_t)f * g.max_ns + s) * n;
  double tr = 0.0, ti = 0.0;
  for (int j = 0; j < n; ++j) {
    double2 q = Q[j], v = x[j];
    tr += q.x * v.x - q.y * v.y;
    ti += q.x * v.y + q.y * v.x;
  }
  float2 b = resid[((size_t)f * resid_ns + s0 + s) * n + i];
  r32[((size_t)f * g.max_ns + s) * n + i] = make_float2((float)((double)b.x - tr), (float)((double)b.y - ti));
}

__global__ void k_x_out(Geometry g, const double2* __restrict__ x64, int ns, int s0,
                        float2* __restrict__ out, int out_ns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int f = blockIdx.z;
  if (i >= g.nr || s >= ns) return;
  double2 v = x64[((size_t)f * g.max_ns + s) * g.nr + i];
  out[((size_t)f * out_ns + s0 + s) * g.nr + i] = make_float2((float)v.x, (float)v.y);
}

// Largest eigenvalue of each Hhat(w) by power iteration in FP64 (one workgroup
// per frequency), Rayleigh quotient of the final vector.
__global__ void __launch_bounds__(256)
    k_power(Geometry g, const double2* __restrict__ hhat, double* __restrict__ eig, int iters) {
  extern __shared__ double2 sv[];  // v[n], y[n]
  __shared__ double red[256];
  const int f = blockIdx.x;
  const int n = g.nr;
  const double2* H = hhat + (size_t)f * n * n;
  double2* v = sv;
  double2* y = sv + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = make_double2(1.0 + 0.25 * sin(1.0 + i), 0.0);
  __syncthreads();
  double lam = 0.0;
  for (int it = 0; it <= iters; ++it) {
    double part = 0.0, rq = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double tr = 0.0, ti = 0.0;
      for (int j = 0; j < n; ++j) {
        double2 h = H[(size_t)i * n + j], x = v[j];
        tr += h.x * x.x - h.y * x.y;
        ti += h.x * x.y + h.y * x.x;
      }
      y[i] = make_double2(tr, ti);
      part += tr * tr + ti * ti;
      rq += v[i].x * tr + v[i].y * ti;  // Re(conj(v_i) y_i)
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    double ny = sqrt(red[0]);
    __syncthreads();
    red[threadIdx.x] = rq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    double vv_rq = red[0];
    __syncthreads();
    // normalise v's norm into the quotient
    double vn = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) vn += v[i].x * v[i].x + v[i].y * v[i].y;
    red[threadIdx.x] = vn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    lam = vv_rq / red[0];
    __syncthreads();
    if (ny == 0.0) break;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = make_double2(y[i].x / ny, y[i].y / ny);
    __syncthreads();
  }
  if (threadIdx.x == 0) eig[f] = lam;
}

}  // namespace

hipError_t launch_trsm(const Geometry& g, const float2* l32, const float2* rhs, int rhs_ld,
                       int rhs_off, float2* work, int work_ld, int work_off, int cnt, int mode,
                       double2* x64, hipStream_t st) {
  dim3 grid(cdiv(cnt, 64), g.nf);
  hipLaunchKernelGGL(k_trsm, grid, dim3(64), 0, st, g, l32, rhs, rhs_ld, rhs_off, work, work_ld,
                     work_off, cnt, mode, x64);
  return hipGetLastError();
}

hipError_t launch_residual(const Geometry& g, const double2* qhat, const float2* resid,
                           int resid_ns, int s0, int ns, const double2* x64, float2* r32,
                           hipStream_t st) {
  dim3 grid(cdiv(g.nr, 64), ns, g.nf);
  hipLaunchKernelGGL(k_residual, grid, dim3(64), 0, st, g, qhat, resid, resid_ns, s0, x64, r32);
  return hipGetLastError();
}

hipError_t launch_x_out(const Geometry& g, const double2* x64, int ns, int s0, float2* out,
                        int out_ns, hipStream_t st) {
  dim3 grid(cdiv(g.nr, 64), ns, g.nf);
  hipLaunchKernelGGL(k_x_out, grid, dim3(64), 0, st, g, x64, ns, s0, out, out_ns);
  return hipGetLastError();
}

hipError_t launch_power_iter(const Geometry& g, const double2* hhat, double* eig, int iters,
                             hipStream_t st) {
  size_t shmem = 2 * (size_t)g.nr * sizeof(double2);
  hipLaunchKernelGGL(k_power, dim3(g.nf), dim3(256), shmem, st, g, hhat, eig, iters);
  return hipGetLastError();
}

}  // namespace ehi
