// Forward modelling on the survey's medium and the steps either side of the
// deblur.
//
// Paper: the forward operator S = P A(m)^{-1} and the extended source
// delta b = S^T delta d^e (Theory; multiplier-based extended FWI algorithm);
// the data residuals enter the frequency-domain inversion through a transform
// of length 2 Nt and the multipliers leave it through the inverse transform
// cropped to the record (frequency-domain inversion); the Hessian accuracy
// test (numerical examples) compares d - P u^e with the data.
//
// S here maps a source field on the stride subgrid (one value per subgrid
// cell and step) to the receiver traces; its transpose is a forward run in
// reversed time with the traces injected at the receivers, read back on the
// subgrid.  Both step one time level per launch over a batch of fields (no
// temporal blocking: these runs are not on the Hessian's critical path), with
// the same increment form and coefficients as the Green-function march:
//   w <- (b/a) w + ca (16 (u_{z-1} + u_{z+1} + u_{x-1} + u_{x+1})
//                      - (u_{z-2} + u_{z+2} + u_{x-2} + u_{x+2}) - 60 u + 12 h^2 f)
//   u <- u + w
// (ca = kappa / (12 h^2 a), so the source term is kappa f / a).
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int kStepCols = 256;

// One time level of nb_now fields; w is updated in place, u goes from uin to
// uout.  src (may be NULL): subgrid source of this step, field k at
// src + k * src_field, [nzs][nxs].  Ghost rings of uin/uout stay zero.
__global__ void __launch_bounds__(kStepCols)
    k_fd_step(Geometry g, const float* __restrict__ ca, const float* __restrict__ bd,
              const float* __restrict__ uin, float* __restrict__ uout, float* __restrict__ w,
              const float* __restrict__ src, size_t src_field, float src_scale) {
  const int ix = blockIdx.x * kStepCols + threadIdx.x;
  const int iz = blockIdx.y;
  const int k = blockIdx.z;
  if (ix >= g.X) return;
  const int Xp = g.Xp;
  const size_t o = (size_t)(iz + kGhost) * Xp + ix + kGhost;
  const size_t fo = (size_t)k * g.plane() + o;
  const float* u = uin + (size_t)k * g.plane();
  const float cen = u[o];
  const float n1 = (u[o - Xp] + u[o + Xp]) + (u[o - 1] + u[o + 1]);
  const float n2 = (u[o - 2 * Xp] + u[o + 2 * Xp]) + (u[o - 2] + u[o + 2]);
  float lap = 16.f * n1 - n2 - 60.f * cen;
  if (src) {
    const int jz = iz - g.nb, jx = ix - g.nb;
    if (jz >= 0 && jz < g.nz && jx >= 0 && jx < g.nx && (jz & (g.stride - 1)) == 0 &&
        (jx & (g.stride - 1)) == 0)
      lap += src_scale * src[(size_t)k * src_field + (size_t)(jz >> g.sshift) * g.nxs + (jx >> g.sshift)];
  }
  const int dz = max(max(g.nb - iz, iz - (g.nb + g.nz - 1)), 0);
  const int dx = max(max(g.nb - ix, ix - (g.nb + g.nx - 1)), 0);
  const float wn = bd[max(dz, dx)] * w[fo] + ca[o] * lap;
  w[fo] = wn;
  uout[fo] = cen + wn;
}

// Point sources at the receivers, added after the step (the update is linear
// in the source): w and u of receiver r's cell gain ca 12 h^2 amp, amp =
// data[k][r][col] for field k.  Atomic, so receivers may share a cell.
__global__ void k_inject_points(Geometry g, const float* __restrict__ ca, const int32_t* __restrict__ rec,
                                const float* __restrict__ data, size_t data_field, int col,
                                float src_scale, float* __restrict__ uout, float* __restrict__ w) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= g.nr) return;
  const size_t o = (size_t)(rec[r] + g.nb + kGhost) * g.Xp + (rec[g.nr + r] + g.nb + kGhost);
  const float v = src_scale * ca[o] * data[(size_t)k * data_field + (size_t)r * g.nt + col];
  atomicAdd(&w[(size_t)k * g.plane() + o], v);
  atomicAdd(&uout[(size_t)k * g.plane() + o], v);
}

// dst[k][slot][x'] = u_k on the subgrid (field k at dst + k * dst_field).
__global__ void k_record_subgrid(Geometry g, const float* __restrict__ u, float* __restrict__ dst,
                                 size_t dst_field, int slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= g.nsub) return;
  const int sz = i / g.nxs, sx = i % g.nxs;
  const size_t o = (size_t)((sz << g.sshift) + g.nb + kGhost) * g.Xp + (sx << g.sshift) + g.nb + kGhost;
  dst[(size_t)k * dst_field + (size_t)slot * g.nsub + i] = u[(size_t)k * g.plane() + o];
}

// d[k][r][col] = u_k at receiver r.
__global__ void k_record_points(Geometry g, const int32_t* __restrict__ rec, const float* __restrict__ u,
                                float* __restrict__ d, size_t d_field, int col) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= g.nr) return;
  const size_t o = (size_t)(rec[r] + g.nb + kGhost) * g.Xp + (rec[g.nr + r] + g.nb + kGhost);
  d[(size_t)k * d_field + (size_t)r * g.nt + col] = u[(size_t)k * g.plane() + o];
}

// ---- residual spectra and the inverse transform ------------------------------

constexpr int kTq = 64;  // rows (source, receiver) per workgroup
constexpr int kTn = 64;  // samples per LDS stage
constexpr int kMaxNf = 64;

// R[f][q] = sum_{n=1}^{nt} dres[q][n-1] tw[n-1][f], q = source * nr + receiver.
// A workgroup owns 64 rows; thread (row tid % 64, group tid / 64) sums the
// frequencies f = group, group + 4, ... in FP64.  Samples and twiddles pass
// through LDS in stages of 64 samples.
__global__ void __launch_bounds__(256)
    k_resid_spectra(int nt, int nf, int nq, const float* __restrict__ dres, const float2* __restrict__ tw,
                    float2* __restrict__ R) {
  __shared__ float Ds[kTq][kTn + 1];
  __shared__ float2 Ts[kTn][kMaxNf];
  const int q0 = blockIdx.x * kTq;
  const int tid = threadIdx.x;
  const int qi = tid & 63, fg = tid >> 6;
  double2 acc[kMaxNf / 4];
#pragma unroll
  for (int j = 0; j < kMaxNf / 4; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int n0 = 0; n0 < nt; n0 += kTn) {
    __syncthreads();
    for (int e = tid; e < kTq * kTn; e += 256) {
      const int a = e / kTn, b = e % kTn;  // row, sample: consecutive lanes read consecutive samples
      Ds[a][b] = (q0 + a < nq && n0 + b < nt) ? dres[(size_t)(q0 + a) * nt + n0 + b] : 0.f;
    }
    for (int e = tid; e < kTn * nf; e += 256) {
      const int b = e / nf, f = e % nf;
      Ts[b][f] = n0 + b < nt ? tw[(size_t)(n0 + b) * nf + f] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int b = 0; b < kTn; ++b) {
      const double x = (double)Ds[qi][b];
#pragma unroll
      for (int j = 0; j < kMaxNf / 4; ++j) {
        const int f = fg + 4 * j;
        if (f < nf) {
          const float2 t = Ts[b][f];
          acc[j].x += x * (double)t.x;
          acc[j].y += x * (double)t.y;
        }
      }
    }
  }
  if (q0 + qi >= nq) return;
#pragma unroll
  for (int j = 0; j < kMaxNf / 4; ++j) {
    const int f = fg + 4 * j;
    if (f < nf) R[(size_t)f * nq + q0 + qi] = make_float2((float)acc[j].x, (float)acc[j].y);
  }
}

// x[q][n-1] = sum_f c_f Re(X[f][q] conj(tw[n-1][f])), n = 1..nt: the inverse
// 2nt-point transform of bins 0..nt cropped to the record (conj(tw) =
// exp(+i w n dt)); c_f = 1/(2nt) for bins 0 and nt (bit f of edge set),
// 2/(2nt) otherwise.  A workgroup owns 64 rows x 64 samples; thread (sample
// tid % 64, group tid / 64) sums 16 rows in FP64.  LDS: X by frequency and row,
// twiddles by frequency and sample (lanes read consecutive samples).
__global__ void __launch_bounds__(256)
    k_to_time(int nt, int nf, int nq, const float2* __restrict__ X, const float2* __restrict__ tw,
              unsigned long long edge, double inv2nt, float* __restrict__ x) {
  __shared__ float2 Xs[kMaxNf][kTq];
  __shared__ float2 Ts[kMaxNf][kTn];
  const int q0 = blockIdx.x * kTq, n0 = blockIdx.y * kTn;
  const int tid = threadIdx.x;
  for (int e = tid; e < nf * kTq; e += 256) {
    const int f = e / kTq, a = e % kTq;
    Xs[f][a] = q0 + a < nq ? X[(size_t)f * nq + q0 + a] : make_float2(0.f, 0.f);
  }
  for (int e = tid; e < kTn * nf; e += 256) {
    const int b = e / nf, f = e % nf;
    Ts[f][b] = n0 + b < nt ? tw[(size_t)(n0 + b) * nf + f] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int b = tid & 63, qg = tid >> 6;
  double acc[kTq / 4];
#pragma unroll
  for (int j = 0; j < kTq / 4; ++j) acc[j] = 0.0;
  for (int f = 0; f < nf; ++f) {
    const float2 t = Ts[f][b];
    const double c = ((edge >> f) & 1ull) ? inv2nt : 2.0 * inv2nt;
    const double tr = c * (double)t.x, ti = c * (double)t.y;
#pragma unroll
    for (int j = 0; j < kTq / 4; ++j) {
      const float2 v = Xs[f][qg * (kTq / 4) + j];
      acc[j] += (double)v.x * tr + (double)v.y * ti;
    }
  }
  if (n0 + b >= nt) return;
#pragma unroll
  for (int j = 0; j < kTq / 4; ++j) {
    const int q = q0 + qg * (kTq / 4) + j;
    if (q < nq) x[(size_t)q * nt + n0 + b] = (float)acc[j];
  }
}

// err = dd - pred per source (len values each) and relerr[s] = sum err^2 /
// sum obs^2 in FP64; one workgroup per source.
__global__ void __launch_bounds__(256)
    k_misfit(const float* __restrict__ dd, const float* __restrict__ pred, const float* __restrict__ obs,
             size_t len, float* __restrict__ err, double* __restrict__ relerr) {
  __shared__ double se[256], so[256];
  const size_t base = (size_t)blockIdx.x * len;
  double e2 = 0.0, o2 = 0.0;
  for (size_t i = threadIdx.x; i < len; i += 256) {
    const float e = dd[base + i] - pred[base + i];
    if (err) err[base + i] = e;
    const double o = (double)obs[base + i];
    e2 += (double)e * (double)e;
    o2 += o * o;
  }
  se[threadIdx.x] = e2;
  so[threadIdx.x] = o2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      se[threadIdx.x] += se[threadIdx.x + h];
      so[threadIdx.x] += so[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) relerr[blockIdx.x] = se[0] / so[0];
}

// ---- conjugate gradients on Q x = dd, Q = S S^T + mu I (the Krylov baseline) --
// Vectors are float32 records [ns][len]; scalars per record are FP64 device
// arrays.  One workgroup per record, a fixed reduction order (deterministic).
constexpr int kCgThreads = 1024;

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kCgThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// x = 0, r = p = dd, rr = r.r
__global__ void __launch_bounds__(kCgThreads)
    k_cg_init(const float* __restrict__ dd, float* __restrict__ x, float* __restrict__ r,
              float* __restrict__ p, size_t len, double* __restrict__ rr) {
  __shared__ double red[kCgThreads];
  const size_t base = (size_t)blockIdx.x * len;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < len; i += kCgThreads) {
    const float v = dd[base + i];
    x[base + i] = 0.f;
    r[base + i] = v;
    p[base + i] = v;
    acc += (double)v * (double)v;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) rr[blockIdx.x] = t;
}

// Ap += mu p (Ap holds S S^T p on entry), pAp = p.Ap
__global__ void __launch_bounds__(kCgThreads)
    k_cg_shift_dot(float* __restrict__ Ap, const float* __restrict__ p, float mu, size_t len,
                   double* __restrict__ pAp) {
  __shared__ double red[kCgThreads];
  const size_t base = (size_t)blockIdx.x * len;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < len; i += kCgThreads) {
    const float pv = p[base + i];
    const float a = fmaf(mu, pv, Ap[base + i]);
    Ap[base + i] = a;
    acc += (double)pv * (double)a;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) pAp[blockIdx.x] = t;
}

// alpha = rr / pAp; x += alpha p; r -= alpha Ap; rr_new = r.r; fit = |r + mu x|^2
// (dd - S S^T x = r + mu x: the accuracy test's misfit of the current iterate)
__global__ void __launch_bounds__(kCgThreads)
    k_cg_update(float* __restrict__ x, float* __restrict__ r, const float* __restrict__ p,
                const float* __restrict__ Ap, const double* __restrict__ rr, const double* __restrict__ pAp,
                float mu, size_t len, double* __restrict__ rr_new, double* __restrict__ fit) {
  __shared__ double red[kCgThreads];
  const size_t base = (size_t)blockIdx.x * len;
  const double den = pAp[blockIdx.x];
  const float alpha = den > 0.0 ? (float)(rr[blockIdx.x] / den) : 0.f;
  double a2 = 0.0, f2 = 0.0;
  for (size_t i = threadIdx.x; i < len; i += kCgThreads) {
    const float xv = fmaf(alpha, p[base + i], x[base + i]);
    const float rv = fmaf(-alpha, Ap[base + i], r[base + i]);
    x[base + i] = xv;
    r[base + i] = rv;
    a2 += (double)rv * (double)rv;
    const double e = (double)rv + (double)mu * (double)xv;
    f2 += e * e;
  }
  const double t1 = block_sum(a2, red);
  const double t2 = block_sum(f2, red);
  if (threadIdx.x == 0) {
    rr_new[blockIdx.x] = t1;
    fit[blockIdx.x] = t2;
  }
}

// p = r + (rr_new / rr) p
__global__ void __launch_bounds__(kCgThreads)
    k_cg_direction(float* __restrict__ p, const float* __restrict__ r, const double* __restrict__ rr_new,
                   const double* __restrict__ rr, size_t len) {
  const size_t base = (size_t)blockIdx.x * len;
  const double den = rr[blockIdx.x];
  const float beta = den > 0.0 ? (float)(rr_new[blockIdx.x] / den) : 0.f;
  for (size_t i = threadIdx.x; i < len; i += kCgThreads) p[base + i] = fmaf(beta, p[base + i], r[base + i]);
}

// ---- block dot products and linear combinations (the GMRES basis) ---------
// Vector j of record s at v + j * vstride + s * len.

// out[s][j] = V_j[s] . w[s] (FP64), one workgroup per (j, s)
__global__ void __launch_bounds__(256)
    k_mdot(const float* __restrict__ v, size_t vstride, int nvec, const float* __restrict__ w, size_t len,
           double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x, sidx = blockIdx.y;
  const float* a = v + (size_t)j * vstride + (size_t)sidx * len;
  const float* b = w + (size_t)sidx * len;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < len; i += 256) acc += (double)a[i] * (double)b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)sidx * nvec + j] = red[0];
}

// dst[s][i] = beta dst[s][i] + sum_j coef[s][j] V_j[s][i] (FP64 sum)
__global__ void __launch_bounds__(256)
    k_combine(const float* __restrict__ v, size_t vstride, int nvec, const double* __restrict__ coef,
              size_t len, double beta, float* __restrict__ dst) {
  __shared__ double c[1024];
  const int sidx = blockIdx.y;
  for (int j = threadIdx.x; j < nvec; j += 256) c[j] = coef[(size_t)sidx * nvec + j];
  __syncthreads();
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  float* d = dst + (size_t)sidx * len;
  double acc = beta != 0.0 ? beta * (double)d[i] : 0.0;
  const float* a = v + (size_t)sidx * len + i;
  for (int j = 0; j < nvec; ++j) acc += c[j] * (double)a[(size_t)j * vstride];
  d[i] = (float)acc;
}

}  // namespace

hipError_t launch_mdot(const float* v, size_t vstride, int nvec, const float* w, int ns, size_t len,
                       double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot, dim3(nvec, ns), dim3(256), 0, st, v, vstride, nvec, w, len, out);
  return hipGetLastError();
}

hipError_t launch_combine(const float* v, size_t vstride, int nvec, const double* coef, int ns, size_t len,
                          double beta, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((len + 255) / 256), ns), dim3(256), 0, st, v, vstride, nvec,
                     coef, len, beta, dst);
  return hipGetLastError();
}

hipError_t launch_cg_init(const float* dd, float* x, float* r, float* p, int ns, size_t len, double* rr,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init, dim3(ns), dim3(kCgThreads), 0, st, dd, x, r, p, len, rr);
  return hipGetLastError();
}

hipError_t launch_cg_shift_dot(float* Ap, const float* p, float mu, int ns, size_t len, double* pAp,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_cg_shift_dot, dim3(ns), dim3(kCgThreads), 0, st, Ap, p, mu, len, pAp);
  return hipGetLastError();
}

hipError_t launch_cg_update(float* x, float* r, const float* p, const float* Ap, const double* rr,
                            const double* pAp, float mu, int ns, size_t len, double* rr_new, double* fit,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(ns), dim3(kCgThreads), 0, st, x, r, p, Ap, rr, pAp, mu, len, rr_new,
                     fit);
  return hipGetLastError();
}

hipError_t launch_cg_direction(float* p, const float* r, const double* rr_new, const double* rr, int ns,
                               size_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_direction, dim3(ns), dim3(kCgThreads), 0, st, p, r, rr_new, rr, len);
  return hipGetLastError();
}

hipError_t launch_fd_step(const Geometry& g, const float* ca, const float* bd, const float* uin,
                          float* uout, float* w, int nb_now, const float* src, size_t src_field,
                          hipStream_t st) {
  const float scale = (float)(12.0 * g.h * g.h);
  hipLaunchKernelGGL(k_fd_step, dim3(cdiv(g.X, kStepCols), g.Z, nb_now), dim3(kStepCols), 0, st, g, ca,
                     bd, uin, uout, w, src, src_field, scale);
  return hipGetLastError();
}

hipError_t launch_inject_points(const Geometry& g, const float* ca, const int32_t* rec, const float* data,
                                size_t data_field, int col, int nb_now, float* uout, float* w,
                                hipStream_t st) {
  const float scale = (float)(12.0 * g.h * g.h);
  hipLaunchKernelGGL(k_inject_points, dim3(cdiv(g.nr, 64), nb_now), dim3(64), 0, st, g, ca, rec, data,
                     data_field, col, scale, uout, w);
  return hipGetLastError();
}

hipError_t launch_record_subgrid(const Geometry& g, const float* u, float* dst, size_t dst_field, int slot,
                                 int nb_now, hipStream_t st) {
  hipLaunchKernelGGL(k_record_subgrid, dim3(cdiv(g.nsub, 256), nb_now), dim3(256), 0, st, g, u, dst,
                     dst_field, slot);
  return hipGetLastError();
}

hipError_t launch_record_points(const Geometry& g, const int32_t* rec, const float* u, float* d,
                                size_t d_field, int col, int nb_now, hipStream_t st) {
  hipLaunchKernelGGL(k_record_points, dim3(cdiv(g.nr, 64), nb_now), dim3(64), 0, st, g, rec, u, d, d_field,
                     col);
  return hipGetLastError();
}

hipError_t launch_resid_spectra(const Geometry& g, const float* dres, int nq, const float2* tw, float2* R,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_resid_spectra, dim3(cdiv(nq, kTq)), dim3(256), 0, st, g.nt, g.nf, nq, dres, tw, R);
  return hipGetLastError();
}

hipError_t launch_to_time(const Geometry& g, const float2* X, int nq, const float2* tw,
                          unsigned long long edge_bins, float* x, hipStream_t st) {
  hipLaunchKernelGGL(k_to_time, dim3(cdiv(nq, kTq), cdiv(g.nt, kTn)), dim3(256), 0, st, g.nt, g.nf, nq, X,
                     tw, edge_bins, 1.0 / (2.0 * g.nt), x);
  return hipGetLastError();
}

hipError_t launch_misfit(const float* dd, const float* pred, const float* obs, int ns, size_t len,
                         float* err, double* relerr, hipStream_t st) {
  hipLaunchKernelGGL(k_misfit, dim3(ns), dim3(256), 0, st, dd, pred, obs, len, err, relerr);
  return hipGetLastError();
}

}  // namespace ehi
