// Multi-source deblurring delta d^e(w) = Qhat(w)^{-1} delta d(w).
//
// Paper: the block-diagonal frequency system is solved separately per frequency
// for every source with the stored blocks (frequency-domain inversion; the
// per-source step of the multiplier-based algorithm computes delta d^e in the
// frequency domain).
//
// The two triangular solves with the Cholesky factor L are applied as products
// with M = L^{-1}: X = M^H (M R).  M is formed once per factorisation in FP64
// (block-column recursion below) and kept as a zero-padded complex64 matrix, so
// every solve is a dense batched product over (row tile, source tile,
// frequency) with no sequential dependency between rows.  In the split-BF16
// precision mode two refinement steps follow: r = R - Qhat X in FP64 (X kept in
// FP64), X += M^H (M r) in FP32.
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int kSb = 32;  // block of the triangular inversion

// ---------------------------------------------------------------------------
// M = L^{-1}, L padded to np = 32 * cdiv(nr, 32) rows with the identity
// (L_pad = diag(L, I), so M_pad = diag(M, I)).
//
// Pass 1 (k_diag_inv): D_I = inverse of the diagonal block L_II in FP64, one
// workgroup of 32 threads (one per column) per (block, job); written to the
// diagonal blocks of the job's FP64 scratch m64.
// Pass 2 (k_tri_inv_cols): block column J of M, one workgroup per (J, job):
// M_JJ = D_J and, for I = J+1, ..., M_IJ = -D_I sum_{K=J}^{I-1} L_IK M_KJ.
// Writes the complex64 copy (zeros above the diagonal) used by the solves.
__global__ void __launch_bounds__(kSb) k_diag_inv(const FactorJob* __restrict__ jobs) {
  const FactorJob jb = jobs[blockIdx.y];
  const int I = blockIdx.x, j = threadIdx.x;
  const int n = jb.nr;
  const int nb = cdiv(n, kSb);
  const int np = nb * kSb;
  if (I >= nb) return;
  const float2* l32 = jb.l32;
  __shared__ double2 Lb[kSb][kSb];
  for (int r = 0; r < kSb; ++r) {
    const int gr = I * kSb + r, gc = I * kSb + j;
    double2 v = make_double2(0.0, 0.0);
    if (gr < n && gc < n) {
      if (j <= r) {
        const float2 x = l32[(size_t)gr * n + gc];
        v = make_double2(x.x, x.y);
      }
    } else if (r == j) {
      v = make_double2(1.0, 0.0);
    }
    Lb[r][j] = v;
  }
  __shared__ double2 Y[kSb][kSb];  // Y[r][j]: column j of the inverse
  __syncthreads();
  // column j of the inverse: forward substitution of Lb y = e_j
  for (int r = 0; r < kSb; ++r) {
    double tr = (r == j) ? 1.0 : 0.0, ti = 0.0;
    for (int k = j; k < r; ++k) {
      const double2 l = Lb[r][k], y = Y[k][j];
      tr -= l.x * y.x - l.y * y.y;
      ti -= l.x * y.y + l.y * y.x;
    }
    const double d = Lb[r][r].x;  // real and positive
    Y[r][j] = (r < j) ? make_double2(0.0, 0.0) : make_double2(tr / d, ti / d);
  }
  double2* out = jb.m64 + ((size_t)I * kSb) * np + I * kSb;
  for (int r = 0; r < kSb; ++r) out[(size_t)r * np + j] = Y[r][j];
}

__device__ __forceinline__ double2 zmac(double2 acc, double2 a, double2 b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
  return acc;
}

__global__ void __launch_bounds__(256) k_tri_inv_cols(const FactorJob* __restrict__ jobs) {
  const FactorJob jb = jobs[blockIdx.y];
  const int J = blockIdx.x;
  const int n = jb.nr;
  const int nb = cdiv(n, kSb);
  const int np = nb * kSb;
  if (J >= nb) return;
  __shared__ double2 Ls[kSb][kSb + 1];
  __shared__ double2 Xs[kSb][kSb + 1];
  __shared__ double2 Ts[kSb][kSb + 1];
  const int tid = threadIdx.x;
  const int r = tid >> 3, c0 = (tid & 7) * 4;  // this thread: row r, columns c0 .. c0 + 3
  double2* m64 = jb.m64;
  float2* m32 = jb.m32;
  auto put32 = [&](int I, int rr, int cc, double2 v) {
    m32[(size_t)(I * kSb + rr) * np + J * kSb + cc] = make_float2((float)v.x, (float)v.y);
  };
  // blocks above the diagonal are zero; the diagonal block is D_J
  for (int I = 0; I < J; ++I)
#pragma unroll
    for (int q = 0; q < 4; ++q) put32(I, r, c0 + q, make_double2(0.0, 0.0));
#pragma unroll
  for (int q = 0; q < 4; ++q) put32(J, r, c0 + q, m64[(size_t)(J * kSb + r) * np + J * kSb + c0 + q]);
  for (int I = J + 1; I < nb; ++I) {
    double2 t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = make_double2(0.0, 0.0);
    for (int K = J; K < I; ++K) {
      __syncthreads();
      // L_IK (zero outside the nr x nr factor) and M_KJ
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = I * kSb + r, gc = K * kSb + c0 + q;
        double2 v = make_double2(0.0, 0.0);
        if (gr < n && gc < n) {
          const float2 x = jb.l32[(size_t)gr * n + gc];
          v = make_double2(x.x, x.y);
        }
        Ls[r][c0 + q] = v;
        Xs[r][c0 + q] = m64[(size_t)(K * kSb + r) * np + J * kSb + c0 + q];
      }
      __syncthreads();
      for (int k = 0; k < kSb; ++k) {
        const double2 a = Ls[r][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) t[q] = zmac(t[q], a, Xs[k][c0 + q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Ts[r][c0 + q] = t[q];
      Ls[r][c0 + q] = m64[(size_t)(I * kSb + r) * np + I * kSb + c0 + q];  // D_I
    }
    __syncthreads();
    double2 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = make_double2(0.0, 0.0);
    for (int k = 0; k < kSb; ++k) {
      const double2 a = Ls[r][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = zmac(x[q], a, Ts[k][c0 + q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = make_double2(-x[q].x, -x[q].y);
      m64[(size_t)(I * kSb + r) * np + J * kSb + c0 + q] = v;
      put32(I, r, c0 + q, v);
    }
    // the next block reads this one back through global memory
    __threadfence_block();
  }
}

// ---------------------------------------------------------------------------
// Batched complex products for the solves, one frequency per blockIdx.z:
//   C(i, j) = sum_k op(A)(i, k) B(k, j),  i < n (receivers), j < ns (sources)
// A: MODE 0: Qhat (FP64, n x n, row-major); MODE 1: M (lower, np x np);
// MODE 2: M^H, i.e. A(i, k) = conj(M(k, i)).  Tiles of M that are zero by
// triangularity are skipped.  B(k, j) = Bm[j * ldb + k] (source-major, as the
// residuals are stored), read as zero for k >= n.
// Workgroup: a 64 x 64 tile of C, each thread a 4 x 4 register tile (rows
// 4 ty + r, columns 4 tx + c); K in stages of 16 through LDS.  The LDS tiles
// keep the register-tile index outermost (entry r * 16 + ty, c * 16 + tx), so
// the lanes of a half-wave read consecutive elements.
enum { kEpiStore = 0, kEpiResid = 1, kEpiX64Set = 2, kEpiX64Add = 3, kEpiOut = 4 };

struct GemmArgs {
  const void* A;    // float2 or double2
  size_t sA;        // per-frequency stride (elements)
  int lda;
  const void* B;    // float2 (FP32) or double2 (FP64)
  size_t sB;
  int ldb;
  int n, ns;        // rows of C (receivers), columns (sources)
  int kmax;         // K extent (n for Qhat, np for M; B rows >= n read as zero)
  float2* C;        // float2 outputs (kEpiStore, kEpiResid, kEpiOut)
  size_t sC;
  int ldc;
  const float2* R;  // residuals (kEpiResid)
  size_t sR;
  int ldr;
  double2* X;       // FP64 iterate (kEpiX64Set/Add/Out)
  size_t sX;
  int ldx;
};

template <typename T> struct Cx;
template <> struct Cx<float> { typedef float2 t; };
template <> struct Cx<double> { typedef double2 t; };

constexpr int kGm = 64, kGn = 64, kGk = 16;

template <typename T, int MODE, int EPI>
__global__ void __launch_bounds__(256) k_cgemm(GemmArgs a) {
  typedef typename Cx<T>::t C2;
  __shared__ C2 As[kGk][kGm];
  __shared__ C2 Bs[kGk][kGn];
  const int f = blockIdx.z;
  const int i0 = blockIdx.y * kGm, j0 = blockIdx.x * kGn;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const C2* A = static_cast<const C2*>(a.A) + (size_t)f * a.sA;
  const C2* B = static_cast<const C2*>(a.B) + (size_t)f * a.sB;
  C2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = C2{0, 0};
  int kbeg = 0, kend = min(a.kmax, a.n);
  if (MODE == 1) kend = min(kend, i0 + kGm);             // M(i, k) = 0 for k > i
  if (MODE == 2) kbeg = i0 / kGk * kGk;                  // conj(M(k, i)) = 0 for k < i
  for (int k0 = kbeg; k0 < kend; k0 += kGk) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if (MODE == 2) {
        const int kk = e / kGm, ii = e % kGm;          // contiguous along i
        const int gk = k0 + kk, gi = i0 + ii;
        C2 v = C2{0, 0};
        if (gk < kend && gi < a.kmax) {
          const C2 m = A[(size_t)gk * a.lda + gi];
          v = C2{m.x, -m.y};
        }
        As[kk][(ii & 3) * 16 + (ii >> 2)] = v;
      } else {
        const int ii = e / kGk, kk = e % kGk;          // contiguous along k
        const int gk = k0 + kk, gi = i0 + ii;
        As[kk][(ii & 3) * 16 + (ii >> 2)] = (gk < kend && gi < a.kmax) ? A[(size_t)gi * a.lda + gk] : C2{0, 0};
      }
      const int jj = e / kGk, kk = e % kGk;
      const int gk = k0 + kk, gj = j0 + jj;
      Bs[kk][(jj & 3) * 16 + (jj >> 2)] = (gk < kend && gj < a.ns) ? B[(size_t)gj * a.ldb + gk] : C2{0, 0};
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kGk; ++kk) {
      C2 av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[kk][r * 16 + ty];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][c * 16 + tx];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[r][c].x += av[r].x * bv[c].x - av[r].y * bv[c].y;
          acc[r][c].y += av[r].x * bv[c].y + av[r].y * bv[c].x;
        }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + tx * 4 + c;
    if (j >= a.ns) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + ty * 4 + r;
      if (i >= a.n) continue;
      const C2 v = acc[r][c];
      if (EPI == kEpiStore) {
        a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] = make_float2((float)v.x, (float)v.y);
      } else if (EPI == kEpiResid) {
        const float2 rr = a.R[(size_t)f * a.sR + (size_t)j * a.ldr + i];
        a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] =
            make_float2((float)((double)rr.x - (double)v.x), (float)((double)rr.y - (double)v.y));
      } else {
        double2* xp = a.X + (size_t)f * a.sX + (size_t)j * a.ldx + i;
        if (EPI == kEpiX64Set) {
          *xp = make_double2((double)v.x, (double)v.y);
        } else if (EPI == kEpiX64Add) {
          double2 o = *xp;
          o.x += (double)v.x;
          o.y += (double)v.y;
          *xp = o;
        } else {  // kEpiOut
          const double2 o = *xp;
          a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] =
              make_float2((float)(o.x + (double)v.x), (float)(o.y + (double)v.y));
        }
      }
    }
  }
}

template <typename T, int MODE, int EPI>
hipError_t run_gemm(const GemmArgs& a, int nf, hipStream_t st) {
  dim3 grid(cdiv(a.ns, kGn), cdiv(a.n, kGm), nf);
  hipLaunchKernelGGL((k_cgemm<T, MODE, EPI>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
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

int solve_blocks(const Geometry& g) { return cdiv(g.nr, kSb); }

hipError_t launch_minv_jobs(const FactorJob* jobs, int njobs, int max_nr, hipStream_t st) {
  const int nb = cdiv(max_nr, kSb);
  hipLaunchKernelGGL(k_diag_inv, dim3(nb, njobs), dim3(kSb), 0, st, jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_inv_cols, dim3(nb, njobs), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_apply(const Geometry& g, const float2* m32, const double2* qhat, const float2* R,
                        int rld, int s0, int cnt, int refine, float2* y32, float2* r32,
                        double2* x64, float2* out, hipStream_t st) {
  const int n = g.nr, np = solve_blocks(g) * kSb;
  const size_t nn = (size_t)n * n, npp = (size_t)np * np;
  const size_t sv = (size_t)g.max_ns * n;  // scratch per frequency
  GemmArgs a{};
  a.n = n;
  a.ns = cnt;
  // Y = M R
  a.A = m32; a.sA = npp; a.lda = np; a.kmax = np;
  a.B = R + (size_t)s0 * n; a.sB = (size_t)rld * n; a.ldb = n;
  a.C = y32; a.sC = sv; a.ldc = n;
  hipError_t e = run_gemm<float, 1, kEpiStore>(a, g.nf, st);
  if (e != hipSuccess) return e;
  // X = M^H Y
  a.B = y32; a.sB = sv; a.ldb = n;
  if (refine == 0) {
    a.C = out + (size_t)s0 * n; a.sC = (size_t)rld * n; a.ldc = n;
    return run_gemm<float, 2, kEpiStore>(a, g.nf, st);
  }
  a.X = x64; a.sX = sv; a.ldx = n;
  e = run_gemm<float, 2, kEpiX64Set>(a, g.nf, st);
  if (e != hipSuccess) return e;
  for (int it = 0; it < refine; ++it) {
    // r = R - Qhat X (FP64)
    GemmArgs q = a;
    q.A = qhat; q.sA = nn; q.lda = n; q.kmax = n;
    q.B = x64; q.sB = sv; q.ldb = n;
    q.R = R + (size_t)s0 * n; q.sR = (size_t)rld * n; q.ldr = n;
    q.C = r32; q.sC = sv; q.ldc = n;
    e = run_gemm<double, 0, kEpiResid>(q, g.nf, st);
    if (e != hipSuccess) return e;
    // Y = M r
    GemmArgs y = a;
    y.A = m32; y.sA = npp; y.lda = np; y.kmax = np;
    y.B = r32; y.sB = sv; y.ldb = n;
    y.C = y32; y.sC = sv; y.ldc = n;
    e = run_gemm<float, 1, kEpiStore>(y, g.nf, st);
    if (e != hipSuccess) return e;
    // X += M^H Y (the last step writes the complex64 result)
    GemmArgs x = y;
    x.B = y32;
    if (it + 1 < refine) {
      e = run_gemm<float, 2, kEpiX64Add>(x, g.nf, st);
    } else {
      x.C = out + (size_t)s0 * n; x.sC = (size_t)rld * n; x.ldc = n;
      e = run_gemm<float, 2, kEpiOut>(x, g.nf, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_power_iter(const Geometry& g, const double2* hhat, double* eig, int iters,
                             hipStream_t st) {
  size_t shmem = 2 * (size_t)g.nr * sizeof(double2);
  hipLaunchKernelGGL(k_power, dim3(g.nf), dim3(256), shmem, st, g, hhat, eig, iters);
  return hipGetLastError();
}

}  // namespace ehi
