// Multi-source deblurring delta d^e(w) = Qhat(w)^{-1} delta d(w).
//
// Paper: the block-diagonal frequency system is solved separately per frequency
// for every source with the stored blocks (frequency-domain inversion; the
// per-source step of the multiplier-based algorithm computes delta d^e in the
// frequency domain).  The factor L (complex64 copy) drives blocked forward and
// back substitution; in the split-BF16 precision mode two refinement steps
// compute the residual R - Qhat X in FP64 and correct X (accumulated in FP64).
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

// ---------------------------------------------------------------------------
// Blocked multi-source solves.  L is split into 32 x 32 blocks; the inverses of
// the diagonal blocks are formed once after the factorisation, so every block
// step of the forward solve  X_I = inv(L_II) (B_I - sum_{J<I} L_IJ X_J)  and of
// the back solve with L^H is a pair of small dense products over the sources of
// a tile, with no row-by-row dependency chain inside a block.

constexpr int kSb = 32;  // solve block

// inv[I] = inverse of the diagonal block L_II of a job's complex64 factor,
// computed in FP64 (rows past nr are padded with the identity).  One thread per
// column of the block; grid (blocks, jobs).
__global__ void __launch_bounds__(kSb) k_diag_inv(const FactorJob* __restrict__ jobs) {
  const FactorJob jb = jobs[blockIdx.y];
  const int I = blockIdx.x, j = threadIdx.x;
  const int n = jb.nr;
  if (I >= cdiv(n, kSb)) return;
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
  float2* out = jb.linv + (size_t)I * kSb * kSb;
  for (int r = 0; r < kSb; ++r) out[r * kSb + j] = make_float2((float)Y[r][j].x, (float)Y[r][j].y);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Workgroup of 256 threads = CT sources x RG row groups; thread (c, gq) owns,
// inside every 32-row block, rows gq*RPT .. gq*RPT + RPT - 1 of source column c.
template <int CT>
struct Tile {
  static constexpr int RG = 256 / CT;
  static constexpr int RPT = kSb / RG;
};

// In-place solve of L L^H x = b for the tile's columns held in xs[row][c].
template <int CT>
__device__ void tile_solve(const Geometry& g, const float2* __restrict__ L,
                           const float2* __restrict__ inv, float2 (*xs)[CT + 1], int c, int gq) {
  constexpr int RPT = Tile<CT>::RPT;
  const int n = g.nr;
  const int nb = cdiv(n, kSb);
  float2 t[RPT];
  // forward
  for (int I = 0; I < nb; ++I) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = I * kSb + gq * RPT + q;
      float2 acc = xs[r][c];
      if (r < n) {
        const float2* Lr = L + (size_t)r * n;
        for (int k = 0; k < I * kSb; ++k) {
          const float2 p = cmul(Lr[k], xs[k][c]);
          acc.x -= p.x;
          acc.y -= p.y;
        }
      }
      t[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) xs[I * kSb + gq * RPT + q][c] = t[q];
    __syncthreads();
    const float2* Ib = inv + (size_t)I * kSb * kSb;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rr = gq * RPT + q;
      float2 acc = make_float2(0.f, 0.f);
      for (int k = 0; k <= rr; ++k) {
        const float2 p = cmul(Ib[rr * kSb + k], xs[I * kSb + k][c]);
        acc.x += p.x;
        acc.y += p.y;
      }
      t[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) xs[I * kSb + gq * RPT + q][c] = t[q];
    __syncthreads();
  }
  // backward with L^H
  for (int I = nb - 1; I >= 0; --I) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = I * kSb + gq * RPT + q;
      float2 acc = xs[r][c];
      if (r < n) {
        for (int k = (I + 1) * kSb; k < n; ++k) {
          const float2 p = cmulc(L[(size_t)k * n + r], xs[k][c]);
          acc.x -= p.x;
          acc.y -= p.y;
        }
      }
      t[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) xs[I * kSb + gq * RPT + q][c] = t[q];
    __syncthreads();
    const float2* Ib = inv + (size_t)I * kSb * kSb;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rr = gq * RPT + q;
      float2 acc = make_float2(0.f, 0.f);
      for (int k = rr; k < kSb; ++k) {
        const float2 p = cmulc(Ib[k * kSb + rr], xs[I * kSb + k][c]);
        acc.x += p.x;
        acc.y += p.y;
      }
      t[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) xs[I * kSb + gq * RPT + q][c] = t[q];
    __syncthreads();
  }
}

// One (frequency, tile of CT sources): X = Qhat^{-1} R.  refine = 0: FP32
// solve only, written to out.  refine = 2: FP32 solve, then two steps of
// r = R - Qhat X in FP64, d = solve(r), X += d with X kept in FP64 (x64 scratch).
template <int CT>
__global__ void __launch_bounds__(256)
    k_apply(Geometry g, const float2* __restrict__ l32, const float2* __restrict__ inv,
            const double2* __restrict__ qhat, const float2* __restrict__ R, int rld, int s0, int cnt,
            int refine, double2* __restrict__ x64, float2* __restrict__ out) {
  extern __shared__ float2 xs_raw[];
  float2(*xs)[CT + 1] = reinterpret_cast<float2(*)[CT + 1]>(xs_raw);
  const int f = blockIdx.y;
  const int c = threadIdx.x % CT, gq = threadIdx.x / CT;
  const int sl = blockIdx.x * CT + c;  // source inside this call's chunk
  const bool sv = sl < cnt;
  const int n = g.nr;
  const int nb = cdiv(n, kSb);
  constexpr int RPT = Tile<CT>::RPT;
  const float2* L = l32 + (size_t)f * n * n;
  const float2* Iv = inv + (size_t)f * nb * kSb * kSb;
  const float2* Rc = R + ((size_t)f * rld + s0 + (sv ? sl : 0)) * n;
  double2* xc = x64 + ((size_t)f * g.max_ns + (sv ? sl : 0)) * n;
  // rows owned by this thread: I*32 + gq*RPT + q
  for (int I = 0; I < nb; ++I)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = I * kSb + gq * RPT + q;
      xs[r][c] = (sv && r < n) ? Rc[r] : make_float2(0.f, 0.f);
    }
  __syncthreads();
  tile_solve<CT>(g, L, Iv, xs, c, gq);
  if (refine > 0) {
    for (int I = 0; I < nb; ++I)
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = I * kSb + gq * RPT + q;
        if (sv && r < n) xc[r] = make_double2((double)xs[r][c].x, (double)xs[r][c].y);
      }
    __threadfence_block();
    __syncthreads();
    const double2* Q = qhat + (size_t)f * n * n;
    for (int it = 0; it < refine; ++it) {
      for (int I = 0; I < nb; ++I)
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = I * kSb + gq * RPT + q;
          float2 v = make_float2(0.f, 0.f);
          if (sv && r < n) {
            const double2* Qr = Q + (size_t)r * n;
            double tr = (double)Rc[r].x, ti = (double)Rc[r].y;
            for (int k = 0; k < n; ++k) {
              const double2 a = Qr[k], b = xc[k];
              tr -= a.x * b.x - a.y * b.y;
              ti -= a.x * b.y + a.y * b.x;
            }
            v = make_float2((float)tr, (float)ti);
          }
          xs[r][c] = v;
        }
      __syncthreads();
      tile_solve<CT>(g, L, Iv, xs, c, gq);
      for (int I = 0; I < nb; ++I)
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = I * kSb + gq * RPT + q;
          if (sv && r < n) {
            double2 o = xc[r];
            o.x += (double)xs[r][c].x;
            o.y += (double)xs[r][c].y;
            xc[r] = o;
          }
        }
      __threadfence_block();
      __syncthreads();
    }
  }
  float2* Oc = out + ((size_t)f * rld + s0 + (sv ? sl : 0)) * n;
  for (int I = 0; I < nb; ++I)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = I * kSb + gq * RPT + q;
      if (sv && r < n) Oc[r] = refine > 0 ? make_float2((float)xc[r].x, (float)xc[r].y) : xs[r][c];
    }
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

hipError_t launch_diag_inv_jobs(const FactorJob* jobs, int njobs, int max_nr, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_inv, dim3(cdiv(max_nr, kSb), njobs), dim3(kSb), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_apply(const Geometry& g, const float2* l32, const float2* inv,
                        const double2* qhat, const float2* R, int rld, int s0, int cnt, int refine,
                        double2* x64, float2* out, hipStream_t st) {
  const int npad = solve_blocks(g) * kSb;
#define EHI_APPLY(CTV)                                                                          \
  {                                                                                             \
    const size_t sh = (size_t)npad * ((CTV) + 1) * sizeof(float2);                              \
    hipLaunchKernelGGL(k_apply<CTV>, dim3(cdiv(cnt, CTV), g.nf), dim3(256), sh, st, g, l32, inv, \
                       qhat, R, rld, s0, cnt, refine, x64, out);                                 \
  }
  // dynamic LDS npad * (CT + 1) * 8 bytes: <= 64 KiB up to 224 / 448 rows
  if (npad <= 224) EHI_APPLY(32)
  else if (npad <= 448) EHI_APPLY(16)
  else {
    // once per process (thread-safe static initialisation)
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_apply<8>), hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (attr != hipSuccess) return attr;
    EHI_APPLY(8)
  }
#undef EHI_APPLY
  return hipGetLastError();
}

hipError_t launch_power_iter(const Geometry& g, const double2* hhat, double* eig, int iters,
                             hipStream_t st) {
  size_t shmem = 2 * (size_t)g.nr * sizeof(double2);
  hipLaunchKernelGGL(k_power, dim3(g.nf), dim3(256), shmem, st, g, hhat, eig, iters);
  return hipGetLastError();
}

}  // namespace ehi
