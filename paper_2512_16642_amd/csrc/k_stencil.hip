// Green-function time stepping and the DFT accumulated during the time loop.
//
// Paper: the Green function of receiver j is the wavefield of a Dirac source at
// the receiver (Direct Hessian-inverse computation, block equation of the
// Hessian); Nr PDE solves build the Hessian (computational cost section).  The
// Fourier representation of each Green function at the needed frequencies
// (Fourier-domain Hessian) is accumulated while stepping, so the time samples
// never leave a short staging window (the discussion proposes on-the-fly
// computation to avoid storing the wavefields).
//
// Time stepping: k_march advances T time levels per launch.  A workgroup owns
// a band of kBand columns of one receiver's grid (overlapping its neighbours by
// 2T columns on each side, the halo the T steps consume) and marches down the
// rows.  Each thread owns one column and keeps, for every level, a window of
// five rows of u and a three-row delay line of w in registers; level t at row q
// is computed as soon as level t-1 has produced row q+2, so the levels form a
// pipeline skewed by two rows.  x-neighbours come from one LDS row per level
// (double-buffered, one barrier per marched row).  HBM sees each cell of u and
// w read once and written once per T steps.
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int kBand = 256;  // columns per workgroup (one per thread)

template <int N>
__device__ __forceinline__ void push(float (&a)[N], float v) {
#pragma unroll
  for (int i = 0; i < N - 1; ++i) a[i] = a[i + 1];
  a[N - 1] = v;
}

// Increment-form recurrence (per cell, FP32):
//   w <- ba * w + ca * (16 (u_{z-1} + u_{z+1} + u_{x-1} + u_{x+1})
//                        - (u_{z-2} + u_{z+2} + u_{x-2} + u_{x+2}) - 60 u)
//   u <- u + w
// ca = kappa / (12 h^2 a), ba = b / a (FP64-rounded coefficients).
//
// Inputs: level-0 fields uin, win (sample n_in); outputs: level-T fields uout,
// wout.  Levels beyond nlev pass their input through unchanged, so a launch
// can advance fewer than T steps.  Level t's sample (n_in + t) is written to
// staging slot slot0 + t - 1 on the stride subgrid.
template <int T>
__global__ void __launch_bounds__(kBand)
    k_march(Geometry g, const float* __restrict__ ca, const float* __restrict__ ba,
            const float* __restrict__ uin, const float* __restrict__ win, float* __restrict__ uout,
            float* __restrict__ wout, float* __restrict__ stage, int slot0, int nlev) {
  constexpr int B = kBand - 4 * T;  // output columns per band
  __shared__ float lds[2][T][kBand + 4];
  const int tid = threadIdx.x;
  const int r = blockIdx.y;
  const int x0 = blockIdx.x * B - 2 * T;  // padded-grid column of thread 0
  const int c = x0 + tid;
  const bool colv = (c >= 0 && c < g.X);
  const bool own = (tid >= 2 * T && tid < kBand - 2 * T && colv);
  const int P = g.Xp;
  const size_t plane = g.plane();
  const float* ui = uin + (size_t)r * plane;
  const float* wi = win + (size_t)r * plane;
  float* uo = uout + (size_t)r * plane;
  float* wo = wout + (size_t)r * plane;
  float* st = stage + (size_t)r * kChunk * g.nsub;
  // subgrid column of this thread (or -1)
  const int jx = c - g.nb;
  const int sx = (jx >= 0 && jx < g.nx && (jx % g.stride) == 0) ? jx / g.stride : -1;

  if (tid < 2) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        lds[b][t][tid] = 0.f;
        lds[b][t][kBand + 2 + tid] = 0.f;
      }
  }

  float uw[T][5];  // uw[t]: level-t rows q-2..q+2 for the level-(t+1) update of row q
  float wd[T][3];  // wd[t]: level-t w of rows q..q+2
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 5; ++i) uw[t][i] = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) wd[t][i] = 0.f;
  }

  const int Z = g.Z;
  for (int k = 0; k < Z + 2 * T; ++k) {
    // level 0: ingest row k
    float u0 = 0.f, w0 = 0.f;
    if (colv && k < Z) {
      const size_t o = (size_t)(k + kGhost) * P + (c + kGhost);
      u0 = ui[o];
      w0 = wi[o];
    }
    push(uw[0], u0);
    push(wd[0], w0);
    const int buf = k & 1;
    lds[buf][0][tid + 2] = uw[0][2];
#pragma unroll
    for (int t = 1; t < T; ++t) lds[buf][t][tid + 2] = uw[t][3];
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= T; ++t) {
      const int q = k - 2 * t;
      float un = 0.f, wn = 0.f;
      if (colv && q >= 0 && q < Z) {
        const float cen = uw[t - 1][2];
        if (t <= nlev) {
          const float* L = lds[buf][t - 1];
          const float n1 = (L[tid + 1] + L[tid + 3]) + (uw[t - 1][1] + uw[t - 1][3]);
          const float n2 = (L[tid] + L[tid + 4]) + (uw[t - 1][0] + uw[t - 1][4]);
          const float lap = 16.f * n1 - n2 - 60.f * cen;
          const size_t o = (size_t)(q + kGhost) * P + (c + kGhost);
          wn = ba[o] * wd[t - 1][0] + ca[o] * lap;
          un = cen + wn;
          const int jz = q - g.nb;
          if (own && sx >= 0 && jz >= 0 && jz < g.nz && (jz % g.stride) == 0) {
            st[(size_t)(slot0 + t - 1) * g.nsub + (size_t)(jz / g.stride) * g.nxs + sx] = un;
          }
        } else {
          un = cen;
          wn = wd[t - 1][0];
        }
      }
      if (t < T) {
        push(uw[t], un);
        push(wd[t], wn);
      } else if (own && q >= 0 && q < Z) {
        const size_t o = (size_t)(q + kGhost) * P + (c + kGhost);
        uo[o] = un;
        wo[o] = wn;
      }
    }
  }
}

constexpr int kDftThreads = 256;
constexpr int kDftFB = 8;  // frequencies per register block

// ghat[f][r0 + r][x] (+)= sum_{tau < cnt} tw[n0 - 1 + tau][f] * stage[r][tau][x].
__global__ void __launch_bounds__(kDftThreads)
    k_dft_chunk(Geometry g, const float* __restrict__ stage, const float2* __restrict__ tw,
                int n0, int cnt, int first, int r0, float2* __restrict__ ghat) {
  extern __shared__ float2 stw[];  // [cnt][nf]
  const int nf = g.nf;
  for (int i = threadIdx.x; i < cnt * nf; i += blockDim.x) stw[i] = tw[(size_t)(n0 - 1) * nf + i];
  __syncthreads();
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (x >= g.nsub) return;
  const float* s = stage + (size_t)r * kChunk * g.nsub + x;
  for (int f0 = 0; f0 < nf; f0 += kDftFB) {
    float re[kDftFB], im[kDftFB];
#pragma unroll
    for (int k = 0; k < kDftFB; ++k) re[k] = im[k] = 0.f;
    for (int t = 0; t < cnt; ++t) {
      float v = s[(size_t)t * g.nsub];
#pragma unroll
      for (int k = 0; k < kDftFB; ++k) {
        if (f0 + k < nf) {
          float2 c = stw[t * nf + f0 + k];
          re[k] += v * c.x;
          im[k] += v * c.y;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kDftFB; ++k) {
      int f = f0 + k;
      if (f < nf) {
        size_t o = ((size_t)f * g.nr + r0 + r) * g.nsub + x;
        if (first) {
          ghat[o] = make_float2(re[k], im[k]);
        } else {
          float2 a = ghat[o];
          ghat[o] = make_float2(a.x + re[k], a.y + im[k]);
        }
      }
    }
  }
}

}  // namespace

int march_bands(const Geometry& g) { return cdiv(g.X, kBand - 4 * g.tblock); }

hipError_t launch_march(const Geometry& g, const float* ca, const float* ba, const float* uin,
                        const float* win, float* uout, float* wout, float* stage, int slot0,
                        int nlev, int nrb_now, hipStream_t st) {
  dim3 grid(march_bands(g), nrb_now);
  switch (g.tblock) {
    case 2:
      hipLaunchKernelGGL(k_march<2>, grid, dim3(kBand), 0, st, g, ca, ba, uin, win, uout, wout,
                         stage, slot0, nlev);
      break;
    case 4:
      hipLaunchKernelGGL(k_march<4>, grid, dim3(kBand), 0, st, g, ca, ba, uin, win, uout, wout,
                         stage, slot0, nlev);
      break;
    case 8:
      hipLaunchKernelGGL(k_march<8>, grid, dim3(kBand), 0, st, g, ca, ba, uin, win, uout, wout,
                         stage, slot0, nlev);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dft_chunk(const Geometry& g, const float* stage, const float2* tw, int n0,
                            int cnt, bool first, int r0, int nrb_now, float2* ghat,
                            hipStream_t st) {
  dim3 grid(cdiv(g.nsub, kDftThreads), nrb_now);
  size_t shmem = (size_t)cnt * g.nf * sizeof(float2);
  hipLaunchKernelGGL(k_dft_chunk, grid, dim3(kDftThreads), shmem, st, g, stage, tw, n0, cnt,
                     first ? 1 : 0, r0, ghat);
  return hipGetLastError();
}

}  // namespace ehi
