// Green-function time stepping and the DFT accumulated during the time loop.
//
// Paper: the Green function of receiver j is the wavefield of a Dirac source at
// the receiver (Direct Hessian-inverse computation, block equation of the
// Hessian); Nr PDE solves build the Hessian (computational cost section).  The
// Fourier representation of each Green function at the needed frequencies
// (Fourier-domain Hessian) is accumulated here while stepping, so the time
// samples never leave a short staging window (the discussion proposes
// on-the-fly computation to avoid storing the wavefields).
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int kStepBX = 64;
constexpr int kStepBY = 4;

// One time step for every cell of the padded grid and every receiver of the
// batch (blockIdx.z).  Increment form of the 2nd-order-in-time recurrence:
//   w <- (b/a) w + kappa/(12 h^2 a) * (16 (sum of 4 nearest) - (sum of 4 next) - 60 u)
//   u_next = u + w
// The sample u_next on the stride subgrid goes to staging slot `slot`.
__global__ void __launch_bounds__(kStepBX* kStepBY)
    k_step(Geometry g, const float* __restrict__ ca, const float* __restrict__ ba,
           const float* __restrict__ ucur, float* __restrict__ unext, float* __restrict__ w,
           float* __restrict__ stage, int slot) {
  int ix = blockIdx.x * kStepBX + threadIdx.x;
  int iz = blockIdx.y * kStepBY + threadIdx.y;
  int r = blockIdx.z;
  if (ix >= g.X || iz >= g.Z) return;
  const size_t plane = g.plane();
  const int P = g.Xp;
  const size_t o = (size_t)(iz + kGhost) * P + (ix + kGhost);
  const float* u = ucur + (size_t)r * plane;
  float c = u[o];
  float n1 = (u[o - 1] + u[o + 1]) + (u[o - P] + u[o + P]);
  float n2 = (u[o - 2] + u[o + 2]) + (u[o - 2 * P] + u[o + 2 * P]);
  float lap = 16.f * n1 - n2 - 60.f * c;
  size_t ow = (size_t)r * plane + o;
  float wn = ba[o] * w[ow] + ca[o] * lap;
  w[ow] = wn;
  float un = c + wn;
  unext[ow] = un;
  int jz = iz - g.nb, jx = ix - g.nb;
  if (jz >= 0 && jz < g.nz && jx >= 0 && jx < g.nx && (jz % g.stride) == 0 &&
      (jx % g.stride) == 0) {
    stage[((size_t)r * kChunk + slot) * g.nsub + (size_t)(jz / g.stride) * g.nxs + jx / g.stride] = un;
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

hipError_t launch_step(const Geometry& g, const float* ca, const float* ba, const float* ucur,
                       float* unext, float* w, float* stage, int slot, int nrb_now,
                       hipStream_t st) {
  dim3 grid(cdiv(g.X, kStepBX), cdiv(g.Z, kStepBY), nrb_now);
  hipLaunchKernelGGL(k_step, grid, dim3(kStepBX, kStepBY), 0, st, g, ca, ba, ucur, unext, w,
                     stage, slot);
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
