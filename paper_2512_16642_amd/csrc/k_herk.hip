// Hessian assembly Hhat(w) = Ghat(w) Ghat(w)^H over the grid, per frequency.
//
// Paper: the Fourier diagonal of block (i, j) is the transform of the
// cross-correlation of the two Green functions summed over space (Fourier-domain
// Hessian and computation of the Fourier diagonals); with the final spectra
// ghat_i(w, x) it is sum_x ghat_i conj(ghat_j).  Only tiles on or above the
// diagonal are computed; the reduction mirrors them (Hermitian fill of the
// paper's algorithm).  The grid sum is split into partitions (split-K) so the
// launch fills the chip; partitions are reduced in FP64 in a fixed order.
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int T = kHerkTile;  // 32
constexpr int KC = 32;        // grid points per LDS stage

__device__ inline void tile_of_pair(int p, int nt, int* ti, int* tj) {
  // enumerate pairs ti <= tj row by row
  int i = 0;
  while (p >= nt - i) {
    p -= nt - i;
    ++i;
  }
  *ti = i;
  *tj = i + p;
}

// Plain FP32 form: 16x16 threads, each 2x2 outputs of a 32x32 tile.
// Accumulation is two-level: each KC-wide stage is summed from zero, then added
// to the running sum, which keeps the FP32 error growth at sqrt(K/KC).
__global__ void __launch_bounds__(256)
    k_herk_fp32(Geometry g, const float2* __restrict__ ghat, float2* __restrict__ hpart,
                int split) {
  __shared__ float2 sa[T][KC + 1];
  __shared__ float2 sb[T][KC + 1];
  const int ntile = cdiv(g.nr, T);
  int ti, tj;
  tile_of_pair(blockIdx.x, ntile, &ti, &tj);
  const int f = blockIdx.y;
  const int ks = blockIdx.z;
  const int kchunk = cdiv(cdiv(g.nsub, split), KC) * KC;
  const int k0 = ks * kchunk;
  const int k1 = min(g.nsub, k0 + kchunk);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const float2* A = ghat + (size_t)f * g.nr * g.nsub;
  float accr[2][2] = {{0, 0}, {0, 0}}, acci[2][2] = {{0, 0}, {0, 0}};
  for (int kb = k0; kb < k1; kb += KC) {
    for (int e = threadIdx.x; e < T * KC; e += 256) {
      int row = e / KC, col = e % KC;
      int k = kb + col;
      int ia = ti * T + row, ib = tj * T + row;
      sa[row][col] = (ia < g.nr && k < k1) ? A[(size_t)ia * g.nsub + k] : make_float2(0.f, 0.f);
      sb[row][col] = (ib < g.nr && k < k1) ? A[(size_t)ib * g.nsub + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    float pr[2][2] = {{0, 0}, {0, 0}}, pi[2][2] = {{0, 0}, {0, 0}};
#pragma unroll 4
    for (int k = 0; k < KC; ++k) {
      float2 a0 = sa[ty * 2 + 0][k], a1 = sa[ty * 2 + 1][k];
      float2 b0 = sb[tx * 2 + 0][k], b1 = sb[tx * 2 + 1][k];
      // a * conj(b) = (ar br + ai bi) + i (ai br - ar bi)
      pr[0][0] += a0.x * b0.x + a0.y * b0.y;  pi[0][0] += a0.y * b0.x - a0.x * b0.y;
      pr[0][1] += a0.x * b1.x + a0.y * b1.y;  pi[0][1] += a0.y * b1.x - a0.x * b1.y;
      pr[1][0] += a1.x * b0.x + a1.y * b0.y;  pi[1][0] += a1.y * b0.x - a1.x * b0.y;
      pr[1][1] += a1.x * b1.x + a1.y * b1.y;  pi[1][1] += a1.y * b1.x - a1.x * b1.y;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accr[a][b] += pr[a][b];
        acci[a][b] += pi[a][b];
      }
    __syncthreads();
  }
  float2* out = hpart + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int i = ti * T + ty * 2 + a, j = tj * T + tx * 2 + b;
      if (i < g.nr && j < g.nr) out[(size_t)i * g.nr + j] = make_float2(accr[a][b], acci[a][b]);
    }
}

// hhat[f][i][j] = sum_ks hpart[ks][f][i][j] (FP64, ascending ks) for j >= i,
// mirrored to [j][i] as the conjugate; the diagonal's imaginary part is 0.
__global__ void k_herk_reduce(Geometry g, const float2* __restrict__ hpart, double2* __restrict__ hhat,
                              int split) {
  const int f = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nr * g.nr) return;
  int i = e / g.nr, j = e % g.nr;
  if (j < i) return;
  double sr = 0.0, si = 0.0;
  for (int ks = 0; ks < split; ++ks) {
    float2 v = hpart[((size_t)ks * g.nf + f) * g.nr * g.nr + e];
    sr += (double)v.x;
    si += (double)v.y;
  }
  double2* H = hhat + (size_t)f * g.nr * g.nr;
  if (i == j) {
    H[(size_t)i * g.nr + i] = make_double2(sr, 0.0);
  } else {
    H[(size_t)i * g.nr + j] = make_double2(sr, si);
    H[(size_t)j * g.nr + i] = make_double2(sr, -si);
  }
}

}  // namespace

hipError_t launch_herk_fp32(const Geometry& g, const float2* ghat, float2* hpart, hipStream_t st) {
  int ntile = cdiv(g.nr, T);
  dim3 grid(ntile * (ntile + 1) / 2, g.nf, g.herk_split);
  hipLaunchKernelGGL(k_herk_fp32, grid, dim3(256), 0, st, g, ghat, hpart, g.herk_split);
  return hipGetLastError();
}

hipError_t launch_herk_reduce(const Geometry& g, const float2* hpart, double2* hhat,
                              hipStream_t st) {
  dim3 grid(cdiv(g.nr * g.nr, 256), g.nf);
  hipLaunchKernelGGL(k_herk_reduce, grid, dim3(256), 0, st, g, hpart, hhat, g.herk_split);
  return hipGetLastError();
}

}  // namespace ehi
