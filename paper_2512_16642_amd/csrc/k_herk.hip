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

// Precision form: split-BF16 products on MFMA with FP32 accumulation.
// With g = a + i b, Re H = A A^T + B B^T and Im H = B A^T - A B^T (rows i, j;
// columns = grid points).  Every FP32 value x is split as x = hi + lo + O(2^-17 x)
// with hi = bf16(x), lo = bf16(x - hi), and a product xy is taken as
// hi*hi + hi*lo + lo*hi + lo*lo.  (Without lo*lo the diagonal sum_x |g|^2 is
// biased low by about sum lo^2 / sum x^2 ~ 1e-6, which the ill-conditioned
// low-frequency systems amplify ~100x in the multipliers.)
//
// The MFMA's internal accumulation is biased (the error of the diagonal grows
// linearly with the number of MFMAs chained into one accumulator), so each
// 32-point stage is chained from zero and added to the running FP32 sum with an
// ordinary round-to-nearest add: the bias is bounded by one stage.
//
// Workgroup: 4 waves, a 64 x 64 tile (i-block, j-block) of H for one frequency
// and one grid-point partition; each wave owns a 32 x 32 quarter as 2 x 2
// v_mfma_f32_16x16x32_bf16 tiles for Re and Im.  Per stage, 32 grid points of
// the 128 rows are loaded once, split into hi/lo BF16 planes in LDS, and read
// back as MFMA fragments (lane l: row l % 16, points 8 (l / 16) .. + 7).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBt = 64;  // H tile (rows = cols)
constexpr int kBk = 32;  // grid points per stage (four groups of 8)

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__global__ void __launch_bounds__(256)
    k_herk_bf16(Geometry g, const float2* __restrict__ ghat, float2* __restrict__ hpart, int split) {
  // planes: 0 = Re hi, 1 = Re lo, 2 = Im hi, 3 = Im lo; rows 0..63 i-block, 64..127 j-block;
  // [plane][group of 8 points][row][8]: every fragment is one aligned 16-byte chunk
  __shared__ __attribute__((aligned(16))) unsigned short pl[4][kBk / 8][2 * kBt][8];
  const int nblk = cdiv(g.nr, kBt);
  int bi, bj;
  {
    int p = blockIdx.x, i = 0;
    while (p >= nblk - i) {
      p -= nblk - i;
      ++i;
    }
    bi = i;
    bj = i + p;
  }
  const int ks = blockIdx.y;
  const int f = blockIdx.z;
  const int kchunk = cdiv(cdiv(g.nsub, split), kBk) * kBk;
  const int k0 = ks * kchunk;
  const int k1 = min(g.nsub, k0 + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const float2* G = ghat + (size_t)f * g.nr * g.nsub;

  floatx4 re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  // load assignment: thread -> (row 0..127, 16 consecutive points)
  const int lrow = tid >> 1;
  const int lhalf = tid & 1;
  const int grow = lrow < kBt ? bi * kBt + lrow : bj * kBt + (lrow - kBt);
  const bool rowv = grow < g.nr;
  const float2* Grow = G + (size_t)(rowv ? grow : 0) * g.nsub;

  for (int kb = k0; kb < k1; kb += kBk) {
    __syncthreads();
#pragma unroll 4
    for (int e = 0; e < 16; ++e) {
      const int k = kb + lhalf * 16 + e;
      float2 v = make_float2(0.f, 0.f);
      if (rowv && k < k1) v = Grow[k];
      const unsigned short rh = bf16_rne(v.x), ih = bf16_rne(v.y);
      const int kk = lhalf * 16 + e;
      pl[0][kk >> 3][lrow][kk & 7] = rh;
      pl[1][kk >> 3][lrow][kk & 7] = bf16_rne(v.x - bf16_to_f(rh));
      pl[2][kk >> 3][lrow][kk & 7] = ih;
      pl[3][kk >> 3][lrow][kk & 7] = bf16_rne(v.y - bf16_to_f(ih));
    }
    __syncthreads();
    const int fr = lane & 15, fg = lane >> 4;
    bf16x8 ai[2][4], aj[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ai[a][q] = *reinterpret_cast<const bf16x8*>(&pl[q][fg][wi * 32 + a * 16 + fr][0]);
        aj[a][q] = *reinterpret_cast<const bf16x8*>(&pl[q][fg][kBt + wj * 32 + a * 16 + fr][0]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      // -A_i fragments for the subtracted term of Im
      bf16x8 nrh = -ai[a][0], nrl = -ai[a][1];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        floatx4 r = floatx4{0.f, 0.f, 0.f, 0.f}, m = floatx4{0.f, 0.f, 0.f, 0.f};
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][0], aj[b][0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][0], aj[b][1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][1], aj[b][0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][1], aj[b][1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][3], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][3], r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][0], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][1], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][0], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][1], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[b][2], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[b][3], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[b][2], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[b][3], m, 0, 0, 0);
        re[a][b] += r;
        im[a][b] += m;
      }
    }
  }
  // D[4 (lane / 16) + v][lane % 16] of tile (a, b)
  float2* out = hpart + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bi * kBt + wi * 32 + a * 16 + 4 * (lane >> 4) + v;
        const int j = bj * kBt + wj * 32 + b * 16 + (lane & 15);
        if (i < g.nr && j < g.nr) out[(size_t)i * g.nr + j] = make_float2(re[a][b][v], im[a][b][v]);
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

int herk_bf16_blocks(const Geometry& g) {
  const int nb = cdiv(g.nr, kBt);
  return nb * (nb + 1) / 2;
}

hipError_t launch_herk_split_bf16(const Geometry& g, const float2* ghat, float2* hpart,
                                  hipStream_t st) {
  dim3 grid(herk_bf16_blocks(g), g.herk_split, g.nf);
  hipLaunchKernelGGL(k_herk_bf16, grid, dim3(256), 0, st, g, ghat, hpart, g.herk_split);
  return hipGetLastError();
}

hipError_t launch_herk_reduce(const Geometry& g, const float2* hpart, double2* hhat,
                              hipStream_t st) {
  dim3 grid(cdiv(g.nr * g.nr, 256), g.nf);
  hipLaunchKernelGGL(k_herk_reduce, grid, dim3(256), 0, st, g, hpart, hhat, g.herk_split);
  return hipGetLastError();
}

}  // namespace ehi
