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
// the 128 rows are split into hi/lo BF16 planes and stored in LDS as 16-byte
// fragments [plane][group of 8 points][row] (lane l of an MFMA reads row
// l % 16, points 8 (l / 16) .. + 7: one aligned 16-byte read).  Stages are
// double-buffered: the global loads of stage s + 1 are in flight while the
// MFMAs of stage s run, and one barrier separates stages.
//
// Work items (tile pair, partition, frequency) are laid out so that the tile
// pairs of one (partition, frequency) run on the same XCD (workgroups are
// dealt to the 8 XCDs round-robin): the row blocks they share are then read
// from HBM into that XCD's L2 once instead of once per pair.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// hi/lo split of two FP32 values into packed BF16 pairs (element 0 in the low
// half): hi = bf16(x) (round to nearest even), lo = bf16(x - hi).  The hi pair
// is converted once and its two halves widened back to FP32 by a byte permute
// and a mask, so every value costs one half of each conversion (used where the
// split sits on the per-step path of the finite-record contraction; the
// once-per-stage splits of the final-spectrum forms keep the plain expression,
// which holds fewer registers there).
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, bf16x2{(__bf16)x0, (__bf16)x1});
  // low half moved up by a byte permute (the compiler would otherwise convert
  // x0 a second time to widen it)
  const float h0 = __uint_as_float(__builtin_amdgcn_perm(0u, hi, 0x01000c0cu));
  const float h1 = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, bf16x2{(__bf16)(x0 - h0), (__bf16)(x1 - h1)});
}

constexpr int kBt = 64;  // H tile (rows = cols)
constexpr int kBk = 32;  // grid points per stage (four groups of 8)
constexpr int kXcd = 8;  // XCDs per device


// VEC: every row of ghat starts 16-byte aligned (nsub even), so 8 points load
// as four 16-byte loads.  Every FP32 value x is split as hi = bf16(x),
// lo = bf16(x - hi), both rounded to nearest even by the hardware conversion.
template <bool VEC>
__global__ void __launch_bounds__(256)
    k_herk_bf16(Geometry g, const float2* __restrict__ ghat, float2* __restrict__ hpart, int split) {
  // planes: 0 = Re hi, 1 = Re lo, 2 = Im hi, 3 = Im lo; rows 0..63 i-block, 64..127 j-block
  __shared__ u32x4 pl[2][4][kBk / 8][2 * kBt];
  const int nblk = cdiv(g.nr, kBt);
  const int npair = nblk * (nblk + 1) / 2;
  // XCD-aware work item: consecutive items (the pairs of one partition and
  // frequency) go to the workgroups one XCD receives
  const int n = blockIdx.x;
  const int n8 = gridDim.x / kXcd * kXcd;
  const int item = n < n8 ? (n % kXcd) * (n8 / kXcd) + n / kXcd : n;
  int bi, bj;
  {
    int p = item % npair, i = 0;
    while (p >= nblk - i) {
      p -= nblk - i;
      ++i;
    }
    bi = i;
    bj = i + p;
  }
  const int ks = (item / npair) % split;
  const int f = item / (npair * split);
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

  // load tasks: row lrow (0..127), point groups (tid >> 7) and (tid >> 7) + 2
  const int lrow = tid & (2 * kBt - 1);
  const int grow = lrow < kBt ? bi * kBt + lrow : bj * kBt + (lrow - kBt);
  const bool rowv = grow < g.nr;
  const float2* Grow = G + (size_t)(rowv ? grow : 0) * g.nsub;
  float2 v[2][8];
  auto gload = [&](int kb) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int k = kb + 8 * ((tid >> 7) + 2 * p);
      if (VEC && rowv && k + 8 <= k1) {
        const floatx4* src = reinterpret_cast<const floatx4*>(Grow + k);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const floatx4 q = src[e];
          v[p][2 * e] = make_float2(q[0], q[1]);
          v[p][2 * e + 1] = make_float2(q[2], q[3]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[p][e] = (rowv && k + e < k1) ? Grow[k + e] : make_float2(0.f, 0.f);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int grp = (tid >> 7) + 2 * p;
      unsigned w[4][4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const float2 z0 = v[p][e], z1 = v[p][e + 1];
        const bf16x2 rh = {(__bf16)z0.x, (__bf16)z1.x};
        const bf16x2 ih = {(__bf16)z0.y, (__bf16)z1.y};
        const bf16x2 rl = {(__bf16)(z0.x - (float)rh[0]), (__bf16)(z1.x - (float)rh[1])};
        const bf16x2 il = {(__bf16)(z0.y - (float)ih[0]), (__bf16)(z1.y - (float)ih[1])};
        w[0][e >> 1] = __builtin_bit_cast(unsigned, rh);
        w[1][e >> 1] = __builtin_bit_cast(unsigned, rl);
        w[2][e >> 1] = __builtin_bit_cast(unsigned, ih);
        w[3][e >> 1] = __builtin_bit_cast(unsigned, il);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) pl[buf][q][grp][lrow] = u32x4{w[q][0], w[q][1], w[q][2], w[q][3]};
    }
  };

  const int nst = cdiv(k1 - k0, kBk);
  if (nst > 0) {
    gload(k0);
    lstore(0);
  }
  __syncthreads();
  const int fr = lane & 15, fg = lane >> 4;
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) gload(k0 + (st + 1) * kBk);
    bf16x8 ai[2][4], aj[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ai[a][q] = __builtin_bit_cast(bf16x8, pl[buf][q][fg][wi * 32 + a * 16 + fr]);
        aj[a][q] = __builtin_bit_cast(bf16x8, pl[buf][q][fg][kBt + wj * 32 + a * 16 + fr]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      // -A_i fragments for the subtracted term of Im (sign bits flipped)
      const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
      const bf16x8 nrh = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, ai[a][0]) ^ sgn);
      const bf16x8 nrl = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, ai[a][1]) ^ sgn);
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
    if (st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }
  // D[4 (lane / 16) + v][lane % 16] of tile (a, b)
  float2* out = hpart + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int i = bi * kBt + wi * 32 + a * 16 + 4 * (lane >> 4) + v4;
        const int j = bj * kBt + wj * 32 + b * 16 + (lane & 15);
        if (i < g.nr && j < g.nr) out[(size_t)i * g.nr + j] = make_float2(re[a][b][v4], im[a][b][v4]);
      }
}

// The same contraction for surveys of at most 224 receivers, without tile
// pairs: the 32 x 32 block pairs (bi <= bj) of the 32-row blocks, in row-major
// order of the upper triangle, form groups of 16, and one workgroup per
// (frequency, grid-point partition, group) stages every row once per 32-point
// stage (loaded from HBM, split into hi/lo planes, stored in LDS) and computes
// its group's pairs, pair 16 group + w + 8 m on wave w (m < 2: waves w and
// w + 4 share a SIMD, so a partial group still spreads evenly).  Per pair the
// same 2 x 2 MFMA tiles and 16 products per tile as above, 32-point chains from
// zero; stages are double-buffered.  At 200 receivers (28 pairs, 2 groups) the
// spectra are read twice instead of about three times, and split once per
// group instead of once per tile pair.  Output: the upper-triangle blocks of
// hpart (the reduction reads j >= i only).
//
// TILED (more than 224 receivers, whose rows do not all fit in LDS): the
// groups are the tiles of a 4 x 4 tiling of the block-pair triangle.  A tile
// off the diagonal pairs row blocks 4 ti .. + 3 with row blocks 4 tj .. + 3
// (16 pairs, eight blocks staged); a tile on it, the upper triangle of its four
// blocks (10 pairs, four blocks staged).  Every row block is then read by about
// half as many workgroups as there are tiles in a row of the triangle, instead
// of once per 64 x 64 tile pair.
constexpr int kWholeRows = 256;   // rows held in LDS (eight 32-row blocks)
constexpr int kWholeWaves = 8;
constexpr int kWholePairs = 2;    // block pairs per wave
constexpr int kWholeGroup = kWholeWaves * kWholePairs;
constexpr int kWholeTile = 4;     // blocks per side of a tile (TILED)
constexpr int kWholeMaxNr = 224;  // receivers of the untiled form (all rows staged)

template <bool VEC, bool TILED>
__global__ void __launch_bounds__(512)
    k_herk_bf16_whole(Geometry g, const float2* __restrict__ ghat, float2* __restrict__ hpart, int split) {
  __shared__ u32x4 pl[2][4][kBk / 8][kWholeRows];  // [buffer][plane][group of 8 points][row]
  const int nb = cdiv(g.nr, 32);
  const int ntile = cdiv(nb, kWholeTile);
  const int ngroup = TILED ? ntile * (ntile + 1) / 2 : cdiv(nb * (nb + 1) / 2, kWholeGroup);
  const int grp_id = blockIdx.x % ngroup;
  // staged row blocks: s < ni is block i0 + s, s >= ni block j0 + s - ni (TILED);
  // every block in order otherwise
  int i0 = 0, ni = nb, j0 = 0, nj = 0, npair = nb * (nb + 1) / 2, nstage = nb;
  bool diag = true;
  if constexpr (TILED) {
    int ti = 0, p = grp_id;
    while (p >= ntile - ti) {
      p -= ntile - ti;
      ++ti;
    }
    const int tj = ti + p;
    i0 = kWholeTile * ti;
    ni = min(kWholeTile, nb - i0);
    j0 = kWholeTile * tj;
    nj = min(kWholeTile, nb - j0);
    diag = ti == tj;
    npair = diag ? ni * (ni + 1) / 2 : ni * nj;
    nstage = diag ? ni : ni + nj;
  }
  const int rows = nstage * 32;  // rows staged (zero beyond nr)
  const int ks = (blockIdx.x / ngroup) % split;
  const int f = blockIdx.x / (ngroup * split);
  const int kchunk = cdiv(cdiv(g.nsub, split), kBk) * kBk;
  const int k0 = ks * kchunk;
  const int k1 = min(g.nsub, k0 + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const float2* G = ghat + (size_t)f * g.nr * g.nsub;

  // this wave's block pairs: p = 16 group + wave + 8 m (TILED: p = wave + 8 m of
  // the tile), row-major in the upper triangle (off-diagonal tiles: row-major
  // over the ni x nj pairs); pbi/pbj are the staged (LDS) blocks, gbi/gbj the
  // blocks of the Hessian
  int pbi[kWholePairs], pbj[kWholePairs], gbi[kWholePairs], gbj[kWholePairs];
  const int pfirst = (TILED ? 0 : grp_id * kWholeGroup) + wave;
  const int mine = npair > pfirst ? min(kWholePairs, (npair - pfirst + kWholeWaves - 1) / kWholeWaves) : 0;
#pragma unroll
  for (int m = 0; m < kWholePairs; ++m) {
    int p = pfirst + kWholeWaves * m, i = 0;
    if (p >= npair) p = 0;
    if (diag) {
      while (p >= ni - i) {
        p -= ni - i;
        ++i;
      }
      pbi[m] = i;
      pbj[m] = i + p;
      gbi[m] = i0 + i;
      gbj[m] = i0 + i + p;
    } else {
      pbi[m] = p / nj;
      pbj[m] = ni + p % nj;
      gbi[m] = i0 + p / nj;
      gbj[m] = j0 + p % nj;
    }
  }
  floatx4 re[kWholePairs][2][2], im[kWholePairs][2][2];
#pragma unroll
  for (int m = 0; m < kWholePairs; ++m)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) re[m][a][b] = im[m][a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  // load tasks: (row, point group) = (task % rows, task / rows), task = tid, tid + 512
  float2 v[2][8];
  auto gload = [&](int kb) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int task = tid + 512 * p;
      const int row = task % rows, grp = task / rows;
      const int sb = row >> 5;  // staged block
      const int grow = (sb < ni ? i0 + sb : j0 + sb - ni) * 32 + (row & 31);
      const bool ok = task < 4 * rows && grow < g.nr;
      const int k = kb + 8 * grp;
      const float2* src = G + (size_t)(ok ? grow : 0) * g.nsub;
      if (VEC && ok && k + 8 <= k1) {
        const floatx4* q4 = reinterpret_cast<const floatx4*>(src + k);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const floatx4 q = q4[e];
          v[p][2 * e] = make_float2(q[0], q[1]);
          v[p][2 * e + 1] = make_float2(q[2], q[3]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[p][e] = (ok && k + e < k1) ? src[k + e] : make_float2(0.f, 0.f);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int task = tid + 512 * p;
      if (task >= 4 * rows) continue;
      const int row = task % rows, grp = task / rows;
      unsigned w[4][4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const float2 z0 = v[p][e], z1 = v[p][e + 1];
        const bf16x2 rh = {(__bf16)z0.x, (__bf16)z1.x};
        const bf16x2 ih = {(__bf16)z0.y, (__bf16)z1.y};
        const bf16x2 rl = {(__bf16)(z0.x - (float)rh[0]), (__bf16)(z1.x - (float)rh[1])};
        const bf16x2 il = {(__bf16)(z0.y - (float)ih[0]), (__bf16)(z1.y - (float)ih[1])};
        w[0][e >> 1] = __builtin_bit_cast(unsigned, rh);
        w[1][e >> 1] = __builtin_bit_cast(unsigned, rl);
        w[2][e >> 1] = __builtin_bit_cast(unsigned, ih);
        w[3][e >> 1] = __builtin_bit_cast(unsigned, il);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) pl[buf][q][grp][row] = u32x4{w[q][0], w[q][1], w[q][2], w[q][3]};
    }
  };

  const int nst = cdiv(k1 - k0, kBk);
  // waves w and w + 4 share a SIMD: the first four split the next stage before
  // their products and the other four after theirs, so one wave's conversions
  // run beside the other's matrix products.  The early waves load two stages
  // ahead (their split comes first, so its data must already be in flight).
  const bool early = wave < 4;
  if (nst > 0) {
    gload(k0);
    lstore(0);
    if (early && nst > 1) gload(k0 + kBk);
  }
  __syncthreads();
  const int fr = lane & 15, fg = lane >> 4;
  const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (early) {
      if (st + 1 < nst) lstore(buf ^ 1);
      if (st + 2 < nst) gload(k0 + (st + 2) * kBk);
    } else if (st + 1 < nst) {
      gload(k0 + (st + 1) * kBk);
    }
    bf16x8 ai[2][4], aj[2][4];
#pragma unroll
    for (int m = 0; m < kWholePairs; ++m) {
      if (m >= mine) break;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ai[a][q] = __builtin_bit_cast(bf16x8, pl[buf][q][fg][pbi[m] * 32 + a * 16 + fr]);
          aj[a][q] = __builtin_bit_cast(bf16x8, pl[buf][q][fg][pbj[m] * 32 + a * 16 + fr]);
        }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const bf16x8 nrh = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, ai[a][0]) ^ sgn);
        const bf16x8 nrl = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, ai[a][1]) ^ sgn);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          floatx4 r = floatx4{0.f, 0.f, 0.f, 0.f}, mm = floatx4{0.f, 0.f, 0.f, 0.f};
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][0], aj[b][0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][0], aj[b][1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][1], aj[b][0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][1], aj[b][1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][2], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][3], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][2], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][3], r, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][0], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][2], aj[b][1], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][0], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[a][3], aj[b][1], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[b][2], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[b][3], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[b][2], mm, 0, 0, 0);
          mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[b][3], mm, 0, 0, 0);
          re[m][a][b] += r;
          im[m][a][b] += mm;
        }
      }
    }
    if (!early && st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }
  float2* out = hpart + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int m = 0; m < kWholePairs; ++m) {
    if (m >= mine) break;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
          const int i = gbi[m] * 32 + a * 16 + 4 * (lane >> 4) + v4;
          const int j = gbj[m] * 32 + b * 16 + (lane & 15);
          if (i < g.nr && j < g.nr) out[(size_t)i * g.nr + j] = make_float2(re[m][a][b][v4], im[m][a][b][v4]);
        }
  }
}

// Finite-record weighting (the paper's weighting function W(m, n) =
// min(Nt - m, Nt - n) in the algorithm for the Fourier block-diagonal Hessian):
// Hhat_W(w) = (1/Nt) sum_{p=1}^{Nt} Ghat_p(w) Ghat_p(w)^H, Ghat_p the DFT
// truncated after sample p.  One launch per staging window (samples
// n0 .. n0 + cnt - 1), before the DFT advances the spectra: each wave owns one
// 32 x 32 block pair (bi <= bj) of one frequency and grid partition, four
// block pairs to a workgroup (no block below the diagonal or beyond nr is
// computed).
// For every 32-point block of the partition a wave starts from the running
// spectra Ghat_{n0-1} of its 32 i-rows and 32 j-rows (zero for the first
// window), adds one staged sample times its twiddle per step and contracts
// them as the final-spectrum contraction does (hi/lo BF16 planes, four
// products, 32-point MFMA chains from zero).  A lane keeps the running spectra
// of the row and 8-point group its MFMA operands cover (row lane % 16, points
// 8 (lane / 16) ..), so the step loop needs no data exchange between waves;
// rows shared by two waves are updated by both.  Sums: 16 steps in FP32, then
// FP64 (per-lane LDS slots) over steps and blocks, then FP64 over windows
// (hpart64, read-modify-written by the one wave that owns the entry).
// All receivers must be stepped together.
__global__ void __launch_bounds__(256)
    k_herk_r2(Geometry g, const float* __restrict__ stage, const float2* __restrict__ tw,
              const float2* __restrict__ ghat, int n0, int cnt, int first, int gram_lo, int gram_hi,
              double2* __restrict__ hpart64) {
  __shared__ double acc_s[32][256];  // per lane: [a][b][re/im][v] FP64 sums
  // work: the 32 x 32 block pairs (bi <= bj) of the upper triangle, four to a
  // workgroup (one per wave; the waves are independent)
  const int nblk = cdiv(g.nr, 32);
  const int npair = nblk * (nblk + 1) / 2;
  const int ngrp = cdiv(npair, 4);
  const int split = g.herk_split;
  // XCD-aware work item; the frequency varies fastest, so the workgroups that
  // read the same staged rows share an XCD's L2
  const int n = blockIdx.x;
  const int n8 = gridDim.x / kXcd * kXcd;
  const int item = n < n8 ? (n % kXcd) * (n8 / kXcd) + n / kXcd : n;
  const int f = item % g.nf;
  const int rest = item / g.nf;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int pidx = 4 * (rest % ngrp) + wave;
  if (pidx >= npair) return;
  int bi, bj;
  {
    int p = pidx, i = 0;
    while (p >= nblk - i) {
      p -= nblk - i;
      ++i;
    }
    bi = i;
    bj = i + p;
  }
  const int ks = rest / ngrp;
  const int kchunk = cdiv(cdiv(g.nsub, split), kBk) * kBk;
  const int k0 = ks * kchunk;
  const int k1 = min(g.nsub, k0 + kchunk);
  const int fr = lane & 15, fg = lane >> 4;
  // this lane's four rows: i-rows (a = 0, 1), then j-rows (b = 0, 1)
  int row[4];
  bool rv[4];
  const float* Srow[4];
  const float2* Grow[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    row[u] = u < 2 ? bi * 32 + u * 16 + fr : bj * 32 + (u - 2) * 16 + fr;
    rv[u] = row[u] < g.nr;
    Srow[u] = stage + (size_t)(rv[u] ? row[u] : 0) * g.chunk * g.nsub_p;
    Grow[u] = ghat + ((size_t)f * g.nr + (rv[u] ? row[u] : 0)) * g.nsub;
  }
#pragma unroll
  for (int e = 0; e < 32; ++e) acc_s[e][tid] = 0.0;

  for (int kb = k0; kb < k1; kb += kBk) {
    const int kx = kb + 8 * fg;
    float2 S[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        S[u][e] = (!first && rv[u] && kx + e < k1) ? Grow[u][kx + e] : make_float2(0.f, 0.f);
    floatx4 grp[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) grp[a][b][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    auto gload = [&](floatx4 (&q)[4][2], int t) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* src = Srow[u] + (size_t)t * g.nsub_p + kx;
        q[u][0] = *reinterpret_cast<const floatx4*>(src);
        q[u][1] = *reinterpret_cast<const floatx4*>(src + 4);
      }
    };
    // No sample is masked: partitions end on 32-point block boundaries except
    // the last, whose tail lies in the row padding of the staging buffer, which
    // holds zeros; rows at or beyond nr run on row 0's samples and their entries
    // are not stored.
    auto step = [&](int t, const floatx4 (&q)[4][2]) {
      const float2 w = tw[(size_t)(n0 - 1 + t) * g.nf + f];
      bf16x8 fr4[4][4];  // [row][plane]
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float gv[8] = {q[u][0][0], q[u][0][1], q[u][0][2], q[u][0][3],
                             q[u][1][0], q[u][1][1], q[u][1][2], q[u][1][3]};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = gv[e];
          S[u][e].x = fmaf(w.x, x, S[u][e].x);
          S[u][e].y = fmaf(w.y, x, S[u][e].y);
        }
      }
      // kept samples before or after the record advance the running spectra
      // only (wave-uniform)
      if (t < gram_lo || t > gram_hi) return;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        unsigned wd[4][4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const float2 z0 = S[u][e], z1 = S[u][e + 1];
          split_pair(z0.x, z1.x, wd[0][e >> 1], wd[1][e >> 1]);
          split_pair(z0.y, z1.y, wd[2][e >> 1], wd[3][e >> 1]);
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          fr4[u][qq] = __builtin_bit_cast(bf16x8, u32x4{wd[qq][0], wd[qq][1], wd[qq][2], wd[qq][3]});
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        const bf16x8 nrh = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, fr4[a][0]) ^ sgn);
        const bf16x8 nrl = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, fr4[a][1]) ^ sgn);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const bf16x8* ai = fr4[a];
          const bf16x8* aj = fr4[2 + b];
          floatx4 r = floatx4{0.f, 0.f, 0.f, 0.f}, m = floatx4{0.f, 0.f, 0.f, 0.f};
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[0], aj[0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[0], aj[1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[1], aj[0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[1], aj[1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[2], aj[2], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[2], aj[3], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[3], aj[2], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[3], aj[3], r, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[2], aj[0], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[2], aj[1], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[3], aj[0], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[3], aj[1], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[2], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrh, aj[3], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[2], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nrl, aj[3], m, 0, 0, 0);
          grp[a][b][0] += r;
          grp[a][b][1] += m;
        }
      }
      if ((t & 15) == 15 || t == min(cnt - 1, gram_hi)) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
              for (int v4 = 0; v4 < 4; ++v4) acc_s[((a * 2 + b) * 2 + c) * 4 + v4][tid] += (double)grp[a][b][c][v4];
              grp[a][b][c] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
      }
    };
    for (int t = 0; t < cnt; ++t) {
      floatx4 q[4][2];
      gload(q, t);
      step(t, q);
    }
  }
  double2* out = hpart64 + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int i = bi * 32 + a * 16 + 4 * (lane >> 4) + v4;
        const int j = bj * 32 + b * 16 + (lane & 15);
        if (i < g.nr && j < g.nr) {
          double2* o = out + (size_t)i * g.nr + j;
          double2 v = first ? make_double2(0.0, 0.0) : *o;
          v.x += acc_s[((a * 2 + b) * 2 + 0) * 4 + v4][tid];
          v.y += acc_s[((a * 2 + b) * 2 + 1) * 4 + v4][tid];
          *o = v;
        }
      }
}

// Plain FP32 form on the FP32 matrix cores (v_mfma_f32_16x16x4f32): the same
// 64 x 64 tile pairs (bi <= bj), XCD-aware work order and partitions as the
// split-BF16 tile-pair kernel; a wave owns a 32 x 32 quarter as 2 x 2 tiles,
// Re = A_i A_j^T + B_i B_j^T, Im = B_i A_j^T - A_i B_j^T with the FP32 real and
// imaginary planes A, B.  Stages of 32 points of the 128 rows are
// double-buffered in LDS as [point][row] planes (lane l of a 16 x 16 x 4 step
// reads point k0 + l / 16 of row l % 16); each stage's products are chained
// from zero and added to the running FP32 sum (the matrix core's accumulation
// is biased over long chains).
template <bool VEC>
__global__ void __launch_bounds__(256)
    k_herk_fp32_mfma(Geometry g, const float2* __restrict__ ghat, float2* __restrict__ hpart, int split) {
  constexpr int RS = 2 * kBt + 4;                 // row stride of an LDS point row (words)
  __shared__ float sre[2][kBk][RS];
  __shared__ float sim[2][kBk][RS];
  const int nblk = cdiv(g.nr, kBt);
  const int npair = nblk * (nblk + 1) / 2;
  const int n = blockIdx.x;
  const int n8 = gridDim.x / kXcd * kXcd;
  const int item = n < n8 ? (n % kXcd) * (n8 / kXcd) + n / kXcd : n;
  int bi, bj;
  {
    int p = item % npair, i = 0;
    while (p >= nblk - i) {
      p -= nblk - i;
      ++i;
    }
    bi = i;
    bj = i + p;
  }
  const int ks = (item / npair) % split;
  const int f = item / (npair * split);
  const int kchunk = cdiv(cdiv(g.nsub, split), kBk) * kBk;
  const int k0 = ks * kchunk;
  const int k1 = min(g.nsub, k0 + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const float2* G = ghat + (size_t)f * g.nr * g.nsub;
  // load tasks: row lrow (0..127), points 16 (tid >> 7) .. + 15 of the stage
  const int lrow = tid & (2 * kBt - 1);
  const int grow = lrow < kBt ? bi * kBt + lrow : bj * kBt + (lrow - kBt);
  const bool rowv = grow < g.nr;
  const float2* Grow = G + (size_t)(rowv ? grow : 0) * g.nsub;
  const int kofs = 16 * (tid >> 7);
  float2 v[16];
  auto gload = [&](int kb) {
    const int k = kb + kofs;
    if (VEC && rowv && k + 16 <= k1) {
      // rows start 16-byte aligned (nsub even): eight 16-byte loads
      const floatx4* src = reinterpret_cast<const floatx4*>(Grow + k);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const floatx4 q = src[e];
        v[2 * e] = make_float2(q[0], q[1]);
        v[2 * e + 1] = make_float2(q[2], q[3]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = (rowv && k + e < k1) ? Grow[k + e] : make_float2(0.f, 0.f);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      sre[buf][kofs + e][lrow] = v[e].x;
      sim[buf][kofs + e][lrow] = v[e].y;
    }
  };
  floatx4 re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nst = cdiv(k1 - k0, kBk);
  if (nst > 0) {
    gload(k0);
    lstore(0);
  }
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) gload(k0 + (st + 1) * kBk);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int ri = wi * 32 + a * 16 + fr;
        const int rj = kBt + wj * 32 + b * 16 + fr;
        floatx4 r = floatx4{0.f, 0.f, 0.f, 0.f}, m = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kBk; kk += 4) {
          const float ar = sre[buf][kk + fk][ri], ai = sim[buf][kk + fk][ri];
          const float br = sre[buf][kk + fk][rj], bim = sim[buf][kk + fk][rj];
          r = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bim, r, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f32_16x16x4f32(-ar, bim, m, 0, 0, 0);
        }
        re[a][b] += r;
        im[a][b] += m;
      }
    if (st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }
  // D[4 (lane / 16) + v][lane % 16] of tile (a, b)
  float2* out = hpart + ((size_t)ks * g.nf + f) * g.nr * g.nr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int i = bi * kBt + wi * 32 + a * 16 + 4 * (lane >> 4) + v4;
        const int j = bj * kBt + wj * 32 + b * 16 + (lane & 15);
        if (i < g.nr && j < g.nr) out[(size_t)i * g.nr + j] = make_float2(re[a][b][v4], im[a][b][v4]);
      }
}

// hhat = scale[f] sum_ks hpart64[ks] (FP64, ascending ks), mirrored, Im(diag) = 0.
__global__ void k_herk_r2_reduce(Geometry g, const double2* __restrict__ hpart64, const double* __restrict__ scale,
                                 double2* __restrict__ hhat) {
  const int f = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nr * g.nr) return;
  const int i = e / g.nr, j = e % g.nr;
  if (j < i) return;
  double sr = 0.0, si = 0.0;
  for (int ks = 0; ks < g.herk_split; ++ks) {
    const double2 v = hpart64[((size_t)ks * g.nf + f) * g.nr * g.nr + e];
    sr += v.x;
    si += v.y;
  }
  sr *= scale[f];
  si *= scale[f];
  double2* H = hhat + (size_t)f * g.nr * g.nr;
  if (i == j) {
    H[(size_t)i * g.nr + i] = make_double2(sr, 0.0);
  } else {
    H[(size_t)i * g.nr + j] = make_double2(sr, si);
    H[(size_t)j * g.nr + i] = make_double2(sr, -si);
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
  if (g.herk_form == 3) {
    // FP32 products and sums on the vector units (16 x 16 threads per 32 x 32 tile)
    int ntile = cdiv(g.nr, T);
    dim3 grid(ntile * (ntile + 1) / 2, g.nf, g.herk_split);
    hipLaunchKernelGGL(k_herk_fp32, grid, dim3(256), 0, st, g, ghat, hpart, g.herk_split);
    return hipGetLastError();
  }
  const int nb = cdiv(g.nr, kBt);
  const long long items = (long long)nb * (nb + 1) / 2 * g.herk_split * g.nf;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  if (g.nsub % 2 == 0)
    hipLaunchKernelGGL(k_herk_fp32_mfma<true>, dim3((unsigned)items), dim3(256), 0, st, g, ghat, hpart, g.herk_split);
  else
    hipLaunchKernelGGL(k_herk_fp32_mfma<false>, dim3((unsigned)items), dim3(256), 0, st, g, ghat, hpart,
                       g.herk_split);
  return hipGetLastError();
}

int herk_whole_groups(int nr) {
  const int nb = cdiv(nr, 32);
  if (nr > kWholeMaxNr) {
    const int nt = cdiv(nb, kWholeTile);
    return nt * (nt + 1) / 2;
  }
  return cdiv(nb * (nb + 1) / 2, kWholeGroup);
}

int herk_bf16_blocks(const Geometry& g) {
  const int nb = cdiv(g.nr, kBt);
  return nb * (nb + 1) / 2;
}

hipError_t launch_herk_split_bf16(const Geometry& g, const float2* ghat, float2* hpart,
                                  hipStream_t st) {
  if (g.herk_whole) {
    const long long items = (long long)g.nf * g.herk_split * herk_whole_groups(g.nr);
    if (items > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)items);
    const bool tiled = g.nr > kWholeMaxNr;
    if (g.nsub % 2 == 0) {
      if (tiled)
        hipLaunchKernelGGL((k_herk_bf16_whole<true, true>), grid, dim3(512), 0, st, g, ghat, hpart, g.herk_split);
      else
        hipLaunchKernelGGL((k_herk_bf16_whole<true, false>), grid, dim3(512), 0, st, g, ghat, hpart, g.herk_split);
    } else {
      if (tiled)
        hipLaunchKernelGGL((k_herk_bf16_whole<false, true>), grid, dim3(512), 0, st, g, ghat, hpart, g.herk_split);
      else
        hipLaunchKernelGGL((k_herk_bf16_whole<false, false>), grid, dim3(512), 0, st, g, ghat, hpart, g.herk_split);
    }
    return hipGetLastError();
  }
  const long long items = (long long)herk_bf16_blocks(g) * g.herk_split * g.nf;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)items);
  if (g.nsub % 2 == 0)
    hipLaunchKernelGGL(k_herk_bf16<true>, grid, dim3(256), 0, st, g, ghat, hpart, g.herk_split);
  else
    hipLaunchKernelGGL(k_herk_bf16<false>, grid, dim3(256), 0, st, g, ghat, hpart, g.herk_split);
  return hipGetLastError();
}

hipError_t launch_herk_r2_chunk(const Geometry& g, const float* stage, const float2* tw,
                                const float2* ghat, int n0, int cnt, bool first, int gram_lo, int gram_hi,
                                double2* hpart64, hipStream_t st) {
  const int nb32 = cdiv(g.nr, 32);
  const long long items = (long long)cdiv(nb32 * (nb32 + 1) / 2, 4) * g.herk_split * g.nf;
  if (items > 0x7fffffffLL || cnt < 1 || cnt > g.chunk || g.nrb < g.nr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_herk_r2, dim3((unsigned)items), dim3(256), 0, st, g, stage, tw, ghat, n0, cnt,
                     first ? 1 : 0, gram_lo, gram_hi, hpart64);
  return hipGetLastError();
}

hipError_t launch_herk_r2_reduce(const Geometry& g, const double2* hpart64, const double* scale, double2* hhat,
                                 hipStream_t st) {
  dim3 grid(cdiv(g.nr * g.nr, 256), g.nf);
  hipLaunchKernelGGL(k_herk_r2_reduce, grid, dim3(256), 0, st, g, hpart64, scale, hhat);
  return hipGetLastError();
}

hipError_t launch_herk_reduce(const Geometry& g, const float2* hpart, double2* hhat,
                              hipStream_t st) {
  dim3 grid(cdiv(g.nr * g.nr, 256), g.nf);
  hipLaunchKernelGGL(k_herk_reduce, grid, dim3(256), 0, st, g, hpart, hhat, g.herk_split);
  return hipGetLastError();
}

}  // namespace ehi
