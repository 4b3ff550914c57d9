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
// ca = kappa / (12 h^2 a) per cell; ba = b / a depends only on the distance d
// into the absorbing layer and is read from a table bd[d] (both FP64-rounded).
//
// Inputs: level-0 fields uin, win (sample n_in); outputs: level-T fields uout,
// wout.  Levels beyond nlev pass their input through unchanged, so a launch
// can advance fewer than T steps.  Level t's sample (n_in + t) is written to
// staging slot slot0 + t - 1 on the stride subgrid.
//
// Grid: (bands, row segments, receivers).  A segment owns output rows
// [z0, z1) and starts marching 2T rows above z0: level t is exact on rows
// >= z0 - 2T + 2t, so every level is exact on the owned rows.
template <int T>
__global__ void __launch_bounds__(kBand)
    k_march(Geometry g, const float* __restrict__ ca, const float* __restrict__ bd,
            const float* __restrict__ uin, const float* __restrict__ win, float* __restrict__ uout,
            float* __restrict__ wout, float* __restrict__ stage, int slot0, int nlev) {
  constexpr int B = kBand - 4 * T;  // output columns per band
  constexpr int CR = 2 * T + 2;     // rows of the ca ring (reuse distance 2T + 1 barriers)
  __shared__ float lu[2][T][kBand + 4];
  __shared__ float lc[CR][kBand];
  __shared__ float lb[kMaxSponge + 1];
  const int tid = threadIdx.x;
  const int r = blockIdx.z;
  const int x0 = blockIdx.x * B - 2 * T;  // padded-grid column of thread 0
  const int c = x0 + tid;
  const bool colv = (c >= 0 && c < g.X);
  const bool own = (tid >= 2 * T && tid < kBand - 2 * T && colv);
  const int Z = g.Z;
  const int z0 = blockIdx.y * g.seg_rows;
  const int z1 = min(Z, z0 + g.seg_rows);
  const int kb = z0 - 2 * T;
  const int P = g.Xp;
  const size_t plane = g.plane();
  const float* ui = uin + (size_t)r * plane;
  const float* wi = win + (size_t)r * plane;
  float* uo = uout + (size_t)r * plane;
  float* wo = wout + (size_t)r * plane;
  float* st = stage + (size_t)r * g.chunk * g.nsub_p;
  const int jx = c - g.nb;
  const int sx = (jx >= 0 && jx < g.nx && (jx % g.stride) == 0) ? jx / g.stride : -1;
  const int dxs = max(max(g.nb - c, c - (g.nb + g.nx - 1)), 0);  // sponge distance in x

  if (tid < 2) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        lu[b][t][tid] = 0.f;
        lu[b][t][kBand + 2 + tid] = 0.f;
      }
  }
  for (int i = tid; i <= g.nb; i += kBand) lb[i] = bd[i];

  float uw[T][5];  // uw[t]: level-t rows q-2..q+2 for the level-(t+1) update of row q
  float wd[T][3];  // wd[t]: level-t w of rows q..q+2
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 5; ++i) uw[t][i] = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) wd[t][i] = 0.f;
  }
  // two-row prefetch queue of level-0 inputs
  float pu[3], pw[3], pc[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = kb + i;
    pu[i] = pw[i] = pc[i] = 0.f;
    if (colv && row >= 0 && row < Z) {
      const size_t o = (size_t)(row + kGhost) * P + (c + kGhost);
      pu[i] = ui[o];
      pw[i] = wi[o];
      pc[i] = ca[o];
    }
  }

  int ring = 0;  // (k - kb) % CR
  const int ke = z1 + 2 * T;
  for (int k = kb; k < ke; ++k) {
    {
      const int row = k + 2;
      pu[2] = pw[2] = pc[2] = 0.f;
      if (colv && row >= 0 && row < Z) {
        const size_t o = (size_t)(row + kGhost) * P + (c + kGhost);
        pu[2] = ui[o];
        pw[2] = wi[o];
        pc[2] = ca[o];
      }
    }
    push(uw[0], pu[0]);
    push(wd[0], pw[0]);
    lc[ring][tid] = pc[0];
    const int buf = (k - kb) & 1;
    lu[buf][0][tid + 2] = uw[0][2];
#pragma unroll
    for (int t = 1; t < T; ++t) lu[buf][t][tid + 2] = uw[t][3];
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= T; ++t) {
      const int q = k - 2 * t;
      float un = 0.f, wn = 0.f;
      if (colv && q >= 0 && q < Z) {
        const float cen = uw[t - 1][2];
        if (t <= nlev) {
          const float* L = lu[buf][t - 1];
          const float n1 = (L[tid + 1] + L[tid + 3]) + (uw[t - 1][1] + uw[t - 1][3]);
          const float n2 = (L[tid] + L[tid + 4]) + (uw[t - 1][0] + uw[t - 1][4]);
          const float lap = 16.f * n1 - n2 - 60.f * cen;
          int slot = ring - 2 * t;
          if (slot < 0) slot += CR;
          const int dzs = max(max(g.nb - q, q - (g.nb + g.nz - 1)), 0);
          const float bq = lb[max(dzs, dxs)];
          wn = bq * wd[t - 1][0] + lc[slot][tid] * lap;
          un = cen + wn;
          const int jz = q - g.nb;
          if (own && sx >= 0 && q >= z0 && q < z1 && jz >= 0 && jz < g.nz && (jz % g.stride) == 0) {
            st[(size_t)(slot0 + t - 1) * g.nsub_p + (size_t)(jz / g.stride) * g.nxs + sx] = un;
          }
        } else {
          un = cen;
          wn = wd[t - 1][0];
        }
      }
      if (t < T) {
        push(uw[t], un);
        push(wd[t], wn);
      } else if (own && q >= z0 && q < z1) {
        const size_t o = (size_t)(q + kGhost) * P + (c + kGhost);
        uo[o] = un;
        wo[o] = wn;
      }
    }
    pu[0] = pu[1];
    pw[0] = pw[1];
    pc[0] = pc[1];
    pu[1] = pu[2];
    pw[1] = pw[2];
    pc[1] = pc[2];
    ring = (ring + 1 == CR) ? 0 : ring + 1;
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kDftKs = 64;  // time samples per LDS twiddle stage

// DFT of one staged chunk as a real matrix product on FP32 MFMA:
//   C[m][x] = sum_tau A[m][tau] S[tau][x],  A[2f][tau] = Re tw, A[2f+1][tau] = Im tw,
//   ghat[f][r0 + r][x] (+)= (C[2f][x], C[2f+1][x]).
// v_mfma_f32_16x16x4f32 tiles: A (16 rows of m x 4 samples) from LDS, B (4
// samples x 16 grid points) from the staging buffer.  A wave owns 64 grid
// points as four 16-column tiles with a permuted column map (tile j, column i
// <-> grid point 4i + j) so each lane loads its four B values with one float4.
// Samples at tau >= cnt and frequencies >= nf are zero; points >= nsub are
// computed (the row pitch is padded) but not stored.
template <int MT>
__global__ void __launch_bounds__(256)
    k_dft_mfma(Geometry g, const float* __restrict__ stage, const float2* __restrict__ tw, int n0,
               int cnt, int first, int r0, float2* __restrict__ ghat) {
  constexpr int MP = 16 * MT;
  __shared__ float As[kDftKs][MP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = blockIdx.y;
  const int col = blockIdx.x * 256 + wave * 64 + 4 * (lane & 15);  // this lane's 4 grid points
  const int krow = lane >> 4;
  const float* S = stage + (size_t)r * g.chunk * g.nsub_p;
  floatx4 acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[mt][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int twoF = 2 * g.nf;
  for (int ks = 0; ks < cnt; ks += kDftKs) {
    __syncthreads();
    for (int e = threadIdx.x; e < kDftKs * MP; e += 256) {
      const int t = e / MP, m = e % MP;
      float v = 0.f;
      if (ks + t < cnt && m < twoF) {
        const float2 z = tw[(size_t)(n0 - 1 + ks + t) * g.nf + (m >> 1)];
        v = (m & 1) ? z.y : z.x;
      }
      As[t][m] = v;
    }
    __syncthreads();
    const int kend = min(kDftKs, cnt - ks);
    for (int k = 0; k < kend; k += 4) {
      const int tau = ks + k + krow;
      floatx4 b = floatx4{0.f, 0.f, 0.f, 0.f};
      if (tau < cnt) b = *reinterpret_cast<const floatx4*>(S + (size_t)tau * g.nsub_p + col);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float a = As[k + krow][16 * mt + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[j], acc[mt][j], 0, 0, 0);
      }
    }
  }
  // lane holds rows m = 16 mt + 4 (lane >> 4) + i, i.e. f = 8 mt + 2 (lane >> 4) + i / 2
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = 8 * mt + 2 * (lane >> 4) + h;
      if (f >= g.nf) continue;
      float2* out = ghat + ((size_t)f * g.nr + r0 + r) * g.nsub;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = col + j;
        if (x < g.nsub) {
          float2 v = make_float2(acc[mt][j][2 * h], acc[mt][j][2 * h + 1]);
          if (!first) {
            const float2 o = out[x];
            v.x += o.x;
            v.y += o.y;
          }
          out[x] = v;
        }
      }
    }
}

}  // namespace

int march_bands(const Geometry& g) { return cdiv(g.X, kBand - 4 * g.tblock); }

hipError_t launch_march(const Geometry& g, const float* ca, const float* bd, const float* uin,
                        const float* win, float* uout, float* wout, float* stage, int slot0,
                        int nlev, int nrb_now, hipStream_t st) {
  if (g.nb > kMaxSponge) return hipErrorInvalidValue;
  dim3 grid(march_bands(g), cdiv(g.Z, g.seg_rows), nrb_now);
  switch (g.tblock) {
    case 2:
      hipLaunchKernelGGL(k_march<2>, grid, dim3(kBand), 0, st, g, ca, bd, uin, win, uout, wout,
                         stage, slot0, nlev);
      break;
    case 4:
      hipLaunchKernelGGL(k_march<4>, grid, dim3(kBand), 0, st, g, ca, bd, uin, win, uout, wout,
                         stage, slot0, nlev);
      break;
    case 8:
      hipLaunchKernelGGL(k_march<8>, grid, dim3(kBand), 0, st, g, ca, bd, uin, win, uout, wout,
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
  dim3 grid(cdiv(g.nsub, 256), nrb_now);
  const int fi = first ? 1 : 0;
  const int mt = cdiv(2 * g.nf, 16);
#define EHI_DFT(M)                                                                             \
  hipLaunchKernelGGL(k_dft_mfma<M>, grid, dim3(256), 0, st, g, stage, tw, n0, cnt, fi, r0, ghat); \
  break;
  switch (mt) {
    case 1: EHI_DFT(1)
    case 2: EHI_DFT(2)
    case 3: EHI_DFT(3)
    case 4: EHI_DFT(4)
    case 5:
    case 6: EHI_DFT(6)
    case 7:
    case 8: EHI_DFT(8)
    default:
      return hipErrorInvalidValue;
  }
#undef EHI_DFT
  return hipGetLastError();
}

}  // namespace ehi
