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
// Grid: (bands, row segments, receiver groups of R).  A segment owns output
// rows [z0, z1) and starts marching 2T rows above z0: level t is exact on rows
// >= z0 - 2T + 2t, so every level is exact on the owned rows.  A thread carries
// R receivers of the same column, which share the coefficients and all index
// and control work.
template <int T, int R>
struct March {
  static constexpr int B = kBand - 4 * T;  // output columns per band
  static constexpr int CR = 2 * T + 2;     // rows of the ca ring (reuse distance 2T + 1 barriers)
  static constexpr int W = kBand + 4;      // LDS row incl. two zero columns per side

  struct Shared {
    float lu[2][R][T][W];
    float lc[CR][kBand];
    float lb[kMaxSponge + 1];
  };

  // per-thread state
  float uw[R][T][5];  // uw[j][t]: level-t rows q-2..q+2 for the level-(t+1) update of row q
  float wd[R][T][3];  // wd[j][t]: level-t w of rows q..q+2
  float pu[R][3], pw[R][3], pc[3];  // two-row prefetch queue of level-0 inputs

  template <int N>
  __device__ __forceinline__ static void push(float (&a)[N], float v) {
#pragma unroll
    for (int i = 0; i < N - 1; ++i) a[i] = a[i + 1];
    a[N - 1] = v;
  }

  // One marched row k; BUF is (k - kb) & 1.  Row, level and receiver
  // conditions are uniform across the workgroup (scalar branches); per-lane
  // conditions are folded into precomputed masks.  Columns outside the grid
  // carry ca = 0 and zero fields, so they stay exactly zero without masking.
  template <int BUF>
  __device__ __forceinline__ void row(Shared& sh, const Geometry& g, int k, int ring, int tid,
                                      bool colv, bool own, bool lane_stg, int dxs, int sx, int z0,
                                      int z1, int nlev, int slot0, const float* const (&ui)[R],
                                      const float* const (&wi)[R], const float* cap,
                                      float* const (&uo)[R], float* const (&wo)[R],
                                      float* const (&st)[R], int nrv) {
    const int Z = g.Z;
    const size_t P = g.Xp;
    {  // prefetch row k + 2 (addresses are clamped in range; invalid lanes select 0)
      const int rowp = k + 2;
      if (rowp >= 0 && rowp < Z) {
        const size_t o = (size_t)(rowp + kGhost) * P;
        const float cv = cap[o];
        pc[2] = colv ? cv : 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const float uv = ui[j][o], wv = wi[j][o];
          pu[j][2] = colv ? uv : 0.f;
          pw[j][2] = colv ? wv : 0.f;
        }
      } else {
        pc[2] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) pu[j][2] = pw[j][2] = 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      push(uw[j][0], pu[j][0]);
      push(wd[j][0], pw[j][0]);
      sh.lu[BUF][j][0][tid + 2] = uw[j][0][2];
#pragma unroll
      for (int t = 1; t < T; ++t) sh.lu[BUF][j][t][tid + 2] = uw[j][t][3];
    }
    sh.lc[ring][tid] = pc[0];
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= T; ++t) {
      const int q = k - 2 * t;
      float un[R], wn[R];
#pragma unroll
      for (int j = 0; j < R; ++j) un[j] = wn[j] = 0.f;
      if (q >= 0 && q < Z) {
        if (t <= nlev) {
          int slot = ring - 2 * t;
          if (slot < 0) slot += CR;
          const float a = sh.lc[slot][tid];
          const int dzs = max(max(g.nb - q, q - (g.nb + g.nz - 1)), 0);
          const float bq = sh.lb[max(dzs, dxs)];
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const float* L = sh.lu[BUF][j][t - 1];
            const float cen = uw[j][t - 1][2];
            const float n1 = (L[tid + 1] + L[tid + 3]) + (uw[j][t - 1][1] + uw[j][t - 1][3]);
            const float n2 = (L[tid] + L[tid + 4]) + (uw[j][t - 1][0] + uw[j][t - 1][4]);
            const float lap = 16.f * n1 - n2 - 60.f * cen;
            wn[j] = bq * wd[j][t - 1][0] + a * lap;
            un[j] = cen + wn[j];
          }
          const int jz = q - g.nb;
          if (q >= z0 && q < z1 && jz >= 0 && jz < g.nz && (jz & (g.stride - 1)) == 0) {
            const size_t so = (size_t)(slot0 + t - 1) * g.nsub_p + (size_t)(jz >> g.sshift) * g.nxs + sx;
#pragma unroll
            for (int j = 0; j < R; ++j)
              if (j < nrv && lane_stg) st[j][so] = un[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < R; ++j) {
            un[j] = uw[j][t - 1][2];
            wn[j] = wd[j][t - 1][0];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (t < T) {
          push(uw[j][t], un[j]);
          push(wd[j][t], wn[j]);
        }
      }
      if (t == T && q >= z0 && q < z1) {
        const size_t o = (size_t)(q + kGhost) * P;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (j < nrv && own) {
            uo[j][o] = un[j];
            wo[j][o] = wn[j];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      pu[j][0] = pu[j][1];
      pw[j][0] = pw[j][1];
      pu[j][1] = pu[j][2];
      pw[j][1] = pw[j][2];
    }
    pc[0] = pc[1];
    pc[1] = pc[2];
  }
};

template <int T, int R>
__global__ void __launch_bounds__(kBand)
    k_march(Geometry g, const float* __restrict__ ca, const float* __restrict__ bd,
            const float* __restrict__ uin, const float* __restrict__ win, float* __restrict__ uout,
            float* __restrict__ wout, float* __restrict__ stage, int slot0, int nlev, int nrb_now) {
  using M = March<T, R>;
  __shared__ typename M::Shared sh;
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * M::B - 2 * T;  // padded-grid column of thread 0
  const int c = x0 + tid;
  const bool colv = (c >= 0 && c < g.X);
  const bool own = (tid >= 2 * T && tid < kBand - 2 * T && colv);
  const int Z = g.Z;
  const int z0 = blockIdx.y * g.seg_rows;
  const int z1 = min(Z, z0 + g.seg_rows);
  const int kb = z0 - 2 * T;
  const size_t plane = g.plane();
  // column offset inside a plane row, clamped into the grid so every load is in range
  const size_t cofs = (size_t)(min(max(c, 0), g.X - 1) + kGhost);
  const int nrv = min(R, nrb_now - (int)blockIdx.z * R);  // valid receivers of this group
  const float* ui[R];
  const float* wi[R];
  float* uo[R];
  float* wo[R];
  float* st[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int rr = j < nrv ? (int)blockIdx.z * R + j : 0;
    ui[j] = uin + (size_t)rr * plane + cofs;
    wi[j] = win + (size_t)rr * plane + cofs;
    uo[j] = uout + (size_t)rr * plane + cofs;
    wo[j] = wout + (size_t)rr * plane + cofs;
    st[j] = stage + (size_t)rr * g.chunk * g.nsub_p;
  }
  const float* cap = ca + cofs;
  const int jx = c - g.nb;
  const int sx = (jx >= 0 && jx < g.nx && (jx & (g.stride - 1)) == 0) ? (jx >> g.sshift) : 0;
  const bool lane_stg = own && jx >= 0 && jx < g.nx && (jx & (g.stride - 1)) == 0;
  const int dxs = max(max(g.nb - c, c - (g.nb + g.nx - 1)), 0);  // sponge distance in x

  if (tid < 2) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          sh.lu[b][j][t][tid] = 0.f;
          sh.lu[b][j][t][kBand + 2 + tid] = 0.f;
        }
  }
#pragma unroll
  for (int i = 0; i < M::CR; ++i) sh.lc[i][tid] = 0.f;
  for (int i = tid; i <= g.nb; i += kBand) sh.lb[i] = bd[i];

  M m;
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int i = 0; i < 5; ++i) m.uw[j][t][i] = 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) m.wd[j][t][i] = 0.f;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int rowp = kb + i;
    const bool ok = colv && rowp >= 0 && rowp < Z;
    const size_t o = (size_t)(min(max(rowp, 0), Z - 1) + kGhost) * g.Xp;
    const float cv = cap[o];
    m.pc[i] = ok ? cv : 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const float uv = ui[j][o], wv = wi[j][o];
      m.pu[j][i] = ok ? uv : 0.f;
      m.pw[j][i] = ok ? wv : 0.f;
    }
  }

  const int ke = z1 + 2 * T;
  int ring = 0;  // (k - kb) % CR
  for (int k = kb; k < ke; k += 2) {
    m.template row<0>(sh, g, k, ring, tid, colv, own, lane_stg, dxs, sx, z0, z1, nlev, slot0, ui, wi,
                      cap, uo, wo, st, nrv);
    ring = (ring + 1 == M::CR) ? 0 : ring + 1;
    if (k + 1 < ke) {
      m.template row<1>(sh, g, k + 1, ring, tid, colv, own, lane_stg, dxs, sx, z0, z1, nlev, slot0,
                        ui, wi, cap, uo, wo, st, nrv);
      ring = (ring + 1 == M::CR) ? 0 : ring + 1;
    }
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
  dim3 grid(march_bands(g), cdiv(g.Z, g.seg_rows), cdiv(nrb_now, g.rpt));
#define EHI_MARCH(TT, RR)                                                                     \
  if (g.tblock == TT && g.rpt == RR) {                                                        \
    hipLaunchKernelGGL((k_march<TT, RR>), grid, dim3(kBand), 0, st, g, ca, bd, uin, win, uout, \
                       wout, stage, slot0, nlev, nrb_now);                                    \
    return hipGetLastError();                                                                 \
  }
  EHI_MARCH(4, 1)
  EHI_MARCH(4, 2)
  EHI_MARCH(8, 1)
  EHI_MARCH(8, 2)
#undef EHI_MARCH
  return hipErrorInvalidValue;
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
