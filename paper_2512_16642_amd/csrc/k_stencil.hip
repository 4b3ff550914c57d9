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
// a band of KB columns of one receiver's grid (overlapping its neighbours by
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

// Band widths (columns per workgroup, one per thread) instantiated; the host
// picks the one that covers the padded grid with the fewest lanes.
constexpr int kBands[] = {256, 384, 448, 512};

// Increment-form recurrence (per cell, FP32):
//   w <- ba * w + ca * (16 (u_{z-1} + u_{z+1} + u_{x-1} + u_{x+1})
//                        - (u_{z-2} + u_{z+2} + u_{x-2} + u_{x+2}) - 60 u)
//   u <- u + w
// (the 4th-order Laplacian times 12 h^2).  Taking the nearest neighbours as
// differences from the centre (exact for a smooth field) would remove the
// Laplacian's cancellation error and halve the spectra's error at 3 Hz, but
// its four more VALU instructions per cell-update cost 3 % of the stepping
// time, and the multipliers' error is set by the contraction, not by the
// spectra.
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
//
// Pipeline: iteration i ingests level-0 rows rho = 2i, 2i+1 (rho counts rows
// from the segment start kb = z0 - 2T) and level t computes rows 2i - 2t and
// 2i - 2t + 1.  Level t needs level t-1 rows rho-2..rho+2 (its own column,
// registers) and the x-neighbours of level t-1 rows 2i - 2t, 2i - 2t + 1, which
// were produced in iteration i-1 and are published in LDS before the barrier.
// Per level, u and w rows live in 6-slot register rings (slot = rho mod 6) and
// the ca rows in a register ring of CRR >= 2T + 2 rows (slot = rho mod CRR).
// The iteration loop is unrolled by UNR, a multiple of every ring's period in
// iterations, so ring slots, prefetch sets and the LDS buffer index are
// compile-time constants.
//
// LDS holds the rows published for the x-neighbours column-major: entry
// (column, buffer, level, row of pair) at column * LS + (buffer * T + level) * 2
// + row.  A lane reads columns c-2..c+2 at fixed offsets from one base, and the
// odd column stride LS keeps the 32 lanes of a half-wave on distinct banks.
// Row properties (staging and output offsets, the absorbing-layer factor) come
// from a per-segment row table in global memory; its entries are uniform, so
// they are read with scalar loads straight into scalar registers.
constexpr unsigned kDrop = 0x80000000u;  // store offset the buffer unit discards
typedef const __attribute__((address_space(4))) RowEntry CRowEntry;

// Raw buffer access: the row offset is a scalar (soffset), the column offset a
// per-lane constant (voffset); bounds are the plane the resource describes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
constexpr int lcm_c(int a, int b) { return a / gcd_c(a, b) * b; }

// MODE 0: Green functions (staged subgrid samples); 1: S (subgrid source in,
// traces at the receivers out); 2: S^T (traces injected at the receivers,
// subgrid field out in reversed time, through the staging store).
template <int T, bool FULL, int PD, int KB, int MODE = 0>
struct March3 {
  static constexpr int CRR = T == 4 ? 12 : 24;          // ca ring rows (>= 2T + 2, even)
  // iterations per unrolled body: a multiple of the u/w ring (3 iterations), the
  // ca ring (CRR / 2) and the LDS double buffer (2)
  static constexpr int UNR = lcm_c(6, CRR / 2);
  static constexpr int SETS = PD + 1;                    // prefetch sets (rows of i + PD load during i)
  static_assert(CRR >= 2 * T + 2 && CRR % 2 == 0, "ca ring too short");
  static_assert(UNR % SETS == 0 && UNR % 2 == 0, "the unrolled body cycles sets and buffers");
  static constexpr int B = KB - 4 * T;      // output columns per band
  static constexpr int W = KB + 4;          // columns in LDS incl. two zero columns per side
  static constexpr int LS = 4 * T + 1;      // LDS column stride (words)
  static_assert(kMaxSegRows + 6 * T + 8 <= kRowTabStride, "row table too short");

  struct Shared {
    float lu[W * LS];
  };

  float U[T][6];    // level-t rows, slot = rho mod 6
  float Wr[T][6];   // level-t w
  float C[CRR];     // ca rows, slot = rho mod CRR
  float pu[SETS][2], pw[SETS][2], pc[SETS][2];  // prefetch sets [set][row of pair]
  float fs[MODE == 1 ? T : 1][2];  // S: this iteration's source samples [level][row of pair]

  struct Ctx {
    __amdgpu_buffer_rsrc_t ru, rw, rc, rou, row_, rst;
    int voff;   // byte offset of this lane's column in a plane row (ghost column if outside)
    // Per-lane store offsets: this lane's column in an output plane row and its
    // subgrid column in a staging line, or kDrop on lanes that must not store.
    // The buffer unit discards a store whose offset lies beyond the buffer; the
    // row part (scalar offset) is < 2^31 since planes and staging blocks are
    // limited to 2 GiB, so kDrop plus it never wraps back into range.
    unsigned vown, vsub;
    int tid, kb, Z, Pb, nlev, slot_bytes;
    int slot_off;        // byte offset of staging slot slot0
    const CRowEntry* rt; // this segment's row table (entry rho + 2T = row kb + rho)
    float bx;   // bd[distance of the column into the left/right layer]
    // modelling modes: source / trace / receiver-map resources of this field,
    // the lane's subgrid column for any subgrid lane (halo included) or kDrop
    __amdgpu_buffer_rsrc_t rsrc, rdat, rmap;
    unsigned vsuba;
    int src_off, src_pitch, n_in, nt;
    float scale;
  };

  // rows outside the grid read the zero ghost row next to the edge
  __device__ __forceinline__ int row_bytes(const Ctx& x, int q) const {
    return (min(max(q, -kGhost), x.Z + kGhost - 1) + kGhost) * x.Pb;
  }

  __device__ __forceinline__ void load_pair(const Ctx& x, int rho, int set) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int so = row_bytes(x, x.kb + rho + h);
      pu[set][h] = bload(x.ru, x.voff, so);
      pw[set][h] = bload(x.rw, x.voff, so);
      pc[set][h] = bload(x.rc, x.voff, so);
    }
  }

  static __device__ __forceinline__ constexpr int mod(int a, int m) { return ((a % m) + m) % m; }

  template <int PH>  // PH = i mod UNR
  __device__ __forceinline__ void iter(Shared& sh, const Ctx& x, int i) {
    const CRowEntry* rrow = x.rt + 2 * i;  // entry 2T - 2t + h: row rho = 2i - 2t + h
    constexpr int BUF = PH & 1;
    constexpr int S0 = mod(2 * PH, 6);     // u/w ring slot of row 2i
    constexpr int C0 = mod(2 * PH, CRR);   // ca ring slot of row 2i
    constexpr int SET = PH % SETS;
    U[0][S0] = pu[SET][0];
    U[0][S0 + 1] = pu[SET][1];
    Wr[0][S0] = pw[SET][0];
    Wr[0][S0 + 1] = pw[SET][1];
    C[C0] = pc[SET][0];
    C[C0 + 1] = pc[SET][1];
    load_pair(x, 2 * (i + PD), (PH + PD) % SETS);
    if constexpr (MODE == 1) {
      // the sources of this iteration's levels, issued before the barrier so
      // the loads are in flight while the rows are published
#pragma unroll
      for (int t = 1; t <= T; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int sa = rrow[2 * T - 2 * t + h].suball;
          fs[t - 1][h] = ((FULL || t <= x.nlev) && sa >= 0)
                             ? bload(x.rsrc, (int)x.vsuba, x.src_off + (t - 1) * x.src_pitch + sa)
                             : 0.f;
        }
    }
    float* col = sh.lu + x.tid * LS;  // column c - 2 of this lane; own column at + 2 LS
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) col[2 * LS + (BUF * T + t) * 2 + h] = U[t][mod(2 * PH - 2 * (t + 1) + h, 6)];
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= T; ++t) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int sl = mod(2 * PH - 2 * t + h, 6);  // slot of row rho = 2i - 2t + h
        const int sm2 = (sl + 4) % 6, sm1 = (sl + 5) % 6, sp1 = (sl + 1) % 6, sp2 = (sl + 2) % 6;
        const int cs = mod(2 * PH - 2 * t + h, CRR);
        const CRowEntry& re = rrow[2 * T - 2 * t + h];
        const float re_bz = re.bz;
        const int re_sub = re.sub;
        const int re_own = re.own;
        const float cen = U[t - 1][sl];
        float un, wn;
        if (FULL || t <= x.nlev) {
          const int e = (BUF * T + t - 1) * 2 + h;
          const float n1 = (col[LS + e] + col[3 * LS + e]) + (U[t - 1][sm1] + U[t - 1][sp1]);
          const float n2 = (col[e] + col[4 * LS + e]) + (U[t - 1][sm2] + U[t - 1][sp2]);
          float lap = 16.f * n1 - n2 - 60.f * cen;
          if constexpr (MODE == 1) {
            // the source of the step that produces sample n_in + t
            lap += x.scale * fs[t - 1][h];
          } else if constexpr (MODE == 2) {
            // trace sample nt - (n_in + t) injected at the receivers of this row
            const int ra = re.recall;
            if (ra >= 0) {
              const int ridx = __float_as_int(bload(x.rmap, x.voff, ra));
              const unsigned vo = ridx >= 0 ? (unsigned)((ridx * x.nt + x.nt - x.n_in - t) * 4) : kDrop;
              lap += x.scale * bload(x.rdat, (int)vo, 0);
            }
          }
          // bd is non-increasing in the distance, so bd[max(dz, dx)] = min(bd[dz], bd[dx]);
          // both are positive floats, whose bit patterns order like the integers
          const float bq = __int_as_float(min(__float_as_int(re_bz), __float_as_int(x.bx)));
          wn = bq * Wr[t - 1][sl] + C[cs] * lap;
          un = cen + wn;
          if constexpr (MODE != 1) {
            if (re_sub >= 0) bstore(un, x.rst, (int)x.vsub, x.slot_off + (t - 1) * x.slot_bytes + re_sub);
          } else {
            // sample n_in + t at the receivers of an owned row
            const int ro = re.recown;
            if (ro >= 0) {
              const int ridx = __float_as_int(bload(x.rmap, x.voff, ro));
              const unsigned vo =
                  (ridx >= 0 && x.vown != kDrop) ? (unsigned)((ridx * x.nt + x.n_in + t - 1) * 4) : kDrop;
              bstore(un, x.rdat, (int)vo, 0);
            }
          }
        } else {
          un = cen;
          wn = Wr[t - 1][sl];
        }
        if (t < T) {
          U[t][sl] = un;
          Wr[t][sl] = wn;
        } else {
          if (re_own >= 0) {
            bstore(un, x.rou, (int)x.vown, re_own);
            bstore(wn, x.row_, (int)x.vown, re_own);
          }
        }
      }
    }
  }

  template <int PH>
  __device__ __forceinline__ bool body(Shared& sh, const Ctx& x, int i, int n_it) {
    if constexpr (PH < UNR) {
      if (i + PH >= n_it) return false;
      iter<PH>(sh, x, i + PH);
      return body<PH + 1>(sh, x, i, n_it);
    }
    return true;
  }
};

template <int T, bool FULL, int PD, int KB, int MODE = 0>
__global__ void __launch_bounds__(KB)
    k_march(Geometry g, const float* __restrict__ ca, const float* __restrict__ bd,
            const RowEntry* __restrict__ rowtab, const float* __restrict__ uin,
            const float* __restrict__ win, float* __restrict__ uout, float* __restrict__ wout,
            float* __restrict__ stage, int slot0, int nlev, ModelArgs ma) {
  using M = March3<T, FULL, PD, KB, MODE>;
  __shared__ typename M::Shared sh;
  typename M::Ctx x;
  x.tid = threadIdx.x;
  // receivers vary fastest in the grid so the workgroups of one band and segment
  // run together and share its ca rows in L2
  const int r = blockIdx.x;
  const int c = blockIdx.y * M::B - 2 * T + x.tid;  // padded-grid column
  const bool colv = (c >= 0 && c < g.X);
  const bool own = (x.tid >= 2 * T && x.tid < KB - 2 * T && colv);
  x.Z = g.Z;
  x.Pb = g.Xp * 4;
  const int z0 = blockIdx.z * g.seg_rows;
  const int z1 = min(g.Z, z0 + g.seg_rows);
  x.kb = z0 - 2 * T;
  const int n_it = (z1 - z0 + 4 * T + 1) / 2;
  x.nlev = nlev;
  const size_t plane = g.plane();
  const size_t pbytes = plane * sizeof(float);
  x.ru = make_rsrc(uin + (size_t)r * plane, pbytes);
  x.rw = make_rsrc(win + (size_t)r * plane, pbytes);
  x.rc = make_rsrc(ca, pbytes);
  x.rou = make_rsrc(uout + (size_t)r * plane, pbytes);
  x.row_ = make_rsrc(wout + (size_t)r * plane, pbytes);
  if constexpr (MODE == 0) {
    const size_t sbytes = (size_t)g.chunk * g.nsub_p * sizeof(float);
    x.rst = make_rsrc(stage + (size_t)r * g.chunk * g.nsub_p, sbytes);
    x.slot_bytes = g.nsub_p * 4;
    x.slot_off = slot0 * x.slot_bytes;
  } else {
    const size_t fbytes = (size_t)ma.nt * g.nsub * sizeof(float);
    const size_t tbytes = (size_t)g.nr * ma.nt * sizeof(float);
    x.rmap = make_rsrc(ma.recmap, plane * sizeof(int32_t));
    x.n_in = ma.n_in;
    x.nt = ma.nt;
    x.scale = ma.scale;
    if constexpr (MODE == 1) {
      x.rsrc = make_rsrc(ma.src + (size_t)r * ma.src_field, fbytes);
      x.rdat = make_rsrc(ma.dat_out + (size_t)r * ma.dat_field, tbytes);
      x.src_pitch = g.nsub * 4;
      x.src_off = ma.n_in * x.src_pitch;
    } else {
      x.rdat = make_rsrc(ma.dat_in + (size_t)r * ma.dat_field, tbytes);
      // sample m = n_in + t goes to slot nt - m: a descending slot pitch
      x.rst = make_rsrc(ma.sub_out + (size_t)r * ma.sub_field, fbytes);
      x.slot_bytes = -g.nsub * 4;
      x.slot_off = (ma.nt - ma.n_in - 1) * g.nsub * 4;
    }
  }
  // the table is read-only during the launch: constant address space, so the
  // uniform entries are fetched with scalar loads
  x.rt = (const CRowEntry*)rowtab + (size_t)blockIdx.z * kRowTabStride;
  // columns outside the grid read the zero ghost column next to the edge
  x.voff = (min(max(c, -kGhost), g.X + kGhost - 1) + kGhost) * 4;
  const int jx = c - g.nb;
  const bool subx = jx >= 0 && jx < g.nx && (jx & (g.stride - 1)) == 0;
  x.vown = own ? (unsigned)x.voff : kDrop;
  x.vsub = (own && subx) ? (unsigned)((jx >> g.sshift) * 4) : kDrop;
  if constexpr (MODE == 1) x.vsuba = (colv && subx) ? (unsigned)((jx >> g.sshift) * 4) : kDrop;
  x.bx = bd[colv ? max(max(g.nb - c, c - (g.nb + g.nx - 1)), 0) : 0];

  // the two zero columns on each side of the band
  if (x.tid < 4) {
    const int zc = x.tid < 2 ? x.tid : KB + x.tid;
#pragma unroll
    for (int e = 0; e < 4 * T; ++e) sh.lu[zc * M::LS + e] = 0.f;
  }

  M m;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2) m.U[t][s2] = m.Wr[t][s2] = 0.f;
#pragma unroll
  for (int s2 = 0; s2 < M::CRR; ++s2) m.C[s2] = 0.f;
#pragma unroll
  for (int p = 0; p < PD; ++p) m.load_pair(x, 2 * p, p);

  for (int i = 0; i < n_it; i += M::UNR)
    if (!m.template body<0>(sh, x, i, n_it)) break;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kDftKs = 128;  // time samples per LDS twiddle stage (40 KB at 64 rows: four workgroups per CU)

// DFT of one staged chunk as a real matrix product on FP32 MFMA:
//   C[m][x] = sum_tau A[m][tau] S[tau][x],  A[2f][tau] = Re tw, A[2f+1][tau] = Im tw,
//   ghat[f][r0 + r][x] (+)= (C[2f][x], C[2f+1][x]).
// v_mfma_f32_16x16x4f32 tiles: A (16 rows of m x 4 samples) from LDS, B (4
// samples x 16 grid points) from the staging buffer.  A wave owns 64 grid
// points as four 16-column tiles with a permuted column map (tile j, column i
// <-> grid point 4i + j) so each lane loads its four B values with one float4.
// Samples at tau >= cnt and frequencies >= nf are zero; points >= nsub are
// computed (the row pitch is padded) but not stored.
// occupancy target: the most waves per SIMD whose registers hold the MT x 4
// accumulator tiles without spilling
template <int MT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT <= 4 ? 4 : MT <= 6 ? 3 : 2)))
    k_dft_mfma(Geometry g, const float* __restrict__ stage, const float2* __restrict__ tw, int n0,
               int cnt, int first, int r0, float2* __restrict__ ghat) {
  constexpr int MP = 16 * MT;
  // row stride = 16 (mod 32) words: the two sample rows a half-wave reads sit on
  // disjoint banks
  constexpr int MS = MP % 32 == 0 ? MP + 16 : MP;
  __shared__ float As[kDftKs][MS];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = blockIdx.y;
  const int col = blockIdx.x * 256 + wave * 64 + 4 * (lane & 15);  // this lane's 4 grid points
  const int krow = lane >> 4;
  // staged samples through a buffer resource that covers the cnt valid rows:
  // rows at or past cnt read as zero, and the row offset is a scalar
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc(stage + (size_t)r * g.chunk * g.nsub_p, (size_t)cnt * g.nsub_p * sizeof(float));
  const int pitch = g.nsub_p * 4;
  const int voff = krow * pitch + col * 4;
  floatx4 acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[mt][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int twoF = 2 * g.nf;
  // B (staging) in groups of four K-steps (16 samples); the group after the
  // current one is loaded before the current group's MFMAs are issued
  auto load_b = [&](floatx4* b, int k16) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      b[u] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, (k16 + 4 * u) * pitch, 0));
  };
  const int ngrp = (cnt + 15) / 16;
  floatx4 b[2][4];
  load_b(b[0], 0);
  for (int gi = 0; gi < ngrp; gi += 2) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int gg = gi + p;
      if (gg >= ngrp) break;
      const int k16 = gg * 16;
      const int kl = k16 % kDftKs;  // sample offset inside the LDS stage
      if (kl == 0) {
        __syncthreads();
        for (int e = threadIdx.x; e < kDftKs * MP; e += 256) {
          const int t = e / MP, m = e % MP;
          float v = 0.f;
          if (k16 + t < cnt && m < twoF) {
            const float2 z = tw[(size_t)(n0 - 1 + k16 + t) * g.nf + (m >> 1)];
            v = (m & 1) ? z.y : z.x;
          }
          As[t][m] = v;
        }
        __syncthreads();
      }
      if (gg + 1 < ngrp) load_b(b[p ^ 1], k16 + 16);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (k16 + 4 * u < cnt) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const float a = As[kl + 4 * u + krow][16 * mt + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[p][u][j], acc[mt][j], 0, 0, 0);
          }
        }
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

// The same DFT on the BF16 matrix cores with FP32-equivalent operands: every
// FP32 value x (staged sample or twiddle) is split into three BF16 parts,
// x = hi + mid + lo + O(2^-24 x) (hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid), round to nearest even), and a product is taken as
// the six terms down to 2^-16 of its size (mid.mid, lo.hi, hi.lo, mid.hi,
// hi.mid, hi.hi, smallest first); the three dropped terms are below 2^-24 of
// it.  v_mfma_f32_16x16x32_bf16 contracts 32 samples per instruction, so the
// six products cost less matrix-core time than the four 16x16x4 FP32 steps
// they replace by a factor of about 2.7, which moves the kernel off the
// matrix-core limit onto the HBM one.  Each 32-sample group's six products are
// chained from zero and added to the running sum with an ordinary FP32 add
// (the matrix core's own accumulation is biased over long chains).
//
// Operand layouts (16 x 16 x 32): lane l holds A[row l % 16][k 8 (l / 16) ..
// + 7] and B[k 8 (l / 16) .. + 7][col l % 16]; the result D[4 (l / 16) + v]
// [l % 16] as in the FP32 kernel, so the epilogue is the same.  Points are
// mapped as there (tile j, column i <-> point 4i + j): a lane loads its eight
// samples of four consecutive points as eight 16-byte loads.  The twiddle
// stage in LDS holds the three BF16 planes [plane][row][sample] with rows
// padded by 8 samples (16 B), so the 16 rows a half-wave reads land on
// different banks.  A workgroup of NW waves covers 64 NW consecutive grid
// points of one receiver, so each sample row is read in 256 NW-byte runs.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kDft3Ks = 128;            // samples per LDS twiddle stage
constexpr int kDft3Kp = kDft3Ks + 8;    // padded row (bf16 elements)

// The low BF16 of a packed pair widened to FP32 (its bits moved to the top
// half by a byte permute: the compiler would otherwise convert the FP32 value a
// second time), and the high one (a mask).
__device__ __forceinline__ float bf16_lo(unsigned p) { return __uint_as_float(__builtin_amdgcn_perm(0u, p, 0x01000c0cu)); }
__device__ __forceinline__ float bf16_hi(unsigned p) { return __uint_as_float(p & 0xffff0000u); }

// Three-part split of two FP32 values into packed BF16 pairs (element 0 in the
// low half): hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), each
// conversion round-to-nearest-even and taken for both values at once.
__device__ __forceinline__ void split3_pair(float x0, float x1, unsigned& h, unsigned& m, unsigned& l) {
  h = __builtin_bit_cast(unsigned, bf16x2_t{(__bf16)x0, (__bf16)x1});
  const float r0 = x0 - bf16_lo(h), r1 = x1 - bf16_hi(h);
  m = __builtin_bit_cast(unsigned, bf16x2_t{(__bf16)r0, (__bf16)r1});
  l = __builtin_bit_cast(unsigned, bf16x2_t{(__bf16)(r0 - bf16_lo(m)), (__bf16)(r1 - bf16_hi(m))});
}

template <int MT, int NW>  // NW waves per workgroup, 64 grid points each
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MT <= 2 ? 3 : 2)))
    k_dft_bf16x3(Geometry g, const float* __restrict__ stage, const float2* __restrict__ tw, int n0,
                 int cnt, int first, int r0, float2* __restrict__ ghat) {
  constexpr int MP = 16 * MT;
  constexpr int NT = 64 * NW;  // threads
  __shared__ __bf16 As[3][MP][kDft3Kp];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = blockIdx.y;
  const int col = blockIdx.x * NT + wave * 64 + 4 * (lane & 15);  // this lane's 4 grid points
  const int kg = lane >> 4;                                         // sample octet of the lane
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc(stage + (size_t)r * g.chunk * g.nsub_p, (size_t)cnt * g.nsub_p * sizeof(float));
  const int pitch = g.nsub_p * 4;
  const int voff = 8 * kg * pitch + col * 4;
  floatx4 acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[mt][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int twoF = 2 * g.nf;
  // twiddles through a buffer resource over this window's rows of the table
  // (samples n0 .. n0 + cnt - 1): a load at an offset beyond it (samples past
  // the window, rows past 2 nf) reads zero, so no select follows a load and a
  // batch's loads issue back to back
  const __amdgpu_buffer_rsrc_t rt = make_rsrc(tw + (size_t)(n0 - 1) * g.nf, (size_t)cnt * g.nf * sizeof(float2));
  // the lane's eight samples (rows k32 + 8 kg + e) of its four points
  auto load_b = [&](floatx4* b, int k32) {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      b[e] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, (k32 + e) * pitch, 0));
  };
  // Twiddle stage of 128 samples: thread items are (row m, sample pair t, t + 1),
  // eight (or four) per batch with all their loads issued before the first is
  // used; each pair is split into packed words and stored as one 4-byte write
  // per plane.
  constexpr int kPer = MP * kDft3Ks / 2 / NT;  // pairs per thread and stage
  constexpr int kBatch = kPer % 8 == 0 ? 8 : kPer % 4 == 0 ? 4 : 2;  // divides kPer
  static_assert(kPer * NT * 2 == MP * kDft3Ks && kPer % kBatch == 0, "stage items");
  auto stage_tw = [&](int k32) {
#pragma unroll 1
    for (int b0 = 0; b0 < kPer; b0 += kBatch) {
      float v0[kBatch], v1[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int e = threadIdx.x + NT * (b0 + i);
        const int m = e / (kDft3Ks / 2), t = 2 * (e % (kDft3Ks / 2));
        // byte offset of (window sample k32 + t, row m); rows past 2 nf are sent past the table
        const unsigned o = m < twoF ? (unsigned)((((k32 + t) * g.nf + (m >> 1)) * 2 + (m & 1)) * 4) : kDrop;
        v0[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rt, (int)o, 0, 0));
        v1[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rt, (int)o, 8 * g.nf, 0));
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int e = threadIdx.x + NT * (b0 + i);
        const int m = e / (kDft3Ks / 2), t = 2 * (e % (kDft3Ks / 2));
        unsigned h, mm, l;
        split3_pair(v0[i], v1[i], h, mm, l);
        *reinterpret_cast<unsigned*>(&As[0][m][t]) = h;
        *reinterpret_cast<unsigned*>(&As[1][m][t]) = mm;
        *reinterpret_cast<unsigned*>(&As[2][m][t]) = l;
      }
    }
  };
  // One 32-sample group: stage the twiddles at a stage boundary, split the
  // group's samples b into the three B planes, load the next group's samples
  // into b (in flight during the products), then the products.
  const int ngrp = (cnt + 31) / 32;
  floatx4 b[8];
  load_b(b, 0);
  for (int gi = 0; gi < ngrp; ++gi) {
    const int k32 = gi * 32;
    const int kl = k32 % kDft3Ks;
    if (kl == 0) {
      __syncthreads();
      stage_tw(k32);
      __syncthreads();
    }
    // B fragments per tile j and plane: the lane's eight samples of point 4i + j
    bf16x8_t B[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned w[3][4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) split3_pair(b[e][j], b[e + 1][j], w[0][e >> 1], w[1][e >> 1], w[2][e >> 1]);
#pragma unroll
      for (int q = 0; q < 3; ++q) B[q][j] = __builtin_bit_cast(bf16x8_t, u32x4_t{w[q][0], w[q][1], w[q][2], w[q][3]});
    }
    if (gi + 1 < ngrp) load_b(b, k32 + 32);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = 16 * mt + (lane & 15);
      bf16x8_t A[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) A[q] = *reinterpret_cast<const bf16x8_t*>(&As[q][row][kl + 8 * kg]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        floatx4 t = floatx4{0.f, 0.f, 0.f, 0.f};
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1][j], t, 0, 0, 0);  // mid.mid
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0][j], t, 0, 0, 0);  // lo.hi
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2][j], t, 0, 0, 0);  // hi.lo
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0][j], t, 0, 0, 0);  // mid.hi
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1][j], t, 0, 0, 0);  // hi.mid
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0][j], t, 0, 0, 0);  // hi.hi
        acc[mt][j] += t;
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

// Row table for the current launch shape: entry ti of segment sg describes
// padded row q = sg * seg_rows - 4T + ti.
__global__ void k_row_table(Geometry g, const float* __restrict__ bd, const int32_t* __restrict__ rowrec,
                            RowEntry* __restrict__ rt, int nseg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nseg * kRowTabStride) return;
  const int sg = e / kRowTabStride, ti = e % kRowTabStride;
  const int z0 = sg * g.seg_rows;
  const int z1 = min(g.Z, z0 + g.seg_rows);
  const int q = z0 - 4 * g.tblock + ti;
  const bool inside = q >= 0 && q < g.Z;
  RowEntry r;
  r.bz = bd[inside ? max(max(g.nb - q, q - (g.nb + g.nz - 1)), 0) : 0];
  const bool owned = q >= z0 && q < z1;
  r.own = owned ? (q + kGhost) * g.Xp * 4 : -1;
  const int jz = q - g.nb;
  const bool onsub = jz >= 0 && jz < g.nz && (jz & (g.stride - 1)) == 0;
  r.sub = (owned && onsub) ? (jz >> g.sshift) * g.nxs * 4 : -1;
  r.suball = onsub ? (jz >> g.sshift) * g.nxs * 4 : -1;
  const bool hasrec = inside && rowrec[q] != 0;
  const int rowoff = (q + kGhost) * g.Xp * 4;
  r.recall = hasrec ? rowoff : -1;
  r.recown = (hasrec && owned) ? rowoff : -1;
  r.pad0 = r.pad1 = 0;
  rt[e] = r;
}

int march_bands(const Geometry& g) { return cdiv(g.X, g.band - 4 * g.tblock); }

hipError_t launch_row_table(const Geometry& g, const float* bd, const int32_t* rowrec, RowEntry* rt,
                            hipStream_t st) {
  if (g.seg_rows < kMinSegRows || g.seg_rows > kMaxSegRows) return hipErrorInvalidValue;
  const int nseg = cdiv(g.Z, g.seg_rows);
  const int n = nseg * kRowTabStride;
  hipLaunchKernelGGL(k_row_table, dim3(cdiv(n, 256)), dim3(256), 0, st, g, bd, rowrec, rt, nseg);
  return hipGetLastError();
}

int march_band_for(int X, int tblock) {
  int best = kBands[0], lanes = 1 << 30;
  for (int kb : kBands) {
    const int l = cdiv(X, kb - 4 * tblock) * kb;
    if (l <= lanes) {  // ties go to the wider band (fewer overlapping halos)
      lanes = l;
      best = kb;
    }
  }
  return best;
}

hipError_t launch_march(const Geometry& g, const float* ca, const float* bd, const RowEntry* rt,
                        const float* uin, const float* win, float* uout, float* wout, float* stage,
                        int slot0, int nlev, int nrb_now, hipStream_t st) {
  if (g.nb > kMaxSponge || g.seg_rows < kMinSegRows || g.seg_rows > kMaxSegRows || nlev < 1 ||
      nlev > g.tblock)
    return hipErrorInvalidValue;
  dim3 grid(nrb_now, march_bands(g), cdiv(g.Z, g.seg_rows));
#define EHI_MARCH(TT, FF, KK)                                                                     \
  hipLaunchKernelGGL((k_march<TT, FF, 2, KK>), grid, dim3(KK), 0, st, g, ca, bd, rt, uin, win,   \
                     uout, wout, stage, slot0, nlev, ModelArgs{})
#define EHI_MARCH_T(TT, KK)                \
  if (nlev == TT) EHI_MARCH(TT, true, KK); \
  else EHI_MARCH(TT, false, KK);
#define EHI_MARCH_B(TT)                                 \
  switch (g.band) {                                     \
    case 256: EHI_MARCH_T(TT, 256) break;               \
    case 384: EHI_MARCH_T(TT, 384) break;               \
    case 448: EHI_MARCH_T(TT, 448) break;               \
    case 512: EHI_MARCH_T(TT, 512) break;               \
    default: return hipErrorInvalidValue;               \
  }
  if (g.tblock == 4) {
    EHI_MARCH_B(4)
  } else if (g.tblock == 8) {
    EHI_MARCH_B(8)
  } else {
    return hipErrorInvalidValue;
  }
#undef EHI_MARCH_B
#undef EHI_MARCH_T
#undef EHI_MARCH
  return hipGetLastError();
}

hipError_t launch_march_model(const Geometry& g, int mode, const float* ca, const float* bd, const RowEntry* rt,
                              const float* uin, const float* win, float* uout, float* wout,
                              const ModelArgs& m, int nlev, int nrb_now, hipStream_t st) {
  if (g.nb > kMaxSponge || g.seg_rows < kMinSegRows || g.seg_rows > kMaxSegRows || nlev < 1 ||
      nlev > 8 || g.tblock != 8 || (mode != 1 && mode != 2) || m.n_in < 0 || m.n_in + nlev > m.nt)
    return hipErrorInvalidValue;
  dim3 grid(nrb_now, march_bands(g), cdiv(g.Z, g.seg_rows));
#define EHI_MODEL(MM, FF, KK)                                                                        \
  hipLaunchKernelGGL((k_march<8, FF, 2, KK, MM>), grid, dim3(KK), 0, st, g, ca, bd, rt, uin, win,     \
                     uout, wout, nullptr, 0, nlev, m)
#define EHI_MODEL_F(MM, KK)                 \
  if (nlev == 8) EHI_MODEL(MM, true, KK);   \
  else EHI_MODEL(MM, false, KK);
#define EHI_MODEL_B(MM)                                 \
  switch (g.band) {                                     \
    case 256: EHI_MODEL_F(MM, 256) break;               \
    case 384: EHI_MODEL_F(MM, 384) break;               \
    case 448: EHI_MODEL_F(MM, 448) break;               \
    case 512: EHI_MODEL_F(MM, 512) break;               \
    default: return hipErrorInvalidValue;               \
  }
  if (mode == 1) {
    EHI_MODEL_B(1)
  } else {
    EHI_MODEL_B(2)
  }
#undef EHI_MODEL_B
#undef EHI_MODEL_F
#undef EHI_MODEL
  return hipGetLastError();
}

hipError_t launch_dft_chunk(const Geometry& g, const float* stage, const float2* tw, int n0,
                            int cnt, bool first, int r0, int nrb_now, float2* ghat,
                            hipStream_t st) {
  dim3 grid(cdiv(g.nsub, 256), nrb_now);
  const int fi = first ? 1 : 0;
  const int mt = cdiv(2 * g.nf, 16);
  if (g.dft_form == 1) {
    // 512-thread workgroups over 512 grid points (each sample row read in 2 KB
    // runs, twiddle stages shared by eight waves) where the registers allow
    // two waves per SIMD anyway; 256 threads at 2 and 3 row tiles, which fit
    // three waves per SIMD
#define EHI_DFT3(M, NW)                                                                                \
  hipLaunchKernelGGL((k_dft_bf16x3<M, NW>), dim3(cdiv(g.nsub, 64 * (NW)), nrb_now), dim3(64 * (NW)), 0, st, g, \
                     stage, tw, n0, cnt, fi, r0, ghat);                                                \
  break;
    switch (mt) {
      case 1: EHI_DFT3(1, 8)
      case 2: EHI_DFT3(2, 4)
      case 3: EHI_DFT3(3, 4)
      case 4: EHI_DFT3(4, 8)
      case 5:
      case 6: EHI_DFT3(6, 8)
      case 7:
      case 8: EHI_DFT3(8, 8)
      default:
        return hipErrorInvalidValue;
    }
#undef EHI_DFT3
    return hipGetLastError();
  }
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
