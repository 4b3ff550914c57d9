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
// precision mode refinement steps follow (one by default, 0-4 selectable):
// r = R - Qhat X in FP64 (X kept in FP64), X += M^H (M r) in FP32.  These products run on the matrix cores
// (k_cgemm_sk); k_cgemm, a 64 x 64 tiling on FMAs with a choice of B layout
// and of the summation type, serves the DCT passes and the compressed
// contraction.
#include <hip/hip_runtime.h>

#include <algorithm>

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
// Batched complex products on FMAs, one batch entry (frequency) per blockIdx.z:
//   C(i, j) = sum_{k < kdim} op(A)(i, k) B(k, j),  i < n, j < ns
// A (arows rows, row-major): MODE 0: A itself (Qhat, or a transform matrix);
// MODE 1: M (lower, np x np); MODE 2: M^H, i.e. A(i, k) = conj(M(k, i)); MODE 3:
// conj(A) elementwise.  Tiles of M that are zero by triangularity are skipped.  B(k, j) = Bm[j * ldb + k]
// (BT = 0: source-major, as the residuals are stored) or Bm[k * ldb + j]
// (BT = 1).  C(i, j) is stored at C[j * ldc + i].
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
  int n, ns;        // rows of C, columns of C
  int kdim;         // K extent
  int arows;        // rows of A (n for Qhat, np for M)
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

// T: type of the operands in memory and LDS; TA: type of the products and sums.
template <typename T, int MODE, int EPI, int BT = 0, typename TA = T>
__global__ void __launch_bounds__(256) k_cgemm(GemmArgs a) {
  typedef typename Cx<T>::t C2;
  typedef typename Cx<TA>::t A2;
  // two LDS stages: stage k + 1 is loaded into registers while stage k is
  // multiplied, then stored into the other buffer (one barrier per stage)
  __shared__ C2 As[2][kGk][kGm];
  __shared__ C2 Bs[2][kGk][kGn];
  const int f = blockIdx.z;
  const int i0 = blockIdx.y * kGm, j0 = blockIdx.x * kGn;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const C2* A = static_cast<const C2*>(a.A) + (size_t)f * a.sA;
  const C2* B = static_cast<const C2*>(a.B) + (size_t)f * a.sB;
  A2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = A2{0, 0};
  int kbeg = 0, kend = a.kdim;
  if (MODE == 1) kend = min(kend, i0 + kGm);             // M(i, k) = 0 for k > i
  if (MODE == 2) kbeg = i0 / kGk * kGk;                  // conj(M(k, i)) = 0 for k < i
  // element q of this thread's share of a stage: (stage row kk, LDS column)
  // of A and of B; the LDS column keeps the register-tile index outermost
  auto a_slot = [&](int q, int& kk, int& ii) {
    const int e = tid + 256 * q;
    if (MODE == 2) { kk = e / kGm; ii = e % kGm; }      // contiguous along i
    else { ii = e / kGk; kk = e % kGk; }                // contiguous along k
  };
  auto b_slot = [&](int q, int& kk, int& jj) {
    const int e = tid + 256 * q;
    if (BT) { kk = e / kGn; jj = e % kGn; }             // contiguous along j
    else { jj = e / kGk; kk = e % kGk; }                // contiguous along k
  };
  C2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int kk, ii, jj, kb;
      a_slot(q, kk, ii);
      const int gk = k0 + kk, gi = i0 + ii;
      C2 v = C2{0, 0};
      if (gk < kend && gi < a.arows) {
        if (MODE == 2) {
          const C2 m = A[(size_t)gk * a.lda + gi];
          v = C2{m.x, -m.y};
        } else {
          v = A[(size_t)gi * a.lda + gk];
          if (MODE == 3) v.y = -v.y;                     // A(i, k) = conj(Am[i * lda + k])
        }
      }
      ra[q] = v;
      b_slot(q, kb, jj);
      const int hk = k0 + kb, gj = j0 + jj;
      rb[q] = (hk < kend && gj < a.ns) ? (BT ? B[(size_t)hk * a.ldb + gj] : B[(size_t)gj * a.ldb + hk])
                                       : C2{0, 0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int kk, ii, jj, kb;
      a_slot(q, kk, ii);
      As[buf][kk][(ii & 3) * 16 + (ii >> 2)] = ra[q];
      b_slot(q, kb, jj);
      Bs[buf][kb][(jj & 3) * 16 + (jj >> 2)] = rb[q];
    }
  };
  if (kbeg < kend) gload(kbeg);
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kGk, buf ^= 1) {
    sstore(buf);
    __syncthreads();
    if (k0 + kGk < kend) gload(k0 + kGk);
#pragma unroll 4
    for (int kk = 0; kk < kGk; ++kk) {
      A2 av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const C2 v = As[buf][kk][r * 16 + ty];
        av[r] = A2{(TA)v.x, (TA)v.y};
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const C2 v = Bs[buf][kk][c * 16 + tx];
        bv[c] = A2{(TA)v.x, (TA)v.y};
      }
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
      const A2 v = acc[r][c];
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

template <typename T, int MODE, int EPI, int BT = 0, typename TA = T>
hipError_t run_gemm(const GemmArgs& a, int nf, hipStream_t st) {
  dim3 grid(cdiv(a.ns, kGn), cdiv(a.n, kGm), nf);
  hipLaunchKernelGGL((k_cgemm<T, MODE, EPI, BT, TA>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The deblur products on the matrix cores: the same C(i, j) = sum_k op(A)(i, k)
// B(k, j) as k_cgemm (MODE 0, 1 or 2; B source-major; the same epilogues), in
// the operand precision T on v_mfma_f32_16x16x4f32 (T = float) or
// v_mfma_f64_16x16x4f64 (T = double), products and sums in T.
// The matrix cores form the transpose D(j, i) = sum_k B(k, j) op(A)(i, k): row
// index = source j, column index = i, so the 16 lanes of a result row hold 16
// consecutive i, the contiguous index of every output.  A complex product is
// four real ones: Re D = Br Ar - Bi Ai, Im D = Br Ai + Bi Ar (the FP64 form
// takes three, below).
typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef double mf64x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
// Result layout: lane l holds rows row(l / 16, v), v < 4, of column l % 16
// (measured for both instructions on gfx950).
template <> struct Mfma<float> {
  typedef mf32x4 v4;
  static __device__ __forceinline__ int row(int l4, int v) { return 4 * l4 + v; }
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef mf64x4 v4;
  static __device__ __forceinline__ int row(int l4, int v) { return 4 * v + l4; }
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// The epilogues of the matrix-core products: value (vx, vy) of C(i, j) of
// frequency f (see GemmArgs).
template <int EPI>
__device__ __forceinline__ void epi_store(const GemmArgs& a, int f, int j, int i, double vx, double vy) {
  if (EPI == kEpiStore) {
    a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] = make_float2((float)vx, (float)vy);
  } else if (EPI == kEpiResid) {
    const float2 rr = a.R[(size_t)f * a.sR + (size_t)j * a.ldr + i];
    a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] =
        make_float2((float)((double)rr.x - vx), (float)((double)rr.y - vy));
  } else {
    double2* xp = a.X + (size_t)f * a.sX + (size_t)j * a.ldx + i;
    if (EPI == kEpiX64Set) {
      *xp = make_double2(vx, vy);
    } else if (EPI == kEpiX64Add) {
      double2 o = *xp;
      o.x += vx;
      o.y += vy;
      *xp = o;
    } else {  // kEpiOut
      const double2 o = *xp;
      a.C[(size_t)f * a.sC + (size_t)j * a.ldc + i] = make_float2((float)(o.x + vx), (float)(o.y + vy));
    }
  }
}

// The deblur's products (C has as many rows as there are receivers, a few
// hundred), split-K: a 32 x 32 tile of C per workgroup, so the grid holds
// about four times as many workgroups as with 64 x 64 tiles (the form this
// replaced, measured slower at every size from 16 to 400 receivers) and
// triangular tiles are skipped at 32-row granularity.  The tile's K range is dealt out to the
// four waves in slices of 4 (slice m of wave w: k = kbeg + 16 m + 4 w + 0..3),
// each wave accumulating the whole tile (2 x 2 matrix-core tiles of 16 x 16)
// over its slices, with operands read straight from memory (M, Qhat and the
// right-hand sides of one frequency are L2-resident) and kept PF slices
// ahead in registers.  The four partial tiles are then summed through LDS in
// a fixed order, wave w finishing tile (w >> 1, w & 1).  The longest chain of
// dependent matrix-core steps is a quarter of a 64 x 64 tile's.
constexpr int kSkT = 32;

// Operand loads of the split-K products through buffer resources: an offset
// past the resource (rows past the matrix, or kSkDrop for k outside the
// product's K range) reads zero, and the slice's step is a scalar offset, so
// a lane computes its offsets once.
constexpr unsigned kSkDrop = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sk_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename C2> __device__ __forceinline__ C2 sk_load(__amdgpu_buffer_rsrc_t r, unsigned vo, int so);
template <> __device__ __forceinline__ float2 sk_load<float2>(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, so, 0));
}
template <> __device__ __forceinline__ double2 sk_load<double2>(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, so, 0));
}

template <typename T, int MODE, int EPI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_cgemm_sk(GemmArgs a) {
  typedef typename Cx<T>::t C2;
  typedef typename Mfma<T>::v4 V4;
  // FP64 (the refinement residual): each complex product as three real ones,
  // P1 = Br Ar, P2 = Bi Ai, P3 = (Br + Bi)(Ar + Ai), Re = P1 - P2,
  // Im = P3 - P1 - P2 (the cancellation costs a bit or two of FP64's 53);
  // FP32: the four real products
  constexpr bool G3 = sizeof(T) == 8;
  constexpr int PF = G3 ? 2 : 4;        // slices in flight per wave
  __shared__ T red[4][2][2][2][4][64];  // [wave][jt][it][re, im][v][lane]
  const int f = blockIdx.z;
  const int i0 = blockIdx.y * kSkT, j0 = blockIdx.x * kSkT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const C2* A = static_cast<const C2*>(a.A) + (size_t)f * a.sA;
  const C2* B = static_cast<const C2*>(a.B) + (size_t)f * a.sB;
  int kbeg = 0, kend = a.kdim;
  if (MODE == 1) kend = min(kend, i0 + kSkT);  // M(i, k) = 0 for k > i
  if (MODE == 2) kbeg = i0;                    // conj(M(k, i)) = 0 for k < i
  const int nsl = kend > kbeg ? cdiv(kend - kbeg, 16) : 0;  // slices per wave
  V4 dr[2][2], di[2][2];          // [j tile][i tile]; FP64: P1, P2
  V4 d3[G3 ? 2 : 1][G3 ? 2 : 1];  // FP64: P3
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int it = 0; it < 2; ++it) dr[jt][it] = di[jt][it] = V4{0, 0, 0, 0};
#pragma unroll
  for (int jt = 0; jt < (G3 ? 2 : 1); ++jt)
#pragma unroll
    for (int it = 0; it < (G3 ? 2 : 1); ++it) d3[jt][it] = V4{0, 0, 0, 0};
  C2 pa[PF][2], pb[PF][2];
  // resources over this frequency's A (arows x lda) and B (ns x ldb); the
  // lane's byte offsets at slice 0 and the per-slice steps
  constexpr int SZ = (int)sizeof(C2);
  const __amdgpu_buffer_rsrc_t rsa = sk_rsrc(A, (size_t)a.arows * a.lda * SZ);
  const __amdgpu_buffer_rsrc_t rsb = sk_rsrc(B, (size_t)a.ns * a.ldb * SZ);
  const int kl = kbeg + 4 * wave + l4;
  unsigned ao[2], bo[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int gi = i0 + 16 * it + l16;
    ao[it] = (unsigned)((MODE == 2 ? kl * a.lda + gi : gi * a.lda + kl) * SZ);
  }
#pragma unroll
  for (int jt = 0; jt < 2; ++jt) bo[jt] = (unsigned)(((j0 + 16 * jt + l16) * a.ldb + kl) * SZ);
  const int astep = (MODE == 2 ? 16 * a.lda : 16) * SZ, bstep = 16 * SZ;
  auto load = [&](int m, C2 (&ra)[2], C2 (&rb)[2]) {
    const bool kin = kl + 16 * m < kend;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const C2 v = sk_load<C2>(rsa, kin ? ao[it] : kSkDrop, m * astep);
      ra[it] = MODE == 2 ? C2{v.x, -v.y} : v;
    }
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) rb[jt] = sk_load<C2>(rsb, kin ? bo[jt] : kSkDrop, m * bstep);
  };
#pragma unroll
  for (int p = 0; p < PF; ++p) load(p, pa[p], pb[p]);
  for (int m = 0; m < nsl; m += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      if (m + p < nsl) {
        const C2 av[2] = {pa[p][0], pa[p][1]};
        const C2 bv[2] = {pb[p][0], pb[p][1]};
        load(m + p + PF, pa[p], pb[p]);
        if constexpr (G3) {
          const T as[2] = {av[0].x + av[0].y, av[1].x + av[1].y};
          const T bs[2] = {bv[0].x + bv[0].y, bv[1].x + bv[1].y};
#pragma unroll
          for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int it = 0; it < 2; ++it) {
              dr[jt][it] = Mfma<T>::mac(bv[jt].x, av[it].x, dr[jt][it]);
              di[jt][it] = Mfma<T>::mac(bv[jt].y, av[it].y, di[jt][it]);
              d3[jt][it] = Mfma<T>::mac(bs[jt], as[it], d3[jt][it]);
            }
        } else {
#pragma unroll
          for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int it = 0; it < 2; ++it) {
              dr[jt][it] = Mfma<T>::mac(bv[jt].x, av[it].x, dr[jt][it]);
              dr[jt][it] = Mfma<T>::mac(-bv[jt].y, av[it].y, dr[jt][it]);
              di[jt][it] = Mfma<T>::mac(bv[jt].x, av[it].y, di[jt][it]);
              di[jt][it] = Mfma<T>::mac(bv[jt].y, av[it].x, di[jt][it]);
            }
        }
      }
    }
  }
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if constexpr (G3) {
          red[wave][jt][it][0][v][lane] = dr[jt][it][v] - di[jt][it][v];
          red[wave][jt][it][1][v][lane] = d3[jt][it][v] - dr[jt][it][v] - di[jt][it][v];
        } else {
          red[wave][jt][it][0][v][lane] = dr[jt][it][v];
          red[wave][jt][it][1][v][lane] = di[jt][it][v];
        }
      }
  __syncthreads();
  // lane holds D(row(lane / 16, v), lane % 16) of tile (jt, it)
  const int jt = wave >> 1, it = wave & 1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = j0 + 16 * jt + Mfma<T>::row(l4, v);
    const int i = i0 + 16 * it + l16;
    if (j >= a.ns || i >= a.n) continue;
    T sr = red[0][jt][it][0][v][lane], si = red[0][jt][it][1][v][lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      sr += red[w][jt][it][0][v][lane];
      si += red[w][jt][it][1][v][lane];
    }
    epi_store<EPI>(a, f, j, i, (double)sr, (double)si);
  }
}

template <typename T, int MODE, int EPI>
hipError_t run_gemm_sk(const GemmArgs& a, int nf, hipStream_t st) {
  dim3 grid(cdiv(a.ns, kSkT), cdiv(a.n, kSkT), nf);
  hipLaunchKernelGGL((k_cgemm_sk<T, MODE, EPI>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}


// Largest eigenvalue of each Hhat(w) by power iteration in FP64 (one workgroup
// per frequency), Rayleigh quotient of the final vector.  Eight lanes per row
// (coalesced 128-byte reads of Hhat), and per iteration one workgroup
// reduction of |y|^2, Re(v^H y) and |v|^2 together (wave butterflies, one
// LDS slot per wave).
__global__ void __launch_bounds__(256)
    k_power(Geometry g, const double2* __restrict__ hhat, double* __restrict__ eig, int iters) {
  extern __shared__ double2 sv[];  // v[n], y[n]
  __shared__ double red[3][256 / 64];
  const int f = blockIdx.x;
  const int n = g.nr;
  const double2* H = hhat + (size_t)f * n * n;
  double2* v = sv;
  double2* y = sv + n;
  const int r8 = threadIdx.x & 7;
  const int nw = (int)(blockDim.x >> 6);
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = make_double2(1.0 + 0.25 * sin(1.0 + i), 0.0);
  __syncthreads();
  double lam = 0.0;
  for (int it = 0; it <= iters; ++it) {
    double part = 0.0, rq = 0.0, vn = 0.0;
    for (int i0 = 0; i0 < n; i0 += (int)(blockDim.x >> 3)) {
      const int i = i0 + (int)(threadIdx.x >> 3);
      const bool live = i < n;
      const double2* Hi = H + (size_t)(live ? i : 0) * n;
      double tr = 0.0, ti = 0.0;
      for (int j = r8; j < n; j += 8) {
        const double2 h = Hi[j], x = v[j];
        tr += h.x * x.x - h.y * x.y;
        ti += h.x * x.y + h.y * x.x;
      }
      for (int o = 1; o < 8; o <<= 1) {
        tr += __shfl_xor(tr, o);
        ti += __shfl_xor(ti, o);
      }
      if (live && r8 == 0) {
        y[i] = make_double2(tr, ti);
        part += tr * tr + ti * ti;
        rq += v[i].x * tr + v[i].y * ti;  // Re(conj(v_i) y_i)
        vn += v[i].x * v[i].x + v[i].y * v[i].y;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      part += __shfl_xor(part, o);
      rq += __shfl_xor(rq, o);
      vn += __shfl_xor(vn, o);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = part;
      red[1][threadIdx.x >> 6] = rq;
      red[2][threadIdx.x >> 6] = vn;
    }
    __syncthreads();
    double ys = 0.0, q = 0.0, vs = 0.0;
    for (int w = 0; w < nw; ++w) {
      ys += red[0][w];
      q += red[1][w];
      vs += red[2][w];
    }
    const double ny = sqrt(ys);
    // normalise v's norm into the quotient
    lam = q / vs;
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
  a.A = m32; a.sA = npp; a.lda = np; a.arows = np; a.kdim = n;
  a.B = R + (size_t)s0 * n; a.sB = (size_t)rld * n; a.ldb = n;
  a.C = y32; a.sC = sv; a.ldc = n;
  hipError_t e = run_gemm_sk<float, 1, kEpiStore>(a, g.nf, st);
  if (e != hipSuccess) return e;
  // X = M^H Y
  a.B = y32; a.sB = sv; a.ldb = n;
  if (refine == 0) {
    a.C = out + (size_t)s0 * n; a.sC = (size_t)rld * n; a.ldc = n;
    return run_gemm_sk<float, 2, kEpiStore>(a, g.nf, st);
  }
  a.X = x64; a.sX = sv; a.ldx = n;
  e = run_gemm_sk<float, 2, kEpiX64Set>(a, g.nf, st);
  if (e != hipSuccess) return e;
  for (int it = 0; it < refine; ++it) {
    // r = R - Qhat X (FP64)
    GemmArgs q = a;
    q.A = qhat; q.sA = nn; q.lda = n; q.arows = n; q.kdim = n;
    q.B = x64; q.sB = sv; q.ldb = n;
    q.R = R + (size_t)s0 * n; q.sR = (size_t)rld * n; q.ldr = n;
    q.C = r32; q.sC = sv; q.ldc = n;
    e = run_gemm_sk<double, 0, kEpiResid>(q, g.nf, st);
    if (e != hipSuccess) return e;
    // Y = M r
    GemmArgs y = a;
    y.A = m32; y.sA = npp; y.lda = np; y.arows = np; y.kdim = n;
    y.B = r32; y.sB = sv; y.ldb = n;
    y.C = y32; y.sC = sv; y.ldc = n;
    e = run_gemm_sk<float, 1, kEpiStore>(y, g.nf, st);
    if (e != hipSuccess) return e;
    // X += M^H Y (the last step writes the complex64 result)
    GemmArgs x = y;
    x.B = y32;
    if (it + 1 < refine) {
      e = run_gemm_sk<float, 2, kEpiX64Add>(x, g.nf, st);
    } else {
      x.C = out + (size_t)s0 * n; x.sC = (size_t)rld * n; x.ldc = n;
      e = run_gemm_sk<float, 2, kEpiOut>(x, g.nf, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_dct_compress(const Geometry& g, const float2* ghat, int rows_per_f, int row0, int nrows,
                               const float2* dz, const float2* dx, float2* tmp, float2* gcomp, hipStream_t st) {
  // per spectrum row (frequency, receiver), seen as an nzs x nxs image:
  //   T(ix, kz) = sum_iz Dz(kz, iz) G(iz, ix),  stored [row][ix][kz]
  //   C(kz, kx) = sum_ix Dx(kx, ix) T(ix, kz),  stored [row][kz][kx]
  // (complex64 operands, products and sums in FP64).  Input rows
  // f * rows_per_f + i, i < nrows; output rows f * nr + row0 + i.
  if (nrows < 1 || nrows > 65535 || row0 < 0 || row0 + nrows > g.nr) return hipErrorInvalidValue;
  for (int f = 0; f < g.nf; ++f) {
    float2* t = tmp + (size_t)f * nrows * g.nxs * g.keep_z;
    GemmArgs p{};
    p.A = dz; p.sA = 0; p.lda = g.nzs; p.arows = g.keep_z;
    p.B = ghat + (size_t)f * rows_per_f * g.nsub; p.sB = (size_t)g.nsub; p.ldb = g.nxs;
    p.n = g.keep_z; p.ns = g.nxs; p.kdim = g.nzs;
    p.C = t; p.sC = (size_t)g.nxs * g.keep_z; p.ldc = g.keep_z;
    hipError_t e = run_gemm<float, 0, kEpiStore, 1, double>(p, nrows, st);
    if (e != hipSuccess) return e;
    GemmArgs q{};
    q.A = dx; q.sA = 0; q.lda = g.nxs; q.arows = g.keep_x;
    q.B = t; q.sB = (size_t)g.nxs * g.keep_z; q.ldb = g.keep_z;
    q.n = g.keep_x; q.ns = g.keep_z; q.kdim = g.nxs;
    q.C = gcomp + ((size_t)f * g.nr + row0) * g.keep_z * g.keep_x; q.sC = (size_t)g.keep_z * g.keep_x;
    q.ldc = g.keep_x;
    e = run_gemm<float, 0, kEpiStore, 1, double>(q, nrows, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Hhat = (H + H^H) / 2 in place, one thread per pair i <= j: the product below
// forms H(i, j) and H(j, i) from the same terms in different orders.
__global__ void k_hermitize(int n, double2* __restrict__ H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j < i || j >= n) return;
  double2* M = H + (size_t)blockIdx.z * n * n;
  const double2 a = M[(size_t)i * n + j], b = M[(size_t)j * n + i];
  const double2 v = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
  M[(size_t)i * n + j] = v;
  M[(size_t)j * n + i] = make_double2(v.x, -v.y);
}

// Hhat of the compressed spectra C (complex64 [nf][nr][K]):
//   Hhat(i, j) = sum_k C(i, k) conj(C(j, k)),
// FP32 operands, FP64 products and sums.  The product computes
// conj(Hhat(i, j)) = sum_k conj(C(i, k)) C(j, k) and stores it at [j][i], which
// is where Hhat(j, i) = conj(Hhat(i, j)) belongs.
hipError_t launch_herk_compressed(const Geometry& g, const float2* gcomp, int K, double2* hhat,
                                  hipStream_t st) {
  GemmArgs p{};
  p.A = gcomp; p.sA = (size_t)g.nr * K; p.lda = K; p.arows = g.nr;
  p.B = gcomp; p.sB = (size_t)g.nr * K; p.ldb = K;
  p.n = g.nr; p.ns = g.nr; p.kdim = K;
  p.X = hhat; p.sX = (size_t)g.nr * g.nr; p.ldx = g.nr;
  hipError_t e = run_gemm<float, 3, kEpiX64Set, 0, double>(p, g.nf, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hermitize, dim3(cdiv(g.nr, 256), g.nr, g.nf), dim3(256), 0, st, g.nr, hhat);
  return hipGetLastError();
}

hipError_t launch_power_iter(const Geometry& g, const double2* hhat, double* eig, int iters,
                             hipStream_t st) {
  size_t shmem = 2 * (size_t)g.nr * sizeof(double2);
  hipLaunchKernelGGL(k_power, dim3(g.nf), dim3(256), shmem, st, g, hhat, eig, iters);
  return hipGetLastError();
}

}  // namespace ehi
