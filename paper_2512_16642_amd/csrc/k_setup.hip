// Medium, twiddle and wavefield set-up kernels (paper: Theory section, the
// acoustic wave equation with squared slowness m; Fourier-domain Hessian for
// the transform sign).  Everything here runs once per survey or per receiver
// batch and is negligible next to the time loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ehi_internal.h"

namespace ehi {
namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) p[i] = value;
}

// Max over positive float32 velocities: the bit patterns of positive floats
// order like unsigned integers, so an atomic max on the bits is exact.
__global__ void k_vmax(const float* __restrict__ vel, int n, uint32_t* __restrict__ out) {
  __shared__ uint32_t red[256];
  uint32_t m = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float v = vel[i];
    uint32_t b = v > 0.f ? __float_as_uint(v) : 0u;
    m = b > m ? b : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      uint32_t o = red[threadIdx.x + s];
      if (o > red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, red[0]);
}

// Coefficients of the increment-form recurrence
//   w^{n+1} = (b/a) w^n + kappa/(12 h^2 a) * L12 u^n ,  u^{n+1} = u^n + w^{n+1}
// with L12 the 4th-order Laplacian scaled by 12 h^2 (integer weights
// -1, 16, -30 per axis), kappa = v^2 dt^2, a = 1 + eta dt/2, b = 1 - eta dt/2,
// eta = eta_max (d/nb)^2, eta_max = 3 vmax ln(1000) / (2 nb h), d the cell
// distance into the absorbing layer.  Computed in FP64, rounded once:
// ca[cell] = kappa / (12 h^2 a) on the padded plane (0 on the ghost ring) and
// bd[d] = b / a for d = 0..nb (b/a depends on d only).
//
// ca is rounded stochastically, to the FP32 neighbour above or below with the
// probabilities that make its expected value exact (the choice drawn from a
// hash of the cell index, so it is reproducible).  Rounding to nearest would
// give every cell of a constant-velocity layer the same relative error (up to
// 2^-25): a uniformly perturbed medium whose phase error grows with travel
// time, and the largest part of the Green functions' FP32 error at low
// frequencies.  Dithered, the perturbation has zero mean and no coherent
// effect.
__device__ inline double sponge_eta(const Geometry& g, double vmax, int d) {
  if (g.nb <= 0 || d <= 0) return 0.0;
  double emax = 3.0 * vmax * log(1000.0) / (2.0 * g.nb * g.h);
  double r = (double)d / g.nb;
  return emax * r * r;
}

// 32-bit integer finaliser ("lowbias32", C. Wellons' hash-prospector
// search): a bijection whose output bits are close to independent of the input.
__device__ inline uint32_t cell_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// ce rounded to one of its two FP32 neighbours, the upper with probability
// equal to ce's fractional position between them (exact values stay exact).
__device__ inline float dithered_float(double ce, uint32_t key) {
  const float c = (float)ce;
  float lo = c, hi = c;
  if ((double)c > ce) lo = nextafterf(c, 0.f);
  else if ((double)c < ce) hi = nextafterf(c, __builtin_huge_valf());
  else return c;
  const double f = (ce - (double)lo) / ((double)hi - (double)lo);
  const double r = (double)cell_hash(key) * (1.0 / 4294967296.0);
  return r < f ? hi : lo;
}

__global__ void k_coefficients(Geometry g, const float* __restrict__ vel,
                               const uint32_t* __restrict__ vmax_bits, float* __restrict__ ca,
                               float* __restrict__ bd) {
  int px = blockIdx.x * blockDim.x + threadIdx.x;  // plane column
  int pz = blockIdx.y;                             // plane row
  const double vmax = (double)__uint_as_float(vmax_bits[0]);
  if (pz == 0 && px <= g.nb) {
    double eta = sponge_eta(g, vmax, px);
    bd[px] = (float)((1.0 - eta * g.dt * 0.5) / (1.0 + eta * g.dt * 0.5));
  }
  if (px >= g.Xp || pz >= g.Zp) return;
  size_t o = (size_t)pz * g.Xp + px;
  int iz = pz - kGhost, ix = px - kGhost;  // padded-grid indices
  if (iz < 0 || iz >= g.Z || ix < 0 || ix >= g.X) {
    ca[o] = 0.f;
    return;
  }
  int jz = min(max(iz - g.nb, 0), g.nz - 1);
  int jx = min(max(ix - g.nb, 0), g.nx - 1);
  double v = (double)vel[(size_t)jz * g.nx + jx];
  int dz = max(max(g.nb - iz, iz - (g.nb + g.nz - 1)), 0);
  int dx = max(max(g.nb - ix, ix - (g.nb + g.nx - 1)), 0);
  double eta = sponge_eta(g, vmax, max(dz, dx));
  double a = 1.0 + eta * g.dt * 0.5;
  double kappa = v * v * g.dt * g.dt;
  ca[o] = dithered_float(kappa / (12.0 * g.h * g.h * a), (uint32_t)o);
}

// tw[n-1][f] = exp(-i 2 pi f_hz n dt), n = 1..nt, evaluated in FP64.
__global__ void k_twiddles(int nt, int nf, double dt, const double* __restrict__ freq,
                           float2* __restrict__ tw) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nt * nf) return;
  int n = (int)(i / nf) + 1;
  int f = (int)(i % nf);
  double w = 2.0 * 3.14159265358979323846 * freq[f];
  double th = w * (double)n * dt;
  double s, c;
  sincos(th, &s, &c);
  tw[i] = make_float2((float)c, (float)(-s));
}

// Fields after the impulse: u^1 = w^1 = kappa_r / a_r at the receiver cell
// (f^0 = unit impulse there), zero elsewhere; slot 0 of the staging buffer
// gets the sample u^1 on the subgrid.
__global__ void k_wave_init_point(Geometry g, const float* __restrict__ vel,
                                  const int32_t* __restrict__ rec, int r0, int nrb_now,
                                  float* __restrict__ u0, float* __restrict__ w,
                                  float* __restrict__ stage) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrb_now) return;
  int iz = rec[r0 + r];
  int ix = rec[g.nr + r0 + r];
  double v = (double)vel[(size_t)iz * g.nx + ix];
  // receivers are interior cells: eta = 0 there, a = 1
  float val = (float)(v * v * g.dt * g.dt);
  size_t o = (size_t)r * g.plane() + (size_t)(iz + g.nb + kGhost) * g.Xp + (ix + g.nb + kGhost);
  u0[o] = val;
  w[o] = val;
  if (iz % g.stride == 0 && ix % g.stride == 0) {
    size_t so = (size_t)r * g.chunk * g.nsub_p + (size_t)(iz / g.stride) * g.nxs + ix / g.stride;
    stage[so] = val;
  }
}

// Zero staging slot 0 of every receiver of the batch (sample 1).
__global__ void k_zero_slot0(float* __restrict__ stage, size_t nsub, size_t pitch, int nrb) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i < nsub && r < nrb) stage[(size_t)r * pitch + i] = 0.f;
}

// Zero the padding [used, pitch) of rows of a pitched buffer.
__global__ void k_zero_row_tails(float* __restrict__ p, size_t rows, int used, int pitch) {
  const size_t tail = (size_t)(pitch - used);
  const size_t n = rows * tail;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[(i / tail) * pitch + used + i % tail] = 0.f;
}

__global__ void k_c128_from_c64(const float2* __restrict__ in, double2* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

__global__ void k_c64_from_c128(const double2* __restrict__ in, float2* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// Leading keep rows of the orthonormal DCT-II matrix of size n, evaluated in
// FP64: D[k][m] = s_k cos(pi k (2m + 1) / (2n)), s_0 = sqrt(1/n),
// s_k = sqrt(2/n); stored as complex64 with a zero imaginary part.
__global__ void k_dct_matrix(int n, int keep, float2* __restrict__ d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * keep) return;
  const int k = e / n, m = e % n;
  const double s = k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n);
  const double v = s * cos(M_PI * (double)k * (2.0 * m + 1.0) / (2.0 * n));
  d[e] = make_float2((float)v, 0.f);
}

}  // namespace

hipError_t launch_dct_matrix(int n, int keep, float2* d, hipStream_t st) {
  hipLaunchKernelGGL(k_dct_matrix, dim3(cdiv(n * keep, 256)), dim3(256), 0, st, n, keep, d);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}

hipError_t launch_vmax(const float* vel, int n, uint32_t* out_bits, hipStream_t st) {
  hipError_t e = launch_fill_u32(out_bits, 0u, 1, st);
  if (e != hipSuccess) return e;
  int blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_vmax, dim3(blocks), dim3(256), 0, st, vel, n, out_bits);
  return hipGetLastError();
}

hipError_t launch_coefficients(const Geometry& g, const float* vel, const uint32_t* vmax_bits,
                               float* ca, float* bd, hipStream_t st) {
  dim3 grid(cdiv(std::max(g.Xp, g.nb + 1), 256), g.Zp);
  hipLaunchKernelGGL(k_coefficients, grid, dim3(256), 0, st, g, vel, vmax_bits, ca, bd);
  return hipGetLastError();
}

hipError_t launch_twiddles(const Geometry& g, const double* freq, float2* tw, hipStream_t st) {
  size_t n = (size_t)g.nt * g.nf;
  hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.nt, g.nf,
                     g.dt, freq, tw);
  return hipGetLastError();
}

hipError_t launch_zero_stage_tails(const Geometry& g, float* stage, hipStream_t st) {
  const int tail = g.nsub_p - g.nsub;
  if (tail == 0) return hipSuccess;
  const size_t rows = (size_t)g.windows * g.nrb * g.chunk;
  const size_t n = rows * (size_t)tail;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero_row_tails, dim3(blocks), dim3(256), 0, st, stage, rows, g.nsub, g.nsub_p);
  return hipGetLastError();
}

hipError_t launch_wave_init(const Geometry& g, const float* vel, const int32_t* rec, int r0,
                            int nrb_now, float* u0, float* w, float* stage, hipStream_t st) {
  size_t nplane = (size_t)nrb_now * g.plane();
  hipError_t e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(u0), 0u, nplane, st)) != hipSuccess) return e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(w), 0u, nplane, st)) != hipSuccess) return e;
  // slot 0 of the staging buffer holds sample 1: zero except at the receiver
  hipLaunchKernelGGL(k_zero_slot0, dim3(cdiv(g.nsub, 256), nrb_now), dim3(256), 0, st, stage,
                     (size_t)g.nsub, (size_t)g.chunk * g.nsub_p, nrb_now);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_wave_init_point, dim3(cdiv(nrb_now, 64)), dim3(64), 0, st, g, vel, rec, r0,
                     nrb_now, u0, w, stage);
  return hipGetLastError();
}

hipError_t launch_c128_from_c64(const float2* in, double2* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_c128_from_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_c64_from_c128(const double2* in, float2* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_c64_from_c128, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace ehi
