// Time-axis resampling of the record for the finite-record weighting.
//
// Paper: the numerical examples resample the Green functions and the data to
// the Nyquist rate in time before the Hessian is formed.  The Green functions
// here are impulse responses with content up to the grid's limit, so every
// D-th sample is kept only after a zero-phase low-pass filter (taps h_j,
// j = -K..K, designed on the host): y_q = sum_j h_j g(n_q + j) at the kept
// times n_q = 1 - K + q D, g(n) = 0 outside the record 1..nt.  The running
// spectra and the finite-record Gram average then run over the kept samples
// (one in D), with the filter's passband response divided out per frequency.
//
// The filter reads the current staging window (samples n_w0 .. of this batch
// of receivers, slot (n - 1) % chunk) and the last 2K samples of the previous
// window, which k_hist_copy keeps in a history buffer.
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

constexpr int kDecP = 8;  // kept samples produced together by one pass over the rows

// dec[r][q - q0][x] = y_q(x) for q = q0 .. q0 + cnt - 1, every point x of the
// staging row pitch (the padding columns hold zeros in and out).
__global__ void __launch_bounds__(256)
    k_decimate(Geometry g, const float* __restrict__ stage, const float* __restrict__ hist,
               const float* __restrict__ taps, int q0, int cnt, int n_w0, int n_end, float* __restrict__ dec) {
  // taps padded with zeros so that tp[base - p D] covers every output p of a pass
  __shared__ float tp[2 * kMaxDecimK + 1 + 2 * (kDecP - 1) * kMaxDecim];
  const int K = g.dK, D = g.decim;
  const int pad = (kDecP - 1) * D;
  const int ntap = 2 * K + 1 + 2 * pad;
  for (int i = threadIdx.x; i < ntap; i += blockDim.x) {
    const int j = i - pad;
    tp[i] = (j >= 0 && j <= 2 * K) ? taps[j] : 0.f;
  }
  __syncthreads();
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (x >= g.nsub_p) return;
  const float* st = stage + (size_t)r * g.chunk * g.nsub_p + x;
  const float* hs = hist + (size_t)r * g.dhist * g.nsub_p + x;
  float* out = dec + (size_t)r * g.drows * g.nsub_p + x;
  const int h0 = n_w0 - g.dhist;  // first sample held in the history
  for (int qb = 0; qb < cnt; qb += kDecP) {
    float acc[kDecP];
#pragma unroll
    for (int p = 0; p < kDecP; ++p) acc[p] = 0.f;
    const int nq = 1 - K + (q0 + qb) * D;
    const int nlo = max(nq - K, max(1, h0));
    const int nhi = min(nq + (kDecP - 1) * D + K, n_end);
    for (int n = nlo; n <= nhi; ++n) {
      const float s = n >= n_w0 ? st[(size_t)((n - 1) % g.chunk) * g.nsub_p] : hs[(size_t)(n - h0) * g.nsub_p];
      const int base = n - nq + K + pad;
#pragma unroll
      for (int p = 0; p < kDecP; ++p) acc[p] = fmaf(tp[base - p * D], s, acc[p]);
    }
#pragma unroll
    for (int p = 0; p < kDecP; ++p)
      if (qb + p < cnt) out[(size_t)(qb + p) * g.nsub_p] = acc[p];
  }
}

// hist[r][j][x] = the sample n_end - dhist + 1 + j of the current window
__global__ void k_hist_copy(Geometry g, const float* __restrict__ stage, int n_end, float* __restrict__ hist) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= (size_t)g.dhist * g.nsub_p) return;
  const int j = (int)(e / g.nsub_p);
  const size_t x = e % g.nsub_p;
  const int n = n_end - g.dhist + 1 + j;
  hist[((size_t)r * g.dhist + j) * g.nsub_p + x] = stage[((size_t)r * g.chunk + (n - 1) % g.chunk) * g.nsub_p + x];
}

// tw[q][f] = exp(-i 2 pi f_hz (n_first + q n_step) dt), q = 0..count-1, in FP64.
__global__ void k_twiddles_at(int count, int nf, double dt, const double* __restrict__ freq, int n_first,
                              int n_step, float2* __restrict__ tw) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)count * nf) return;
  const int q = (int)(i / nf), f = (int)(i % nf);
  const double th = 2.0 * 3.14159265358979323846 * freq[f] * (double)(n_first + (long long)q * n_step) * dt;
  double s, c;
  sincos(th, &s, &c);
  tw[i] = make_float2((float)c, (float)(-s));
}

// ghat[f][r][x] *= scale[f]
__global__ void k_scale_spectra(Geometry g, const double* __restrict__ scale, float2* __restrict__ ghat) {
  const size_t per = (size_t)g.nr * g.nsub;
  const size_t n = per * g.nf;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float c = (float)scale[i / per];
    ghat[i].x *= c;
    ghat[i].y *= c;
  }
}

}  // namespace

hipError_t launch_decimate(const Geometry& g, const float* stage, const float* hist, const float* taps, int q0,
                           int cnt, int n_w0, int n_end, int nrb_now, float* dec, hipStream_t st) {
  if (g.decim < 2 || g.decim > kMaxDecim || g.dK > kMaxDecimK || cnt < 1 || cnt > g.drows || g.nsub_p % 256 ||
      n_end < n_w0 || n_end - n_w0 >= g.chunk || n_end > g.nt)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_decimate, dim3(g.nsub_p / 256, nrb_now), dim3(256), 0, st, g, stage, hist, taps, q0, cnt,
                     n_w0, n_end, dec);
  return hipGetLastError();
}

hipError_t launch_hist_copy(const Geometry& g, const float* stage, int n_end, int nrb_now, float* hist,
                            hipStream_t st) {
  if (g.dhist < 1 || g.dhist > g.chunk || n_end < g.dhist) return hipErrorInvalidValue;
  const size_t n = (size_t)g.dhist * g.nsub_p;
  hipLaunchKernelGGL(k_hist_copy, dim3((unsigned)((n + 255) / 256), nrb_now), dim3(256), 0, st, g, stage, n_end,
                     hist);
  return hipGetLastError();
}

hipError_t launch_twiddles_at(int count, int nf, double dt, const double* freq, int n_first, int n_step,
                              float2* tw, hipStream_t st) {
  const size_t n = (size_t)count * nf;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_twiddles_at, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, count, nf, dt, freq,
                     n_first, n_step, tw);
  return hipGetLastError();
}

hipError_t launch_scale_spectra(const Geometry& g, const double* scale, float2* ghat, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_spectra, dim3(2048), dim3(256), 0, st, g, scale, ghat);
  return hipGetLastError();
}

}  // namespace ehi
