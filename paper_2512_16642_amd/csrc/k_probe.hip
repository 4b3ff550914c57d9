// HBM probe: plain streaming kernels with a chosen mix of reads and writes, to
// measure the rate the memory system delivers for a kernel's access mix (the
// ceiling that the marching kernel's measured traffic is compared with).
// Each thread handles 16-byte vectors in a grid-stride loop; reads are used
// in the values written, so none can be elided.
#include <hip/hip_runtime.h>

#include "ehi_internal.h"

namespace ehi {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// R = 1 or 2 arrays read (a, b), W = 0..3 arrays written (c, d, and e over its
// first n4e vectors, n4e <= 2 n4: e[i] and e[n4 + i]).  With W = 0 each thread
// writes the sum of what it read to sink once at the end.
template <int R, int W>
__global__ void __launch_bounds__(256) k_stream(const f4* __restrict__ a, const f4* __restrict__ b,
                                                f4* __restrict__ c, f4* __restrict__ d, f4* __restrict__ e,
                                                size_t n4, size_t n4e, f4* __restrict__ sink) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (; i < n4; i += stride) {
    const f4 x = a[i];
    const f4 y = R > 1 ? b[i] : x;
    if (W >= 1) c[i] = x + y;
    if (W >= 2) d[i] = x - y;
    if (W >= 3 && i < n4e) e[i] = x * y;
    if (W >= 3 && n4 + i < n4e) e[n4 + i] = x * x;
    if (W == 0) acc += x + y;
  }
  if (W == 0) sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_stream_probe(int mode, const void* a, const void* b, void* c, void* d, void* e, size_t bytes,
                               double e_frac, int grid, void* sink, hipStream_t st) {
  const size_t n4 = bytes / 16;
  const size_t n4e = (size_t)(e_frac * (double)n4);
  const f4* A = static_cast<const f4*>(a);
  const f4* B = static_cast<const f4*>(b);
  f4 *C = static_cast<f4*>(c), *D = static_cast<f4*>(d), *E = static_cast<f4*>(e), *S = static_cast<f4*>(sink);
  const dim3 g(grid), t(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_stream<1, 1>), g, t, 0, st, A, B, C, D, E, n4, n4e, S); break;  // copy
    case 1: hipLaunchKernelGGL((k_stream<1, 0>), g, t, 0, st, A, B, C, D, E, n4, n4e, S); break;  // read
    case 2: hipLaunchKernelGGL((k_stream<2, 2>), g, t, 0, st, A, B, C, D, E, n4, n4e, S); break;  // 2 read, 2 write
    case 3: hipLaunchKernelGGL((k_stream<2, 3>), g, t, 0, st, A, B, C, D, E, n4, n4e, S); break;  // + e_frac write
    case 4: hipLaunchKernelGGL((k_stream<2, 0>), g, t, 0, st, A, B, C, D, E, n4, n4e, S); break;  // 2 read
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ehi
