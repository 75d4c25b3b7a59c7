// Streaming kernel that measures the practical HBM ceiling of the access
// patterns the stencils use: read one or two arrays, write one, 16-byte
// lanes, nontemporal stores, grid-stride over a fixed grid of blocks
// (eight waves per CU slot). It does no stencil work; the benchmark quotes
// its GB/s beside the stencils' as the device's achievable bandwidth.
#include "ms_internal.hpp"

namespace ms {
namespace {

typedef __attribute__((ext_vector_type(2))) double d2;

template <bool TWO>
__global__ __launch_bounds__(256) void stream_kernel(const d2* __restrict__ a,
                                                     const d2* __restrict__ b,
                                                     d2* __restrict__ out, int64_t n2) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n2;
       t += (int64_t)gridDim.x * blockDim.x) {
    d2 v = a[t];
    if (TWO) v += b[t];
    __builtin_nontemporal_store(v, out + t);
  }
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int ms_stream_probe(const double* a, const double* b, double* out, int64_t n,
                               int blocks, void* stream) {
  clear_error();
  if (!a || !out || n < 0 || (n & 1) || blocks < 1)
    return set_error(MS_EINVAL, "ms_stream_probe: bad arguments (n must be even)");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
       reinterpret_cast<uintptr_t>(out)) & 15)
    return set_error(MS_EINVAL, "ms_stream_probe: arrays must be 16-byte aligned");
  const size_t bytes = (size_t)n * 8;
  if (overlaps(a, bytes, out, bytes) || (b && overlaps(b, bytes, out, bytes)))
    return set_error(MS_EINVAL, "ms_stream_probe: out overlaps an input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const auto* a2 = reinterpret_cast<const d2*>(a);
  const auto* b2 = reinterpret_cast<const d2*>(b);
  auto* o2 = reinterpret_cast<d2*>(out);
  if (b)
    hipLaunchKernelGGL(stream_kernel<true>, dim3(blocks), dim3(256), 0, s, a2, b2, o2, n / 2);
  else
    hipLaunchKernelGGL(stream_kernel<false>, dim3(blocks), dim3(256), 0, s, a2, b2, o2, n / 2);
  MS_LAUNCH_CHECK();
  return MS_OK;
}
