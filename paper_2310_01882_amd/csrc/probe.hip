// Streaming kernel that measures the practical HBM ceiling of the access
// patterns the stencils use: read one or two arrays, write one, 16-byte
// lanes, nontemporal stores, grid-stride over a fixed grid of blocks
// (eight waves per CU slot). It does no stencil work; the benchmark quotes
// its GB/s beside the stencils' as the device's achievable bandwidth.
#include "ms_internal.hpp"

namespace ms {
namespace {

typedef __attribute__((ext_vector_type(2))) double d2;

// Access forms: one 16-byte element per lane per grid stride (0); kU grid
// strides of loads issued before their stores (1); the same with
// nontemporal loads (2); block-contiguous chunks (3, below). The benchmark
// reports the best.
constexpr int kU = 4;

template <bool TWO, int FORM>
__global__ __launch_bounds__(256) void stream_kernel(const d2* __restrict__ a,
                                                     const d2* __restrict__ b,
                                                     d2* __restrict__ out, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (FORM > 0) {
    for (; t + (kU - 1) * stride < n2; t += kU * stride) {
      d2 v[kU], w[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        v[u] = FORM == 2 ? __builtin_nontemporal_load(a + t + u * stride) : a[t + u * stride];
      if (TWO) {
#pragma unroll
        for (int u = 0; u < kU; ++u)
          w[u] = FORM == 2 ? __builtin_nontemporal_load(b + t + u * stride) : b[t + u * stride];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] += w[u];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) __builtin_nontemporal_store(v[u], out + t + u * stride);
    }
  }
  for (; t < n2; t += stride) {
    d2 v = a[t];
    if (TWO) v += b[t];
    __builtin_nontemporal_store(v, out + t);
  }
}

// Form 3: each block streams through its own contiguous share of the
// arrays, 4 KiB (256 lanes x 16 bytes) per step, two steps of loads in
// flight, as a z-marching stencil block walks its planes.
template <bool TWO>
__global__ __launch_bounds__(256) void stream_chunk_kernel(const d2* __restrict__ a,
                                                           const d2* __restrict__ b,
                                                           d2* __restrict__ out, int64_t n2) {
  const int64_t per = (n2 + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, n2);
  int64_t t = lo + threadIdx.x;
  for (; t + blockDim.x < hi; t += 2 * (int64_t)blockDim.x) {
    d2 v0 = a[t], v1 = a[t + blockDim.x];
    if (TWO) {
      v0 += b[t];
      v1 += b[t + blockDim.x];
    }
    __builtin_nontemporal_store(v0, out + t);
    __builtin_nontemporal_store(v1, out + t + blockDim.x);
  }
  for (; t < hi; t += blockDim.x) {
    d2 v = a[t];
    if (TWO) v += b[t];
    __builtin_nontemporal_store(v, out + t);
  }
}

template <int FORM>
void launch_stream(const d2* a, const d2* b, d2* o, int64_t n2, int blocks, hipStream_t s) {
  if (FORM == 3) {
    if (b)
      hipLaunchKernelGGL(stream_chunk_kernel<true>, dim3(blocks), dim3(256), 0, s, a, b, o, n2);
    else
      hipLaunchKernelGGL(stream_chunk_kernel<false>, dim3(blocks), dim3(256), 0, s, a, b, o, n2);
  } else if (b) {
    hipLaunchKernelGGL((stream_kernel<true, FORM>), dim3(blocks), dim3(256), 0, s, a, b, o, n2);
  } else {
    hipLaunchKernelGGL((stream_kernel<false, FORM>), dim3(blocks), dim3(256), 0, s, a, b, o, n2);
  }
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int ms_stream_probe(const double* a, const double* b, double* out, int64_t n,
                               int blocks, int form, void* stream) {
  clear_error();
  if (!a || !out || n < 0 || (n & 1) || blocks < 1 || form < 0 || form > 3)
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
  if (form == 0) launch_stream<0>(a2, b2, o2, n / 2, blocks, s);
  else if (form == 1) launch_stream<1>(a2, b2, o2, n / 2, blocks, s);
  else if (form == 2) launch_stream<2>(a2, b2, o2, n / 2, blocks, s);
  else launch_stream<3>(a2, b2, o2, n / 2, blocks, s);
  MS_LAUNCH_CHECK();
  return MS_OK;
}
