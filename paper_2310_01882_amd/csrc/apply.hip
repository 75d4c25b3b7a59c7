// General constant-offset stencil apply: the paper's stencil.apply
// (Section 2.2, Listing 2) for linear regions of up to 27 taps of radius 1.
//
// The tap table travels in the kernel arguments; one thread computes one
// interior cell, x fastest, so every tap's reads form coalesced row
// segments and neighbouring threads share cache lines.
#include "ms_internal.hpp"

#pragma clang fp contract(off)

namespace ms {
namespace {

constexpr int kMaxTaps = 27;

template <typename T>
struct ApplyK {
  const T* in;
  const T* rhs;
  T* out;
  int64_t off[kMaxTaps];
  T w[kMaxTaps];
  T rhs_coef, scale;
  int ntaps;
  int nx, ny, nz;
  int64_t sy, sz;
};

template <typename T, bool HAS_RHS>
__global__ __launch_bounds__(256) void apply_kernel(ApplyK<T> a) {
  // blockIdx.x enumerates (row, x-block) pairs, x-blocks fastest.
  const int xblocks = (a.nx + blockDim.x - 1) / blockDim.x;
  const int64_t jk = blockIdx.x / xblocks;
  const int i = (blockIdx.x % xblocks) * blockDim.x + threadIdx.x;
  if (i >= a.nx) return;
  const int j = (int)(jk % a.ny), k = (int)(jk / a.ny);
  const int64_t p = (int64_t)(k + 1) * a.sz + (int64_t)(j + 1) * a.sy + (i + 1);
  T acc = a.w[0] * a.in[p + a.off[0]];
  for (int t = 1; t < a.ntaps; ++t) acc = acc + a.w[t] * a.in[p + a.off[t]];
  if (HAS_RHS) acc = acc + a.rhs_coef * a.rhs[p];
  a.out[p] = a.scale * acc;
}

template <typename T>
int run_apply(const ms_stencil& st, const ms_grid& g, const void* in, const void* rhs, void* out,
              hipStream_t s) {
  ApplyK<T> a{};
  a.in = static_cast<const T*>(in);
  a.rhs = static_cast<const T*>(rhs);
  a.out = static_cast<T*>(out);
  a.ntaps = st.ntaps;
  for (int t = 0; t < st.ntaps; ++t) {
    const ms_tap& tp = st.taps[t];
    a.off[t] = (int64_t)tp.dz * g.sz + (int64_t)tp.dy * g.sy + tp.dx;
    a.w[t] = (T)tp.w;
  }
  a.rhs_coef = (T)st.rhs_coef;
  a.scale = (T)st.scale;
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  a.sy = g.sy; a.sz = g.sz;
  const int64_t blocks = (int64_t)g.ny * g.nz * ((g.nx + 255) / 256);
  if (blocks > 0x7fffffffLL) return set_error(MS_EUNSUPPORTED, "stencil_apply: grid too large");
  const dim3 grid((unsigned)blocks);
  if (rhs)
    hipLaunchKernelGGL((apply_kernel<T, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((apply_kernel<T, false>), grid, dim3(256), 0, s, a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int stencil_apply(const ms_stencil* st, const ms_grid* g, int dtype, const void* in,
                             const void* rhs, void* out, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "stencil_apply")) return rc;
  if (!st) return set_error(MS_EINVAL, "stencil_apply: stencil is NULL");
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "stencil_apply: dtype %d", dtype);
  if (st->ntaps < 1 || st->ntaps > kMaxTaps)
    return set_error(MS_EUNSUPPORTED, "stencil_apply: ntaps %d not in [1, %d]", st->ntaps,
                     kMaxTaps);
  if (!st->taps) return set_error(MS_EINVAL, "stencil_apply: taps is NULL");
  for (int t = 0; t < st->ntaps; ++t) {
    const ms_tap& tp = st->taps[t];
    if (tp.dx < -1 || tp.dx > 1 || tp.dy < -1 || tp.dy > 1 || tp.dz < -1 || tp.dz > 1)
      return set_error(MS_EINVAL, "stencil_apply: tap %d offset (%d,%d,%d) beyond the halo", t,
                       tp.dx, tp.dy, tp.dz);
  }
  if (!in || !out) return set_error(MS_EINVAL, "stencil_apply: in and out required");
  const size_t bytes = (size_t)field_span(*g) * (dtype == MS_F64 ? 8 : 4);
  if (overlaps(in, bytes, out, bytes) || (rhs && overlaps(rhs, bytes, out, bytes)))
    return set_error(MS_EINVAL, "stencil_apply: out aliases an input (apply is out-of-place)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == MS_F64) return run_apply<double>(*st, *g, in, rhs, out, s);
  return run_apply<float>(*st, *g, in, rhs, out, s);
}
