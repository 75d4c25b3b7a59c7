// Jacobi sweeps on a field that stays in host memory (larger than the
// device can or should hold), streamed through the device in z slabs.
//
// The field is cut into slabs of S interior planes. A pass of T sweeps
// uploads each slab with T extra planes on either side (fewer at the field's
// own boundary), runs T sweeps on that extended slab as on a grid of its
// own -- its outermost planes stay fixed, like a Dirichlet halo -- and
// copies the slab's S planes back. After t sweeps only the t planes next to
// an artificial boundary are affected, so the S central planes are exactly
// the field's (a trapezoid in z): every value is bit-identical to
// jacobi_sweeps. Slabs alternate between two streams and two sets of device
// buffers, so one slab's upload overlaps another's sweeps and download; the
// passes read one host buffer and write the other.
#include "ms_internal.hpp"

#include <algorithm>
#include <vector>

namespace ms {
namespace {

struct SlabSet {
  void* a;  // slab iterate (two buffers, ping-pong)
  void* b;
  void* f;  // slab right-hand side
  double* partials;
};

size_t slab_elems(const ms_grid& g, int T, int S) {
  return (size_t)(S + 2 * T + 2) * (size_t)g.sz;
}

// A slab buffer with the host layout's vector phase: interior cell
// (0, 0, ·) lands on a 256-byte boundary, as in the aligned fields.
char* take_slab(Workspace& ws, size_t elems, int esz) {
  char* p = ws.take<char>(elems * esz + 256);
  return p ? p + 256 - esz : nullptr;
}

int check_streamed(const ms_grid* g, int dtype, int T, int S) {
  if (int rc = check_grid(g, "jacobi_sweeps_streamed")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "jacobi_sweeps_streamed: dtype %d", dtype);
  if (T < 1 || T > 4096)
    return set_error(MS_EINVAL, "jacobi_sweeps_streamed: sweeps_per_pass must be in [1, 4096]");
  if (S < 1) return set_error(MS_EINVAL, "jacobi_sweeps_streamed: slab_planes must be >= 1");
  return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" size_t jacobi_sweeps_streamed_workspace_bytes(const ms_grid* g, int dtype,
                                                         int sweeps_per_pass, int slab_planes) {
  if (check_streamed(g, dtype, sweeps_per_pass, slab_planes)) return 0;
  const int esz = dtype == MS_F64 ? 8 : 4;
  const int S = std::min(slab_planes, g->nz);
  const size_t buf = align_up(slab_elems(*g, std::min(sweeps_per_pass, g->nz), S) * esz + 256,
                              256);
  return 2 * (3 * buf + align_up(kPartialsBytes, 256));
}

extern "C" int jacobi_sweeps_streamed(const ms_grid* g, int dtype, void* u, void* u_tmp,
                                      const void* f, int64_t n, int sweeps_per_pass,
                                      int slab_planes, void* work, size_t work_bytes,
                                      void* stream) {
  clear_error();
  if (int rc = check_streamed(g, dtype, sweeps_per_pass, slab_planes)) return rc;
  if (!u || !u_tmp) return set_error(MS_EINVAL, "jacobi_sweeps_streamed: u and u_tmp required");
  if (n < 0) return set_error(MS_EINVAL, "jacobi_sweeps_streamed: n < 0");
  const int esz = dtype == MS_F64 ? 8 : 4;
  const size_t span = (size_t)field_span(*g);
  if (overlaps(u, span * esz, u_tmp, span * esz))
    return set_error(MS_EINVAL, "jacobi_sweeps_streamed: u and u_tmp overlap");
  const size_t need = jacobi_sweeps_streamed_workspace_bytes(g, dtype, sweeps_per_pass,
                                                             slab_planes);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "jacobi_sweeps_streamed: workspace needs %zu bytes", need);
  const int nz = g->nz;
  const int T = std::min(sweeps_per_pass, nz);  // a trapezoid wider than the field is the field
  const int S = std::min(slab_planes, nz);
  const int64_t sz = g->sz;
  hipStream_t caller = static_cast<hipStream_t>(stream);
  MS_HIP_TRY(hipStreamSynchronize(caller));
  if (n == 0) return MS_OK;

  Workspace ws{static_cast<char*>(work), work_bytes};
  const size_t elems = slab_elems(*g, T, S);
  SlabSet set[2];
  for (auto& q : set) {
    q.a = take_slab(ws, elems, esz);
    q.b = take_slab(ws, elems, esz);
    q.f = f ? take_slab(ws, elems, esz) : nullptr;
    if (!f) (void)take_slab(ws, elems, esz);
    q.partials = ws.take<double>((size_t)kPartialSlots * kMaxBlocks);
    if (!q.a || !q.b || (f && !q.f) || !q.partials)
      return set_error(MS_EWORKSPACE, "jacobi_sweeps_streamed: workspace carve failed");
  }
  hipStream_t st[2] = {nullptr, nullptr};
  for (auto& s : st)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto& t : st)
        if (t) (void)hipStreamDestroy(t);
      return set_error(MS_EHIP, "jacobi_sweeps_streamed: stream creation failed");
    }
  char* host[2] = {static_cast<char*>(u), static_cast<char*>(u_tmp)};
  const char* fh = static_cast<const char*>(f);
  const int64_t passes = (n + T - 1) / T;
  int rc = MS_OK;
  for (int64_t p = 0; p < passes && rc == MS_OK; ++p) {
    const int tp = (int)std::min<int64_t>(T, n - p * T);  // sweeps in this pass
    const char* src = host[p % 2];
    char* dst = host[(p + 1) % 2];
    int slab = 0;
    for (int a0 = 0; a0 < nz && rc == MS_OK; a0 += S, ++slab) {
      const int b0 = std::min(a0 + S, nz);
      const int ea = std::max(a0 - tp, 0), eb = std::min(b0 + tp, nz);
      SlabSet& q = set[slab % 2];
      hipStream_t s = st[slab % 2];
      // planes ea .. eb + 1 of the halo-inclusive field (the last one ends
      // where the field's span ends)
      const size_t off = (size_t)ea * sz;
      const size_t cnt = std::min((size_t)(eb + 2) * sz, span) - off;
      ms_grid sub = *g;
      sub.nz = eb - ea;
      hipError_t e = hipMemcpyAsync(q.a, src + off * esz, cnt * esz, hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(q.b, q.a, cnt * esz, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess && f)
        e = hipMemcpyAsync(q.f, fh + off * esz, cnt * esz, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) {
        rc = set_error(MS_EHIP, "jacobi_sweeps_streamed: upload: %s", hipGetErrorString(e));
        break;
      }
      const void* ptrs[3] = {q.a, q.b, q.f};
      const SweepGeom geo = sweep_geom(sub, dtype, vec_alignment(sub, dtype, ptrs, f ? 3 : 2));
      void* bufs[3] = {q.a, q.b, q.a};
      for (int k = 0; k < tp && rc == MS_OK; ++k)
        rc = launch_sweep(sub, dtype, bufs, 2, q.f, q.partials, nullptr, nullptr, k, geo, s);
      if (rc) break;
      const char* res = static_cast<const char*>(tp % 2 ? q.b : q.a);
      // interior planes a0 .. b0 - 1 are halo-inclusive planes a0 + 1 .. b0
      const size_t doff = (size_t)(a0 + 1 - ea) * sz, hoff = (size_t)(a0 + 1) * sz;
      e = hipMemcpyAsync(dst + hoff * esz, res + doff * esz, (size_t)(b0 - a0) * sz * esz,
                         hipMemcpyDeviceToHost, s);
      if (e != hipSuccess)
        rc = set_error(MS_EHIP, "jacobi_sweeps_streamed: download: %s", hipGetErrorString(e));
    }
    // the next pass reads what this one wrote
    for (auto& s : st) {
      const hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess && rc == MS_OK)
        rc = set_error(MS_EHIP, "jacobi_sweeps_streamed: %s", hipGetErrorString(e));
    }
  }
  for (auto& s : st) (void)hipStreamDestroy(s);
  return rc;
}
