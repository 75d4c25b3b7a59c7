// Entry points of the Jacobi hot path: fixed sweeps, the residual norm and
// the convergence-controlled solve (plain FP64, and FP32 storage with FP64
// iterative refinement).
//
// Convergence control runs on the device. Sweep launch k evaluates the norm
// of iterate k-1 and sets a done flag in a control block; later launches
// read the flag first and return at once. The host replays a chunk of m
// launches (as a hipGraph) and looks at the flag once per chunk. Because
// the decision about u_{k-1} is taken while launch k already writes
// u_{k+1}, the solve keeps three buffers (the answer is never the buffer
// being written).
#include "ms_internal.hpp"

#include <chrono>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#pragma clang fp contract(off)

namespace ms {
namespace {

__global__ void ctl_init_kernel(Ctl* c, double tol, int64_t max_sweeps, int ref_from_first,
                                int stall, int keep_res0) {
  c->base = 0;
  c->K = -1;
  c->max_sweeps = max_sweeps;
  c->tol = tol;
  if (!keep_res0) c->res0 = 0.0;
  c->last = 0.0;
  c->done = RUNNING;
  c->ref_from_first = ref_from_first;
  c->stall = stall;
  c->pad = 0;
}

__global__ void ctl_advance_kernel(Ctl* c, int64_t m) { c->base += m; }

// rhat = fl32((f - L(x)) / s) on the interior (s a power of two, applied as
// a multiplication by its exact reciprocal); also zeroes e0's interior.
template <bool HAS_F>
__global__ __launch_bounds__(256) void refine_rhs_kernel(const double* __restrict__ x,
                                                         const double* __restrict__ f,
                                                         float* __restrict__ rhat,
                                                         float* __restrict__ e0, double inv_s,
                                                         int nx, int ny, int nz, int64_t sy,
                                                         int64_t sz, int64_t sy32,
                                                         int64_t sz32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= nx) return;
  const int64_t p = (int64_t)(k + 1) * sz + (int64_t)(j + 1) * sy + (i + 1);
  const double s = ((((x[p + 1] + x[p - 1]) + x[p + sy]) + x[p - sy]) + x[p + sz]) + x[p - sz];
  const double lap = s - x[p] * 6.0;
  const double r = HAS_F ? f[p] - lap : -lap;
  const int64_t q = (int64_t)(k + 1) * sz32 + (int64_t)(j + 1) * sy32 + (i + 1);
  rhat[q] = (float)(r * inv_s);
  e0[q] = 0.0f;
}

// x += s * e on the interior (e: the inner buffer holding the accepted
// iterate).
__global__ __launch_bounds__(256) void refine_update_kernel(double* __restrict__ x,
                                                            const float* __restrict__ e,
                                                            double s, int nx, int64_t sy,
                                                            int64_t sz, int64_t sy32,
                                                            int64_t sz32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= nx) return;
  const int64_t p = (int64_t)(k + 1) * sz + (int64_t)(j + 1) * sy + (i + 1);
  const int64_t q = (int64_t)(k + 1) * sz32 + (int64_t)(j + 1) * sy32 + (i + 1);
  x[p] = x[p] + s * (double)e[q];
}

__global__ void fill_f32_kernel(float* p, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0.0f;
}

int elem_size(int dtype) { return dtype == MS_F64 ? 8 : 4; }

bool is_finite_host(double v) { return std::isfinite(v); }

// s = 2^e with s <= norm / sqrt(N) < 2s (1 if that ratio is 0 or not finite).
double pow2_scale(double norm, double ncells) {
  const double m = norm / std::sqrt(ncells);
  if (m == 0.0 || !std::isfinite(m)) return 1.0;
  int e = 0;
  std::frexp(m, &e);
  return std::ldexp(1.0, e - 1);
}

// Replays chunks of m sweep launches until the control block reports done.
struct ChunkRunner {
  const ms_grid& g;
  int dtype;
  void* bufs[3];
  const void* f;
  double* partials;
  double* hist;
  Ctl* ctl;
  SweepGeom geo;
  int m;
  bool use_graph;
  hipStream_t s;
  int tb;  // sweeps per launch: 1, or 2 (temporal blocking)
  bool rb;  // red-black Gauss-Seidel sweeps (one per launch)

  int enqueue_chunk() {
    for (int i = 0; i < m; ++i) {
      int rc = rb        ? launch_rbgs(g, dtype, bufs, 3, f, partials, hist, ctl, i, s)
               : tb == 2 ? launch_sweep_tb2(g, dtype, bufs, 3, f, partials, hist, ctl, i, s)
                         : launch_sweep(g, dtype, bufs, 3, f, partials, hist, ctl, i, geo, s);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(ctl_advance_kernel, dim3(1), dim3(1), 0, s, ctl, (int64_t)m);
    MS_LAUNCH_CHECK();
    return MS_OK;
  }

  int run(Ctl* host_ctl) {
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    if (use_graph) {
      MS_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      int rc = MS_OK;
      if (e == hipSuccess) {
        hipStream_t keep = s;
        s = cap;
        rc = enqueue_chunk();
        s = keep;
        e = hipStreamEndCapture(cap, &graph);
      }
      if (e == hipSuccess && rc == MS_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cap);
      if (rc) return rc;
      if (e != hipSuccess)
        return set_error(MS_EHIP, "graph capture of the sweep chunk failed: %s",
                         hipGetErrorString(e));
    }
    int rc = MS_OK;
    // Every launch advances the sweep index, so the control block must report
    // completion within max_sweeps + 2 launches; anything longer means the
    // sweeps did not run.
    int64_t launched = 0;
    for (;;) {
      if (launched * tb > host_ctl->max_sweeps + 2 * (int64_t)m * tb + 2) {
        rc = set_error(MS_EHIP, "sweep chunks ran without the control block completing");
        break;
      }
      launched += m;
      if (exec) {
        hipError_t e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) {
          rc = set_error(MS_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
          break;
        }
      } else {
        rc = enqueue_chunk();
        if (rc) break;
      }
      hipError_t e = hipMemcpyAsync(host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        rc = set_error(MS_EHIP, "control read-back: %s", hipGetErrorString(e));
        break;
      }
      if (host_ctl->done != RUNNING) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    return rc;
  }
};

// Buffer holding iterate K once a chunked solve is done. One sweep per
// launch: bufs[K % 3]. Two per launch: launch L keeps u_{2L} in bufs[L % 3];
// an odd K was never stored, so one plain sweep recomputes it from u_{K-1}
// into a buffer no later launch needs.
int locate_iterate(const ms_grid& g, int dtype, void* const bufs[3], const void* f,
                   double* partials, const SweepGeom& geo, int tb, int64_t K, hipStream_t s,
                   void** out) {
  if (tb != 2) {
    *out = bufs[K % 3];
    return MS_OK;
  }
  const int64_t L = K / 2;
  if (K % 2 == 0) {
    *out = bufs[L % 3];
    return MS_OK;
  }
  void* b2[3] = {bufs[L % 3], bufs[(L + 1) % 3], bufs[L % 3]};
  if (int rc = launch_sweep(g, dtype, b2, 2, f, partials, nullptr, nullptr, 0, geo, s)) return rc;
  *out = b2[1];
  return MS_OK;
}

int tb_of(const ms_solve_opts& o) {
  return o.method == MS_METHOD_JACOBI && o.temporal_block == 2 ? 2 : 1;
}
bool rb_of(const ms_solve_opts& o) { return o.method == MS_METHOD_RBGS; }

int auto_chunk(const ms_grid& g, int requested) {
  if (requested > 0) return requested;
  const double cells = (double)g.nx * g.ny * g.nz;
  return cells >= 16.0e6 ? 64 : 256;
}

// Fields carved from a workspace start `phase` elements past a 256-byte
// boundary, so that their interior rows share the vector alignment of the
// caller's field (phase = that field's element offset modulo 32).
constexpr size_t kFieldSlack = 256;

int elem_phase(const void* p, int esz) {
  return (int)((reinterpret_cast<uintptr_t>(p) / esz) % (256 / esz));
}

// FP32 correction grids of the refined solve use their own pitch: rows and
// planes padded to 32 elements and the base one element before a 128-byte
// boundary, so FP32 sweeps get 16-byte lanes whatever the FP64 layout.
ms_grid f32_grid(const ms_grid& g) {
  ms_grid h = g;
  h.sy = ((int64_t)g.nx + 2 + 31) / 32 * 32;
  h.sz = (h.sy * ((int64_t)g.ny + 2) + 31) / 32 * 32;
  return h;
}

struct SolveLayout {
  size_t total;
};

SolveLayout solve_layout(const ms_grid& g, const ms_solve_opts& o) {
  SolveLayout L{};
  size_t t = align_up(sizeof(Ctl), 256) + align_up(kPartialsBytes, 256);
  if (o.precision == MS_SOLVE_F64) {
    const size_t field = align_up((size_t)field_span(g) * 8 + kFieldSlack, 256);
    t += 2 * field + align_up(((size_t)o.max_sweeps + 2) * sizeof(double), 256);
  } else {
    const ms_grid h = f32_grid(g);
    const size_t field = align_up((size_t)field_span(h) * 4 + kFieldSlack, 256);
    t += 4 * field + align_up(((size_t)o.max_inner + 2) * sizeof(double), 256) +
         align_up(sizeof(Ctl), 256);
  }
  L.total = t;
  return L;
}

int check_opts(const ms_solve_opts* o) {
  if (!o) return set_error(MS_EINVAL, "jacobi_solve: opts is NULL");
  if (o->precision != MS_SOLVE_F64 && o->precision != MS_SOLVE_F32_REFINED)
    return set_error(MS_EUNSUPPORTED, "jacobi_solve: unknown precision %d", o->precision);
  if (!(o->rel_tol >= 0.0) || !std::isfinite(o->rel_tol))
    return set_error(MS_EINVAL, "jacobi_solve: rel_tol must be finite and >= 0");
  if (o->max_sweeps < 0) return set_error(MS_EINVAL, "jacobi_solve: max_sweeps < 0");
  if (o->check_every < 0) return set_error(MS_EINVAL, "jacobi_solve: check_every < 0");
  if (o->temporal_block < 0 || o->temporal_block > 2)
    return set_error(MS_EUNSUPPORTED, "jacobi_solve: temporal_block %d not available",
                     o->temporal_block);
  if (o->method != MS_METHOD_JACOBI && o->method != MS_METHOD_RBGS)
    return set_error(MS_EUNSUPPORTED, "jacobi_solve: unknown method %d", o->method);
  if (o->precision == MS_SOLVE_F32_REFINED) {
    if (!(o->inner_eta > 0.0 && o->inner_eta < 1.0))
      return set_error(MS_EINVAL, "jacobi_solve: inner_eta must be in (0, 1)");
    if (o->max_outer < 0 || o->max_inner < 1 || o->stall_window < 0)
      return set_error(MS_EINVAL, "jacobi_solve: bad refinement caps");
  }
  return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

// ------------------------------------------------------------ residual_norm

extern "C" size_t residual_workspace_bytes(const ms_grid* g) {
  if (check_grid(g, "residual_workspace_bytes")) return 0;
  return align_up(kPartialsBytes / 2, 256) + align_up(sizeof(double), 256);
}

extern "C" int residual_norm(const ms_grid* g, int dtype, const void* u, const void* f,
                             double* norm_out, int out_on_device, void* work,
                             size_t work_bytes, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "residual_norm")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "residual_norm: dtype %d", dtype);
  if (!u || !norm_out) return set_error(MS_EINVAL, "residual_norm: u and norm_out required");
  const size_t need = residual_workspace_bytes(g);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "residual_norm: workspace needs %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws{static_cast<char*>(work), work_bytes};
  double* partials = ws.take<double>(kMaxBlocks);
  double* dnorm = ws.take<double>(1);
  if (int rc = launch_residual(*g, dtype, u, f, false, partials, 0, s)) return rc;
  if (int rc = launch_finalize(partials, 0, residual_blocks(*g),
                               out_on_device ? norm_out : dnorm, nullptr, nullptr, 0, s))
    return rc;
  if (!out_on_device) {
    MS_HIP_TRY(hipMemcpyAsync(norm_out, dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    MS_HIP_TRY(hipStreamSynchronize(s));
  }
  return MS_OK;
}

// ------------------------------------------------------------ jacobi_sweeps

extern "C" size_t jacobi_sweeps_workspace_bytes(const ms_grid* g) {
  if (check_grid(g, "jacobi_sweeps_workspace_bytes")) return 0;
  return align_up(kPartialsBytes, 256);
}

namespace ms {
namespace {

// Arguments of jacobi_sweeps_tb other than the workspace; returns 0 or an
// MS_* code with the error text set.
int check_sweeps_args(const ms_grid* g, int dtype, void* u, void* u_tmp, const void* f,
                      int64_t n, int temporal_block) {
  if (int rc = check_grid(g, "jacobi_sweeps")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "jacobi_sweeps: dtype %d", dtype);
  if (temporal_block != 1 && temporal_block != 2)
    return set_error(MS_EUNSUPPORTED, "jacobi_sweeps: temporal_block %d", temporal_block);
  if (!u || !u_tmp) return set_error(MS_EINVAL, "jacobi_sweeps: u and u_tmp required");
  if (n < 0) return set_error(MS_EINVAL, "jacobi_sweeps: n < 0");
  const size_t bytes = (size_t)field_span(*g) * elem_size(dtype);
  if (overlaps(u, bytes, u_tmp, bytes))
    return set_error(MS_EINVAL, "jacobi_sweeps: u and u_tmp overlap");
  if (f && (overlaps(f, bytes, u, bytes) || overlaps(f, bytes, u_tmp, bytes)))
    return set_error(MS_EINVAL, "jacobi_sweeps: f overlaps a sweep buffer");
  return MS_OK;
}

// n sweeps on checked arguments; `partials` holds kPartialsBytes. Nothing in
// it needs to start at zero: every launch writes the slot it later reads.
int sweeps_on(const ms_grid* g, int dtype, void* u, void* u_tmp, const void* f, int64_t n,
              int temporal_block, double* res_dev, double* partials, hipStream_t s) {
  const void* ptrs[3] = {u, u_tmp, f};
  const SweepGeom geo = sweep_geom(*g, dtype, vec_alignment(*g, dtype, ptrs, 3));
  void* bufs[3] = {u, u_tmp, u};
  void* last = u;
  if (temporal_block == 1) {
    for (int64_t k = 0; k < n; ++k)
      if (int rc = launch_sweep(*g, dtype, bufs, 2, f, partials, res_dev, nullptr, k, geo, s))
        return rc;
    if (res_dev && n >= 1)
      if (int rc = launch_finalize(partials, (int)((n - 1) & 3), geo.nblocks, nullptr, nullptr,
                                   res_dev, n - 1, s))
        return rc;
    last = (n & 1) ? u_tmp : u;
  } else {
    const int64_t nl = n / 2;
    for (int64_t l = 0; l < nl; ++l)
      if (int rc = launch_sweep_tb2(*g, dtype, bufs, 2, f, partials, res_dev, nullptr, l, s))
        return rc;
    if (res_dev && nl >= 1)
      for (int64_t k = 2 * nl - 2; k < 2 * nl; ++k)
        if (int rc = launch_finalize(partials, (int)(k & 3), tb2_blocks(*g, dtype), nullptr,
                                     nullptr, res_dev, k, s))
          return rc;
    last = bufs[nl % 2];
    if (n & 1) {
      void* b2[3] = {last, bufs[(nl + 1) % 2], last};
      if (int rc = launch_sweep(*g, dtype, b2, 2, f, partials, nullptr, nullptr, 0, geo, s))
        return rc;
      if (res_dev)
        if (int rc = launch_finalize(partials, 0, geo.nblocks, nullptr, nullptr, res_dev, n - 1, s))
          return rc;
      last = b2[1];
    }
  }
  if (res_dev) {
    const int slot = (int)(n & 3) == 0 ? 1 : (int)(n & 3);  // not slot 0 (odd tail above)
    if (int rc = launch_residual(*g, dtype, last, f, false, partials, slot, s)) return rc;
    if (int rc = launch_finalize(partials, slot, residual_blocks(*g), nullptr, nullptr, res_dev,
                                 n, s))
      return rc;
  }
  return MS_OK;
}

}  // namespace
}  // namespace ms

extern "C" int jacobi_sweeps_tb(const ms_grid* g, int dtype, void* u, void* u_tmp,
                                const void* f, int64_t n, int temporal_block, double* res_dev,
                                void* work, size_t work_bytes, void* stream) {
  clear_error();
  if (int rc = check_sweeps_args(g, dtype, u, u_tmp, f, n, temporal_block)) return rc;
  const size_t need = jacobi_sweeps_workspace_bytes(g);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "jacobi_sweeps: workspace needs %zu bytes", need);
  return sweeps_on(g, dtype, u, u_tmp, f, n, temporal_block, res_dev,
                   static_cast<double*>(work), static_cast<hipStream_t>(stream));
}

// ----------------------------------------------------- jacobi_sweeps_noalloc
//
// The same sweeps with the partials table in a fixed device array instead of
// a caller workspace, for callers that cannot allocate. Each device holds
// its own copy of the array; its address is looked up once per device, with
// that device current, and only that address is handed to kernels.

namespace ms {
namespace {

constexpr size_t kScratchBytes = kPartialsBytes;  // 2 MiB per device
constexpr int kScratchDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch array.
int scratch_address(void** out) {
  int dev = -1;
  MS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return set_error(MS_EUNSUPPORTED, "jacobi_sweeps_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(MS_EHIP, "jacobi_sweeps_noalloc: hipGetSymbolAddress failed: %s",
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MS_OK;
}

}  // namespace
}  // namespace ms

extern "C" size_t jacobi_sweeps_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int jacobi_sweeps_noalloc(const ms_grid* g, int dtype, void* u, void* u_tmp,
                                     const void* f, int64_t n, int temporal_block,
                                     double* res_dev, void* stream) {
  clear_error();
  if (int rc = check_sweeps_args(g, dtype, u, u_tmp, f, n, temporal_block)) return rc;
  const size_t need = jacobi_sweeps_workspace_bytes(g);
  if (need > kScratchBytes)
    return set_error(MS_EWORKSPACE,
                     "jacobi_sweeps_noalloc: needs %zu bytes of scratch, the fixed array "
                     "holds %zu",
                     need, kScratchBytes);
  void* p = nullptr;
  if (int rc = scratch_address(&p)) return rc;
  return sweeps_on(g, dtype, u, u_tmp, f, n, temporal_block, res_dev, static_cast<double*>(p),
                   static_cast<hipStream_t>(stream));
}

extern "C" int rbgs_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp, const void* f,
                           int64_t n, double* res_dev, void* work, size_t work_bytes,
                           void* stream) {
  clear_error();
  if (int rc = check_grid(g, "rbgs_sweeps")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "rbgs_sweeps: dtype %d", dtype);
  if (!u || !u_tmp) return set_error(MS_EINVAL, "rbgs_sweeps: u and u_tmp required");
  if (n < 0) return set_error(MS_EINVAL, "rbgs_sweeps: n < 0");
  const size_t bytes = (size_t)field_span(*g) * elem_size(dtype);
  if (overlaps(u, bytes, u_tmp, bytes))
    return set_error(MS_EINVAL, "rbgs_sweeps: u and u_tmp overlap");
  if (f && (overlaps(f, bytes, u, bytes) || overlaps(f, bytes, u_tmp, bytes)))
    return set_error(MS_EINVAL, "rbgs_sweeps: f overlaps a sweep buffer");
  const size_t need = jacobi_sweeps_workspace_bytes(g);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "rbgs_sweeps: workspace needs %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partials = static_cast<double*>(work);
  void* bufs[3] = {u, u_tmp, u};
  for (int64_t k = 0; k < n; ++k)
    if (int rc = launch_rbgs(*g, dtype, bufs, 2, f, partials, res_dev, nullptr, k, s)) return rc;
  if (res_dev) {
    if (n >= 1)
      if (int rc = launch_finalize(partials, (int)((n - 1) & 3), tb2_blocks(*g, dtype, true),
                                   nullptr, nullptr, res_dev, n - 1, s))
        return rc;
    void* last = (n & 1) ? u_tmp : u;
    const int slot = (int)(n & 3);  // partials[(n - 1) & 3] is final by now
    if (int rc = launch_residual(*g, dtype, last, f, false, partials, slot, s)) return rc;
    if (int rc = launch_finalize(partials, slot, residual_blocks(*g), nullptr, nullptr, res_dev,
                                 n, s))
      return rc;
  }
  return MS_OK;
}

extern "C" int jacobi_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp, const void* f,
                             int64_t n, double* res_dev, void* work, size_t work_bytes,
                             void* stream) {
  return jacobi_sweeps_tb(g, dtype, u, u_tmp, f, n, 1, res_dev, work, work_bytes, stream);
}

// ------------------------------------------------------------- jacobi_solve

extern "C" void ms_solve_opts_default(ms_solve_opts* o) {
  if (!o) return;
  o->rel_tol = 1e-8;
  o->max_sweeps = 10000000;
  o->precision = MS_SOLVE_F64;
  o->check_every = 0;
  o->inner_eta = 1e-5;
  o->max_outer = 20;
  o->max_inner = 5000000;
  o->stall_window = 256;
  o->temporal_block = 2;
  o->use_graph = 1;
  o->method = MS_METHOD_JACOBI;
}

extern "C" size_t jacobi_workspace_bytes(const ms_grid* g, const ms_solve_opts* o) {
  if (check_grid(g, "jacobi_workspace_bytes") || check_opts(o)) return 0;
  return solve_layout(*g, *o).total;
}

namespace ms {
namespace {

template <typename T>
T* take_field(Workspace& ws, const ms_grid& g, int phase) {
  char* p = ws.take<char>((size_t)field_span(g) * sizeof(T) + kFieldSlack);
  return p ? reinterpret_cast<T*>(p) + phase : nullptr;
}

int solve_f64(const ms_grid& g, const ms_solve_opts& o, double* u, const double* f,
              Workspace& ws, double* hist_host, ms_solve_result* res, hipStream_t s) {
  const size_t span = (size_t)field_span(g);
  Ctl* ctl = ws.take<Ctl>(1);
  double* partials = ws.take<double>((size_t)kPartialSlots * kMaxBlocks);
  double* b1 = take_field<double>(ws, g, elem_phase(u, 8));
  double* b2 = take_field<double>(ws, g, elem_phase(u, 8));
  double* hist = ws.take<double>((size_t)o.max_sweeps + 2);
  if (!ctl || !partials || !b1 || !b2 || !hist)
    return set_error(MS_EWORKSPACE, "jacobi_solve: workspace carve failed");
  const void* ptrs[4] = {u, b1, b2, f};
  const SweepGeom geo = sweep_geom(g, MS_F64, vec_alignment(g, MS_F64, ptrs, 4));
  // Every buffer carries the Dirichlet halo; sweeps never write it.
  MS_HIP_TRY(hipMemcpyAsync(b1, u, span * 8, hipMemcpyDeviceToDevice, s));
  MS_HIP_TRY(hipMemcpyAsync(b2, u, span * 8, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(1), 0, s, ctl, o.rel_tol, o.max_sweeps, 0,
                     0, 0);
  MS_LAUNCH_CHECK();
  // res0 = ||r(u^0)||, u^0 = u with its interior zeroed.
  if (int rc = launch_residual(g, MS_F64, u, f, true, partials, 0, s)) return rc;
  if (int rc = launch_finalize(partials, 0, residual_blocks(g), &ctl->res0, nullptr, nullptr,
                               0, s))
    return rc;

  Ctl hc{};
  hc.max_sweeps = o.max_sweeps;
  const int tb = tb_of(o);
  ChunkRunner run{g, MS_F64, {u, b1, b2}, f, partials, hist, ctl, geo,
                  auto_chunk(g, o.check_every), o.use_graph != 0, s, tb, rb_of(o)};
  if (int rc = run.run(&hc)) return rc;
  const int64_t K = hc.K;
  void* ans = nullptr;
  if (int rc = locate_iterate(g, MS_F64, run.bufs, f, partials, geo, tb, K, s, &ans)) return rc;
  if (ans != u) MS_HIP_TRY(hipMemcpyAsync(u, ans, span * 8, hipMemcpyDeviceToDevice, s));
  double res_final = 0.0;
  MS_HIP_TRY(hipMemcpyAsync(&res_final, hist + K, sizeof(double), hipMemcpyDeviceToHost, s));
  if (hist_host)
    MS_HIP_TRY(hipMemcpyAsync(hist_host, hist, (size_t)(K + 1) * sizeof(double),
                              hipMemcpyDeviceToHost, s));
  MS_HIP_TRY(hipStreamSynchronize(s));
  res->sweeps = K;
  res->outer_iters = 0;
  res->res0 = hc.res0;
  res->res_final = res_final;
  res->rel_final = hc.res0 > 0.0 ? res_final / hc.res0 : 0.0;
  int status = MS_OK;
  if (hc.done == NONFINITE)
    status = set_error(MS_ENONFINITE, "jacobi_solve: residual norm is not finite at sweep %lld",
                       (long long)K);
  else if (hc.done != CONVERGED)
    status = set_error(MS_NOT_CONVERGED, "jacobi_solve: not converged after %lld sweeps",
                       (long long)K);
  res->status = status;
  return status;
}

int solve_refined(const ms_grid& g, const ms_solve_opts& o, double* x, const double* f,
                  Workspace& ws, double* hist_host, ms_solve_result* res, hipStream_t s) {
  const ms_grid h = f32_grid(g);
  const size_t span32 = (size_t)field_span(h);
  Ctl* ctl = ws.take<Ctl>(1);
  double* partials = ws.take<double>((size_t)kPartialSlots * kMaxBlocks);
  // base one element before a 128-byte boundary: phase 31 of 64 floats
  float* rhat = take_field<float>(ws, h, 31);
  float* e[3] = {take_field<float>(ws, h, 31), take_field<float>(ws, h, 31),
                 take_field<float>(ws, h, 31)};
  double* hist = ws.take<double>((size_t)o.max_inner + 2);
  Ctl* octl = ws.take<Ctl>(1);
  if (!ctl || !partials || !rhat || !e[0] || !e[1] || !e[2] || !hist || !octl)
    return set_error(MS_EWORKSPACE, "jacobi_solve: workspace carve failed");
  if (g.ny > 65535 || g.nz > 65535)
    return set_error(MS_EUNSUPPORTED, "jacobi_solve: refined path needs ny, nz <= 65535");
  const void* ptrs[4] = {rhat, e[0], e[1], e[2]};
  const SweepGeom geo = sweep_geom(h, MS_F32, vec_alignment(h, MS_F32, ptrs, 4));
  // The correction has homogeneous boundary values: zero every FP32 grid
  // once (halos included); the sweeps never write a halo.
  for (float* p : {rhat, e[0], e[1], e[2]}) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(1024), dim3(256), 0, s, p, (int64_t)span32);
    MS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(1), 0, s, octl, 0.0, (int64_t)0, 0, 0, 0);
  MS_LAUNCH_CHECK();
  if (int rc = launch_residual(g, MS_F64, x, f, true, partials, 0, s)) return rc;
  if (int rc = launch_finalize(partials, 0, residual_blocks(g), &octl->res0, nullptr, nullptr,
                               0, s))
    return rc;
  double res0 = 0.0;
  MS_HIP_TRY(hipMemcpyAsync(&res0, &octl->res0, sizeof(double), hipMemcpyDeviceToHost, s));
  MS_HIP_TRY(hipStreamSynchronize(s));

  const double ncells = (double)g.nx * g.ny * g.nz;
  const dim3 eb(256), eg((g.nx + 255) / 256, g.ny, g.nz);
  int64_t total = 0;
  int outer = 0;
  int status = MS_OK;
  double nr = 0.0, rel = 0.0;
  for (;;) {
    if (int rc = launch_residual(g, MS_F64, x, f, false, partials, 0, s)) return rc;
    if (int rc = launch_finalize(partials, 0, residual_blocks(g), &octl->last, nullptr, nullptr,
                                 0, s))
      return rc;
    MS_HIP_TRY(hipMemcpyAsync(&nr, &octl->last, sizeof(double), hipMemcpyDeviceToHost, s));
    MS_HIP_TRY(hipStreamSynchronize(s));
    rel = res0 > 0.0 ? nr / res0 : 0.0;
    if (hist_host) hist_host[outer] = rel;
    if (!is_finite_host(nr)) {
      status = set_error(MS_ENONFINITE, "jacobi_solve: residual norm not finite (outer %d)", outer);
      break;
    }
    if (res0 == 0.0 || rel <= o.rel_tol) break;
    if (outer == o.max_outer || total >= o.max_sweeps) {
      status = set_error(MS_NOT_CONVERGED, "jacobi_solve: refinement stopped at rel %.3e", rel);
      break;
    }
    const double sc = pow2_scale(nr, ncells);
    if (f)
      hipLaunchKernelGGL(refine_rhs_kernel<true>, eg, eb, 0, s, x, f, rhat, e[0], 1.0 / sc,
                         g.nx, g.ny, g.nz, g.sy, g.sz, h.sy, h.sz);
    else
      hipLaunchKernelGGL(refine_rhs_kernel<false>, eg, eb, 0, s, x, f, rhat, e[0], 1.0 / sc,
                         g.nx, g.ny, g.nz, g.sy, g.sz, h.sy, h.sz);
    MS_LAUNCH_CHECK();
    int64_t cap = o.max_inner;
    if (o.max_sweeps - total < cap) cap = o.max_sweeps - total;
    // No more reduction than brings the outer residual to half the tolerance.
    const double eta = std::max(o.inner_eta, 0.5 * o.rel_tol / rel);
    hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(1), 0, s, ctl, eta, cap, 1,
                       o.stall_window, 0);
    MS_LAUNCH_CHECK();
    Ctl hc{};
    hc.max_sweeps = cap;
    const int tb = tb_of(o);
    ChunkRunner run{h, MS_F32, {e[0], e[1], e[2]}, rhat, partials, hist, ctl, geo,
                    auto_chunk(g, o.check_every), o.use_graph != 0, s, tb, rb_of(o)};
    if (int rc = run.run(&hc)) return rc;
    if (hc.done == NONFINITE) {
      status = set_error(MS_ENONFINITE, "jacobi_solve: inner residual not finite");
      break;
    }
    void* ek = nullptr;
    if (int rc = locate_iterate(h, MS_F32, run.bufs, rhat, partials, geo, tb, hc.K, s, &ek))
      return rc;
    hipLaunchKernelGGL(refine_update_kernel, eg, eb, 0, s, x, static_cast<const float*>(ek), sc,
                       g.nx, g.sy, g.sz, h.sy, h.sz);
    MS_LAUNCH_CHECK();
    total += hc.K;
    ++outer;
  }
  MS_HIP_TRY(hipStreamSynchronize(s));
  res->sweeps = total;
  res->outer_iters = outer;
  res->res0 = res0;
  res->res_final = nr;
  res->rel_final = rel;
  res->status = status;
  return status;
}

}  // namespace
}  // namespace ms

extern "C" int jacobi_solve(const ms_grid* g, const ms_solve_opts* o, double* u, const double* f,
                            void* work, size_t work_bytes, double* hist_host,
                            ms_solve_result* res, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "jacobi_solve")) return rc;
  if (int rc = check_opts(o)) return rc;
  if (!u || !res) return set_error(MS_EINVAL, "jacobi_solve: u and res required");
  const size_t bytes = (size_t)field_span(*g) * 8;
  if (f && overlaps(f, bytes, u, bytes))
    return set_error(MS_EINVAL, "jacobi_solve: f overlaps u");
  const SolveLayout L = solve_layout(*g, *o);
  if (!work || work_bytes < L.total)
    return set_error(MS_EWORKSPACE, "jacobi_solve: workspace needs %zu bytes", L.total);
  if (overlaps(work, L.total, u, bytes) || (f && overlaps(work, L.total, f, bytes)))
    return set_error(MS_EINVAL, "jacobi_solve: workspace overlaps a field");
  Workspace ws{static_cast<char*>(work), work_bytes};
  hipStream_t s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  *res = ms_solve_result{};
  const int rc = o->precision == MS_SOLVE_F64 ? solve_f64(*g, *o, u, f, ws, hist_host, res, s)
                                              : solve_refined(*g, *o, u, f, ws, hist_host, res, s);
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

// ---------------------------------------------------------------- autotuner

extern "C" int ms_autotune_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp,
                                  const void* f, int sweeps_per_trial, void* work,
                                  size_t work_bytes, ms_tuning* best, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "ms_autotune_sweeps")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "ms_autotune_sweeps: dtype %d", dtype);
  if (!u || !u_tmp || !best || sweeps_per_trial < 1)
    return set_error(MS_EINVAL, "ms_autotune_sweeps: bad arguments");
  if (!work || work_bytes < jacobi_sweeps_workspace_bytes(g))
    return set_error(MS_EWORKSPACE, "ms_autotune_sweeps: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* ptrs[3] = {u, u_tmp, f};
  const int vec_ok = vec_alignment(*g, dtype, ptrs, 3);
  double* partials = static_cast<double*>(work);
  void* bufs[3] = {u, u_tmp, u};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MS_HIP_TRY(hipEventCreate(&e0));
  MS_HIP_TRY(hipEventCreate(&e1));
  ms_tuning out{};
  out.us_per_sweep = 1e300;
  const int vmax = dtype == MS_F64 ? 2 : 4;
  int rc = MS_OK;
  for (int vec = vmax; vec >= 1 && rc == MS_OK; vec >>= 1) {
    if (vec > vec_ok) continue;
    for (int wx : {1, 2, 4})
      for (int rows : {2, 4, 8})
        for (int64_t tb : {64, 128, 256, 512, 1024, 2048}) {
          const SweepGeom geo = geom_register(*g, dtype, vec_ok, vec, wx, rows, 0, tb);
          if (geo.vec != vec || geo.nblocks > kMaxBlocks) continue;
          // one untimed sweep, then the timed trial
          for (int k = 0; k <= sweeps_per_trial && rc == MS_OK; ++k) {
            if (k == 1) (void)hipEventRecord(e0, s);
            rc = launch_sweep(*g, dtype, bufs, 2, f, partials, nullptr, nullptr, k, geo, s);
          }
          if (rc) break;
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) {
            rc = set_error(MS_EHIP, "ms_autotune_sweeps: timing failed");
            break;
          }
          float ms_el = 0.0f;
          (void)hipEventElapsedTime(&ms_el, e0, e1);
          const double us = 1e3 * ms_el / sweeps_per_trial;
          if (us < out.us_per_sweep) {
            out.dtype = dtype; out.nx = g->nx; out.ny = g->ny; out.nz = g->nz;
            out.vec_ok = vec_ok; out.vec = geo.vec; out.wx = geo.wx; out.rows = geo.rows;
            out.target_blocks = tb; out.us_per_sweep = us;
          }
        }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  tuned_store(out);
  *best = out;
  return MS_OK;
}

extern "C" int ms_sweep_shape(const ms_grid* g, int dtype, const void* const* bufs, int nbufs,
                              ms_tuning* out) {
  clear_error();
  if (int rc = check_grid(g, "ms_sweep_shape")) return rc;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "ms_sweep_shape: dtype %d", dtype);
  if (!out || nbufs < 0 || (nbufs > 0 && !bufs))
    return set_error(MS_EINVAL, "ms_sweep_shape: bad arguments");
  const int vec_ok = vec_alignment(*g, dtype, bufs, nbufs);
  const SweepGeom geo = sweep_geom(*g, dtype, vec_ok);
  ms_tuning t{};
  const bool tuned = tuned_lookup(*g, dtype, vec_ok, &t);
  *out = ms_tuning{};
  out->dtype = dtype; out->nx = g->nx; out->ny = g->ny; out->nz = g->nz;
  out->vec_ok = vec_ok; out->vec = geo.vec; out->wx = geo.wx; out->rows = geo.rows;
  out->target_blocks = geo.nblocks;
  out->us_per_sweep = tuned ? t.us_per_sweep : 0.0;
  return MS_OK;
}

extern "C" int ms_tuning_get(ms_tuning* out, int cap) { return tuned_export(out, cap); }

extern "C" int ms_tuning_set(const ms_tuning* in, int n) {
  clear_error();
  if (n < 0 || (n > 0 && !in)) return set_error(MS_EINVAL, "ms_tuning_set: bad arguments");
  for (int i = 0; i < n; ++i) {
    const ms_tuning& t = in[i];
    if ((t.dtype != MS_F64 && t.dtype != MS_F32) || t.nx < 1 || t.ny < 1 || t.nz < 1 ||
        (t.vec != 1 && t.vec != 2 && t.vec != 4) || (t.wx != 1 && t.wx != 2 && t.wx != 4) ||
        (t.rows != 2 && t.rows != 4 && t.rows != 8) || t.target_blocks < 1)
      return set_error(MS_EINVAL, "ms_tuning_set: entry %d is not a valid shape", i);
    tuned_store(t);
  }
  return MS_OK;
}

extern "C" void ms_tuning_clear(void) { tuned_clear(); }
