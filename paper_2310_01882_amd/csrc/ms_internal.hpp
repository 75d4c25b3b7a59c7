// Internal declarations shared by the mistencil HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "mistencil.h"

namespace ms {

// ---------------------------------------------------------------- errors

int set_error(int code, const char* fmt, ...);
void clear_error();

#define MS_HIP_TRY(expr)                                                    \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return ::ms::set_error(MS_EHIP, "%s failed: %s (%s:%d)", #expr,       \
                             hipGetErrorString(e_), __FILE__, __LINE__);    \
  } while (0)

#define MS_LAUNCH_CHECK()                                                   \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess)                                                   \
      return ::ms::set_error(MS_EHIP, "kernel launch failed: %s (%s:%d)",   \
                             hipGetErrorString(e_), __FILE__, __LINE__);    \
  } while (0)

// Validates extents and strides of a grid descriptor.
int check_grid(const ms_grid* g, const char* who);

// Number of elements from the base pointer to one past the last halo cell
// (the last plane and row carry no trailing pitch).
inline int64_t field_span(const ms_grid& g) {
  return (int64_t)(g.nz + 1) * g.sz + (int64_t)(g.ny + 1) * g.sy + (g.nx + 2);
}

// True if [a, a + abytes) and [b, b + bbytes) overlap.
inline bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------ device-side control

// Convergence state shared by the launches of one solve. Sweep launch k
// (k = base + offset) evaluates the norm of u_{k-1} that launch k-1 left as
// per-block partials; a kernel boundary separates writer and reader, so no
// intra-kernel cross-block synchronisation is needed.
enum DoneCode : int32_t {
  RUNNING = 0,
  CONVERGED = 1,
  MAXED = 2,
  STALLED = 3,
  NONFINITE = 4,
};

struct Ctl {
  int64_t base;        // sweep index of the first launch of the current chunk
  int64_t K;           // index of the accepted iterate once done != RUNNING
  int64_t max_sweeps;  // last index that may be checked
  double tol;          // relative tolerance
  double res0;         // reference norm
  double last;         // last evaluated norm
  int32_t done;
  int32_t ref_from_first;  // res0 := norm of iterate 0 (inner solves)
  int32_t stall;           // stagnation window in sweeps (0: off)
  int32_t pad;
};

// -------------------------------------------------------- launch geometry

constexpr int kWave = 64;   // wavefront width on CDNA
constexpr int kTileX = 64;  // one wave spans a tile row in x
constexpr int kWavesY = 4;  // waves per block
constexpr int kThreads = kTileX * kWavesY;
// Per-block partial sums live in a fixed-size table so that the workspace
// does not depend on the launch geometry.
constexpr int kMaxBlocks = 65536;

enum SweepVariant : int { kVariantLds = 0, kVariantRegister = 1 };

// Launch geometry of a z-marching sweep. Register-tiled: each wave owns a
// (64*vec) x rows tile, wx waves side by side in x, 4/wx stacked in y.
// LDS-tiled: a block owns a 64 x (4*rows) tile. Every block marches zc planes.
struct SweepGeom {
  int variant;
  int vec;   // x cells per lane (register-tiled)
  int wx;    // waves per block along x (register-tiled)
  int rows;  // rows per thread
  int tiles_x, tiles_y, chunks_z, zc;
  int nblocks;
};

// Largest vector width (elements per lane, up to 16 bytes) for which
// interior cell (0, j, k) of every given field sits on a vector boundary.
int vec_alignment(const ms_grid& g, int dtype, const void* const* ptrs, int n);

// Geometry of the sweeps of one call. vec_ok caps the vector width; the
// defaults can be overridden for tuning through MS_SWEEP_VARIANT (0 lds,
// 1 register), MS_SWEEP_VEC, MS_SWEEP_WX, MS_SWEEP_ROWS and MS_SWEEP_ZC.
SweepGeom sweep_geom(const ms_grid& g, int dtype, int vec_ok);
// LDS-tiled geometry with 4 rows per thread (standalone residual passes).
SweepGeom sweep_geom_lds(const ms_grid& g);
// Register-tiled geometry with explicit parameters (0 picks a default).
SweepGeom geom_register(const ms_grid& g, int dtype, int vec_ok, int vec, int wx, int rows,
                        int zc_hint, int64_t target_blocks);

// Process-wide table of tuned sweep geometries (filled by the autotuner,
// consulted by sweep_geom unless an MS_SWEEP_* override is set).
bool tuned_lookup(const ms_grid& g, int dtype, int vec_ok, ms_tuning* out);
void tuned_store(const ms_tuning& t);
int tuned_export(ms_tuning* out, int cap);
void tuned_clear();

// Maps hardware block ids so that consecutive tiles share an XCD: blocks are
// dispatched round-robin over the 8 XCDs, each with its own L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int xcd = b & 7, slot = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// Deterministic block-wide sum of one double per thread (fixed tree order).
// `red` must hold blockDim.x / 64 doubles of LDS. Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) t += red[w];
  }
  __syncthreads();
  return t;
}

// Sum of `n` partials in a fixed order independent of the launch history.
__device__ __forceinline__ double sum_partials(const double* p, int n, double* red) {
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += p[i];
  return block_sum(t, red);
}

// Evaluate iterate `k`'s norm against the control block (thread 0 only).
__device__ __forceinline__ void judge(Ctl* c, double* hist, int64_t k, double norm) {
  if (hist) hist[k] = norm;
  if (!c) return;
  if (c->done != RUNNING) return;
  if (c->ref_from_first && k == 0) c->res0 = norm;
  c->last = norm;
  const double res0 = c->res0;
  if (!isfinite(norm)) {
    c->done = NONFINITE;
    c->K = k;
  } else if (res0 == 0.0 || norm / res0 <= c->tol) {
    c->done = CONVERGED;
    c->K = k;
  } else if (k >= c->max_sweeps) {
    c->done = MAXED;
    c->K = k;
  } else if (c->stall > 0 && hist && k >= c->stall && norm >= hist[k - c->stall]) {
    c->done = STALLED;
    c->K = k;
  }
}

// ---------------------------------------------------------- kernel entry

struct Workspace {
  char* p;
  size_t left;
  template <typename T>
  T* take(size_t count) {
    size_t bytes = align_up(count * sizeof(T), 256);
    if (bytes > left) return nullptr;
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

// Sweeps (FP64 or FP32 storage) -------------------------------------------
// One sweep per launch: launch index base + k_off = iterate index k; reads
// bufs[k % nbuf], writes bufs[(k + 1) % nbuf].
int launch_sweep(const ms_grid& g, int dtype, void* const bufs[3], int nbuf,
                 const void* f, double* partials, double* hist, Ctl* ctl,
                 int64_t k_off, const SweepGeom& geo, hipStream_t s);

// Two fused sweeps per launch (temporal blocking): launch index L = base +
// k_off covers iterates 2L (read from bufs[L % nbuf]) and 2L + 1 (never
// stored) and writes u_{2L+2} to bufs[(L + 1) % nbuf]; it adds the norms of
// both iterates and judges 2L - 2 and 2L - 1.
int launch_sweep_tb2(const ms_grid& g, int dtype, void* const bufs[3], int nbuf,
                     const void* f, double* partials, double* hist, Ctl* ctl,
                     int64_t k_off, hipStream_t s);
// One red-black Gauss-Seidel sweep per launch on the two-sweep kernel's
// geometry: launch index k = base + k_off reads u_k from bufs[k % nbuf],
// writes u_{k+1} to bufs[(k + 1) % nbuf], adds the norm of u_k into
// partials[k & 3] and judges k - 1 (as launch_sweep does).
int launch_rbgs(const ms_grid& g, int dtype, void* const bufs[3], int nbuf, const void* f,
                double* partials, double* hist, Ctl* ctl, int64_t k_off, hipStream_t s);
// Blocks of the two-sweep kernel (for finalising its last partials).
int tb2_blocks(const ms_grid& g, int dtype, bool rb = false);

// Standalone residual: per-block partials of sum r^2 into partials[slot];
// zero_interior evaluates u with its interior replaced by 0. It launches
// residual_blocks(g) blocks.
int launch_residual(const ms_grid& g, int dtype, const void* u, const void* f,
                    bool zero_interior, double* partials, int slot, hipStream_t s);
int residual_blocks(const ms_grid& g);

// Partials table: four slots of kMaxBlocks doubles; iterate k's partials go
// to slot k & 3 (a two-sweep launch fills two slots, and block 0 of the next
// launch still reads the previous two).
constexpr int kPartialSlots = 4;
constexpr size_t kPartialsBytes = kPartialSlots * (size_t)kMaxBlocks * sizeof(double);

// One-block finalisation: norm = sqrt(sum partials[slot]); writes *out_norm
// (if not null) and judges iterate k against ctl (if not null).
int launch_finalize(const double* partials, int slot, int nblocks, double* out_norm,
                    Ctl* ctl, double* hist, int64_t k, hipStream_t s);

}  // namespace ms
