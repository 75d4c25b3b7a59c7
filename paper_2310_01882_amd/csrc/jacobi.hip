// 7-point Jacobi sweeps with the fused residual-norm reduction, the
// standalone residual pass and their finalisation.
//
// Each block owns a 64 x 16 (x, y) tile of the interior and marches along
// z over a chunk of planes. The current plane of the tile plus its one-cell
// ring is staged in LDS (double-buffered: one barrier per plane); the z
// neighbours stay in registers (previous / current / next plane) and the
// plane after next is prefetched while the current one is computed. A wave
// spans one 64-cell row, so every global access of the centre and of the
// y-halo rows is a fully coalesced 512-byte (FP64) row segment.
//
// Per cell (the 7-point Laplace iteration of the paper's evaluation,
// Section 4.1, as an out-of-place update, Section 2.2):
//   S  = (((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1]) + u[k-1])
//   u' = (S - f) * fl(1/6)          (S * fl(1/6) without f)
//   r  = f - (S - u*6)              (residual of the input field)
// and sum r^2 (FP64) goes to one partial per block.
#include "ms_internal.hpp"

// Bit-exact parity with the oracle needs every operation rounded on its own.
#pragma clang fp contract(off)

namespace ms {

namespace {

template <typename T>
struct SweepK {
  T* buf[3];
  const T* f;
  double* partials;  // [2][nblocks] (sweeps) or [slot][nblocks] (residual)
  double* hist;
  Ctl* ctl;
  int64_t k_off;
  int nbuf;
  int slot;  // residual-only launches: partial slot
  int nx, ny, nz;
  int64_t sy, sz;
  int tiles_x, tiles_y, zc, nblocks;
};

template <typename T>
struct C6;
template <>
struct C6<double> {
  static __device__ __forceinline__ double v() { return 1.0 / 6.0; }
};
template <>
struct C6<float> {
  static __device__ __forceinline__ float v() { return 1.0f / 6.0f; }
};

// Residual of one cell in FP64. FP64 fields: r = f - (S - u*6) as written.
// FP32 fields: the same expression evaluated in FP64 on the exactly widened
// FP32 values (neighbour sum in the same order).
__device__ __forceinline__ double cell_residual(double xp, double xm, double yp, double ym,
                                                double zp, double zm, double c, double f,
                                                bool has_f) {
  const double s = ((((xp + xm) + yp) + ym) + zp) + zm;
  const double lap = s - c * 6.0;
  return has_f ? f - lap : -lap;
}

// WRITE: sweep (write u' and evaluate the residual of u); else residual only.
// ZERO_INT: read the field with its interior replaced by 0 (residual of u^0).
template <typename T, bool HAS_F, bool WRITE, bool ZERO_INT>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepK<T> a) {
  constexpr int R = kRowsPerThread;
  __shared__ T lds[2][kTileY + 2][kTileX + 2];
  __shared__ double red[kWavesY];
  __shared__ int s_done;

  const int64_t k = (a.ctl ? a.ctl->base : 0) + a.k_off;

  // Block 0 finalises the previous launch's norm (written by all blocks of
  // launch k-1, visible after the kernel boundary).
  if (WRITE && blockIdx.x == 0 && k >= 1 && (a.hist || a.ctl)) {
    if (!a.ctl || a.ctl->done == RUNNING) {
      const double t = sum_partials(a.partials + ((k - 1) & 1) * (int64_t)a.nblocks,
                                    a.nblocks, red);
      if (threadIdx.x == 0) judge(a.ctl, a.hist, k - 1, sqrt(t));
    }
  }
  if (a.ctl) {
    if (threadIdx.x == 0) s_done = a.ctl->done;
    __syncthreads();
    if (s_done != RUNNING) return;  // block-uniform
  }

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int i0 = txi * kTileX, j0 = tyi * kTileY;
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
  const int i = i0 + lane;

  const int slot = WRITE ? (int)(k & 1) : a.slot;
  const T* __restrict__ src = WRITE ? a.buf[k % a.nbuf] : a.buf[0];
  T* __restrict__ dst = WRITE ? a.buf[(k + 1) % a.nbuf] : nullptr;
  const T* __restrict__ f = a.f;
  const int64_t sy = a.sy, sz = a.sz;

  // Centre rows of this thread.
  int64_t coff[R];
  bool cload[R], cact[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = j0 + wy * R + r;
    coff[r] = (int64_t)(j + 1) * sy + (i + 1);
    cload[r] = (i <= a.nx) && (j <= a.ny);
    cact[r] = (i < a.nx) && (j < a.ny);
  }

  // Halo ring element owned by this thread (if any).
  int hi = 0, hj = 0, hrow = 0, hcol = 0;
  bool hown = false;
  {
    const int t = threadIdx.x;
    if (t < kTileX) {
      hi = i0 + t; hj = j0 - 1; hrow = 0; hcol = t + 1; hown = true;
    } else if (t < 2 * kTileX) {
      hi = i0 + t - kTileX; hj = j0 + kTileY; hrow = kTileY + 1; hcol = t - kTileX + 1;
      hown = true;
    } else if (t < 2 * kTileX + kTileY) {
      hi = i0 - 1; hj = j0 + (t - 2 * kTileX); hrow = hj - j0 + 1; hcol = 0; hown = true;
    } else if (t < 2 * kTileX + 2 * kTileY) {
      hi = i0 + kTileX; hj = j0 + (t - 2 * kTileX - kTileY); hrow = hj - j0 + 1;
      hcol = kTileX + 1; hown = true;
    }
  }
  const bool hload = hown && hi <= a.nx && hj <= a.ny;
  const int64_t hoff = (int64_t)(hj + 1) * sy + (hi + 1);

  auto interior_cell = [&](int ci, int cj, int ck) {
    return ci >= 0 && ci < a.nx && cj >= 0 && cj < a.ny && ck >= 0 && ck < a.nz;
  };
  auto ld_c = [&](int r, int kk) -> T {
    if (!cload[r]) return T(0);
    if (ZERO_INT && interior_cell(i, j0 + wy * R + r, kk)) return T(0);
    return src[(int64_t)(kk + 1) * sz + coff[r]];
  };
  auto ld_h = [&](int kk) -> T {
    if (!hload) return T(0);
    if (ZERO_INT && interior_cell(hi, hj, kk)) return T(0);
    return src[(int64_t)(kk + 1) * sz + hoff];
  };
  auto ld_f = [&](int r, int kk) -> T {
    if (!HAS_F || !cact[r]) return T(0);
    return f[(int64_t)(kk + 1) * sz + coff[r]];
  };

  T zp[R], zc[R], zn[R], fc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    zp[r] = ld_c(r, z0 - 1);
    zc[r] = ld_c(r, z0);
    zn[r] = ld_c(r, z0 + 1);
    fc[r] = ld_f(r, z0);
  }
  T hcur = ld_h(z0);

  double acc = 0.0;
  int b = 0;
  const T c6 = C6<T>::v();
  for (int kk = z0; kk < z1; ++kk) {
    T pf[R], fn[R];
    T hn = T(0);
    const bool more = kk + 1 < z1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      pf[r] = more ? ld_c(r, kk + 2) : T(0);
      fn[r] = more ? ld_f(r, kk + 1) : T(0);
    }
    if (more) hn = ld_h(kk + 1);

#pragma unroll
    for (int r = 0; r < R; ++r) lds[b][wy * R + r + 1][lane + 1] = zc[r];
    if (hown) lds[b][hrow][hcol] = hcur;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!cact[r]) continue;
      const int row = wy * R + r + 1;
      const T xp = lds[b][row][lane + 2], xm = lds[b][row][lane];
      const T yp = lds[b][row + 1][lane + 1], ym = lds[b][row - 1][lane + 1];
      if (WRITE) {
        const T s = ((((xp + xm) + yp) + ym) + zn[r]) + zp[r];
        const T v = HAS_F ? (s - fc[r]) * c6 : s * c6;
        dst[(int64_t)(kk + 1) * sz + coff[r]] = v;
      }
      const double res = cell_residual(xp, xm, yp, ym, zn[r], zp[r], zc[r], fc[r], HAS_F);
      acc += res * res;
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
      zp[r] = zc[r];
      zc[r] = zn[r];
      zn[r] = pf[r];
      fc[r] = fn[r];
    }
    hcur = hn;
    b ^= 1;
  }

  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) a.partials[(int64_t)slot * a.nblocks + blockIdx.x] = tot;
}

__global__ void finalize_kernel(const double* partials, int nb, double* out, Ctl* ctl,
                                double* hist, int64_t k) {
  __shared__ double red[kWavesY];
  const double t = sum_partials(partials, nb, red);
  if (threadIdx.x == 0) {
    const double n = sqrt(t);
    if (out) *out = n;
    judge(ctl, hist, k, n);
  }
}

template <typename T, bool HAS_F, bool WRITE, bool ZERO_INT>
int launch_t(const SweepK<T>& a, const SweepGeom& geo, hipStream_t s) {
  hipLaunchKernelGGL((sweep_kernel<T, HAS_F, WRITE, ZERO_INT>), dim3(geo.nblocks),
                     dim3(kThreads), 0, s, a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

template <typename T>
SweepK<T> make_args(const ms_grid& g, const SweepGeom& geo) {
  SweepK<T> a{};
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  a.sy = g.sy; a.sz = g.sz;
  a.tiles_x = geo.tiles_x; a.tiles_y = geo.tiles_y; a.zc = geo.zc;
  a.nblocks = geo.nblocks;
  return a;
}

}  // namespace

int launch_sweep(const ms_grid& g, int dtype, void* const bufs[3], int nbuf, const void* f,
                 double* partials, double* hist, Ctl* ctl, int64_t k_off,
                 const SweepGeom& geo, hipStream_t s) {
  if (dtype == MS_F64) {
    auto a = make_args<double>(g, geo);
    for (int q = 0; q < 3; ++q) a.buf[q] = static_cast<double*>(bufs[q]);
    a.f = static_cast<const double*>(f);
    a.partials = partials; a.hist = hist; a.ctl = ctl; a.k_off = k_off; a.nbuf = nbuf;
    return f ? launch_t<double, true, true, false>(a, geo, s)
             : launch_t<double, false, true, false>(a, geo, s);
  }
  auto a = make_args<float>(g, geo);
  for (int q = 0; q < 3; ++q) a.buf[q] = static_cast<float*>(bufs[q]);
  a.f = static_cast<const float*>(f);
  a.partials = partials; a.hist = hist; a.ctl = ctl; a.k_off = k_off; a.nbuf = nbuf;
  return f ? launch_t<float, true, true, false>(a, geo, s)
           : launch_t<float, false, true, false>(a, geo, s);
}

int launch_residual(const ms_grid& g, int dtype, const void* u, const void* f,
                    bool zero_interior, double* partials, int slot, const SweepGeom& geo,
                    hipStream_t s) {
  if (dtype == MS_F64) {
    auto a = make_args<double>(g, geo);
    a.buf[0] = const_cast<double*>(static_cast<const double*>(u));
    a.f = static_cast<const double*>(f);
    a.partials = partials; a.slot = slot; a.nbuf = 1;
    if (zero_interior)
      return f ? launch_t<double, true, false, true>(a, geo, s)
               : launch_t<double, false, false, true>(a, geo, s);
    return f ? launch_t<double, true, false, false>(a, geo, s)
             : launch_t<double, false, false, false>(a, geo, s);
  }
  auto a = make_args<float>(g, geo);
  a.buf[0] = const_cast<float*>(static_cast<const float*>(u));
  a.f = static_cast<const float*>(f);
  a.partials = partials; a.slot = slot; a.nbuf = 1;
  if (zero_interior)
    return f ? launch_t<float, true, false, true>(a, geo, s)
             : launch_t<float, false, false, true>(a, geo, s);
  return f ? launch_t<float, true, false, false>(a, geo, s)
           : launch_t<float, false, false, false>(a, geo, s);
}

int launch_finalize(const double* partials, int slot, int nblocks, double* out_norm, Ctl* ctl,
                    double* hist, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s,
                     partials + (int64_t)slot * nblocks, nblocks, out_norm, ctl, hist, k);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

}  // namespace ms
