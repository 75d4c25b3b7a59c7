// 7-point Jacobi sweeps with the fused residual-norm reduction, the
// standalone residual pass and their finalisation.
//
// Per cell (the 7-point Laplace iteration of the paper's evaluation,
// Section 4.1, as an out-of-place update, Section 2.2):
//   S  = (((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1]) + u[k-1])
//   u' = (S - f) * fl(1/6)          (S * fl(1/6) without f)
//   r  = f - (S - u*6)              (residual of the input field)
// and sum r^2 (FP64) goes to one partial per block.
//
// Two z-marching kernels compute this; both keep the z neighbours in
// registers (previous / current / next plane) and prefetch the plane after
// next while the current one is computed.
//
// * Register-tiled (the default): every wave owns a (64*V) x R tile, lane l
//   holding V consecutive x cells of R consecutive rows, so y neighbours are
//   registers and x neighbours come from the adjacent lane through DPP
//   wave shifts. The cells just outside the wave (two x-halo columns, two
//   y-halo rows) are loaded directly. No LDS and no barrier in the march;
//   V = 2 (FP64) makes each row access one 1 KiB dwordx4 wave load.
// * LDS-tiled: a block stages the current plane of a 64 x 4R tile plus its
//   ring in LDS (double-buffered, one barrier per plane).
//
// Two-stage passes (further down) apply two sweeps per pass over memory, or
// one red-black Gauss-Seidel sweep (red half, then black half), in two
// layouts: LDS-staged 64 x 8 tiles (sweep_tb2_kernel) and one column per
// lane (sweep_tbw_kernel).
#include "ms_internal.hpp"
#include "march.hpp"

// Bit-exact parity with the oracle needs every operation rounded on its own.
#pragma clang fp contract(off)

namespace ms {

namespace {

template <typename T>
struct SweepK {
  T* buf[3];
  const T* f;
  double* partials;  // [kPartialSlots][kMaxBlocks]
  double* hist;
  Ctl* ctl;
  int64_t k_off;
  int nbuf;
  int slot;  // residual-only launches: partial slot
  int nx, ny, nz;
  int64_t sy, sz;
  int tiles_x, tiles_y, zc, nblocks, wx;
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

// Work shared by every sweep launch before its tile: block 0 turns the
// partials of launch k-1 into ||r(u_{k-1})|| and judges it; then the whole
// block returns if the solve is already done. Returns false to exit.
template <typename T, bool WRITE>
__device__ __forceinline__ bool sweep_prologue(const SweepK<T>& a, int64_t k, double* red,
                                               int* s_done) {
  if (WRITE && blockIdx.x == 0 && k >= 1 && (a.hist || a.ctl)) {
    if (!a.ctl || a.ctl->done == RUNNING) {
      const double t = sum_partials(a.partials + ((k - 1) & 3) * (int64_t)kMaxBlocks,
                                    a.nblocks, red);
      if (threadIdx.x == 0) judge(a.ctl, a.hist, k - 1, sqrt(t));
    }
  }
  if (a.ctl) {
    if (threadIdx.x == 0) *s_done = a.ctl->done;
    __syncthreads();
    if (*s_done != RUNNING) return false;  // block-uniform
  }
  return true;
}

// ------------------------------------------------------- vector access

template <typename T, int V>
struct VecT;
template <>
struct VecT<double, 1> { typedef double t; };
template <>
struct VecT<double, 2> { typedef double t __attribute__((ext_vector_type(2))); };
template <>
struct VecT<float, 1> { typedef float t; };
template <>
struct VecT<float, 2> { typedef float t __attribute__((ext_vector_type(2))); };
template <>
struct VecT<float, 4> { typedef float t __attribute__((ext_vector_type(4))); };

template <typename T, int V>
__device__ __forceinline__ T vget(const typename VecT<T, V>::t& x, int v) {
  if constexpr (V == 1) return x;
  else return x[v];
}

// Loads V consecutive elements starting at p; `n` of them exist (0..V).
template <typename T, int V>
__device__ __forceinline__ void load_v(T (&d)[V], const T* __restrict__ p, int n) {
  if (n == V) {
    typedef typename VecT<T, V>::t vt;
    const vt x = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int v = 0; v < V; ++v) d[v] = vget<T, V>(x, v);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) d[v] = v < n ? p[v] : T(0);
  }
}

// Stores the first n of V values at p; nontemporal: the output is not read
// again by this sweep.
template <typename T, int V>
__device__ __forceinline__ void store_v(T* __restrict__ p, const T (&d)[V], int n) {
  if (n == V) {
    typedef typename VecT<T, V>::t vt;
    vt x;
    if constexpr (V == 1) {
      x = d[0];
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) x[v] = d[v];
    }
    __builtin_nontemporal_store(x, reinterpret_cast<vt*>(p));
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (v < n) __builtin_nontemporal_store(d[v], p + v);
  }
}

// ------------------------------------------------ register-tiled kernel

template <typename T, int V, int R, bool HAS_F>
__global__ __launch_bounds__(kThreads) void sweep_rt_kernel(SweepK<T> a) {
  __shared__ double red[kWavesY];
  __shared__ int s_done;
  const int64_t k = (a.ctl ? a.ctl->base : 0) + a.k_off;
  if (!sweep_prologue<T, true>(a, k, red, &s_done)) return;

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wx = w % a.wx, wy = w / a.wx;
  const int wy_n = kWavesY / a.wx;
  const int i0 = (txi * a.wx + wx) * (kWave * V);  // first x cell of this wave
  const int j0 = (tyi * wy_n + wy) * R;            // first row of this wave
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int xi = i0 + lane * V;  // first x cell of this lane

  const T* __restrict__ src = a.buf[k % a.nbuf];
  T* __restrict__ dst = a.buf[(k + 1) % a.nbuf];
  const T* __restrict__ f = a.f;
  const int64_t sy = a.sy, sz = a.sz;
  const int nx = a.nx, ny = a.ny;

  // Elements of this lane that exist (halo included: i <= nx) and that are
  // computed (i < nx).
  const int nload = max(0, min(V, nx + 1 - xi));
  const int nact = max(0, min(V, nx - xi));
  int rload[R + 2];  // rows j0-1 .. j0+R: elements to load
#pragma unroll
  for (int r = -1; r <= R; ++r) rload[r + 1] = (j0 + r <= ny) ? nload : 0;
  const int64_t base = (int64_t)(j0 + 1) * sy + (xi + 1);  // row j0, this lane, plane -1
  const bool left_edge = lane == 0, right_edge = lane == kWave - 1;
  const int xh_r = i0 + kWave * V;  // right x-halo column of the wave
  const bool xh_r_ok = right_edge && xh_r <= nx;

  T zp[R][V], zc[R][V], zn[R][V], fc[R][V];
  T ht[V], hb[V];  // y-halo rows j0-1 and j0+R, current plane
  T xl[R], xr[R];  // x-halo cells, current plane (lanes 0 / 63)

  auto plane = [&](int kk) { return (int64_t)(kk + 1) * sz; };
  auto ld_rows = [&](T(&d)[R][V], int kk) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      load_v<T, V>(d[r], src + plane(kk) + base + r * sy, rload[r + 1]);
  };
  auto ld_f = [&](T(&d)[R][V], int kk) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (HAS_F) {
        load_v<T, V>(d[r], f + plane(kk) + base + r * sy, (j0 + r < ny) ? nact : 0);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) d[r][v] = T(0);
      }
    }
  };
  auto ld_halo = [&](T(&t)[V], T(&b)[V], T(&l)[R], T(&rr)[R], int kk) {
    load_v<T, V>(t, src + plane(kk) + base - sy, rload[0]);
    load_v<T, V>(b, src + plane(kk) + base + R * sy, rload[R + 1]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool rowok = j0 + r <= ny;
      const int64_t row = plane(kk) + (int64_t)(j0 + r + 1) * sy;
      l[r] = (left_edge && rowok) ? src[row + i0] : T(0);       // x = i0 - 1
      rr[r] = (xh_r_ok && rowok) ? src[row + xh_r + 1] : T(0);  // x = i0 + 64V
    }
  };

  ld_rows(zp, z0 - 1);
  ld_rows(zc, z0);
  ld_rows(zn, z0 + 1);
  ld_f(fc, z0);
  ld_halo(ht, hb, xl, xr, z0);

  double acc = 0.0;
  const T c6 = C6<T>::v();
  for (int kk = z0; kk < z1; ++kk) {
    const bool more = kk + 1 < z1;
    T pf[R][V], fn[R][V], htn[V], hbn[V], xln[R], xrn[R];
    if (more) {
      ld_rows(pf, kk + 2);
      ld_f(fn, kk + 1);
      ld_halo(htn, hbn, xln, xrn, kk + 1);
    }
    // x neighbours across lanes (every lane executes the DPP moves)
    T xm0[R], xpl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xm0[r] = lane_from_left(xl[r], zc[r][V - 1]);  // left of element 0
      xpl[r] = lane_from_right(xr[r], zc[r][0]);     // right of element V-1
    }
    const int64_t pk = plane(kk);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool row_act = j0 + r < ny;
      T out[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T xm = v > 0 ? zc[r][v - 1] : xm0[r];
        const T xp = v < V - 1 ? zc[r][v + 1] : xpl[r];
        const T ym = r > 0 ? zc[r - 1][v] : ht[v];
        const T yp = r < R - 1 ? zc[r + 1][v] : hb[v];
        const T s = ((((xp + xm) + yp) + ym) + zn[r][v]) + zp[r][v];
        out[v] = HAS_F ? (s - fc[r][v]) * c6 : s * c6;
        if (row_act && v < nact) {
          const double res = cell_residual(xp, xm, yp, ym, zn[r][v], zp[r][v], zc[r][v],
                                           fc[r][v], HAS_F);
          acc += res * res;
        }
      }
      if (row_act) store_v<T, V>(dst + pk + base + r * sy, out, nact);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          zp[r][v] = zc[r][v];
          zc[r][v] = zn[r][v];
          zn[r][v] = pf[r][v];
          fc[r][v] = fn[r][v];
        }
        xl[r] = xln[r];
        xr[r] = xrn[r];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        ht[v] = htn[v];
        hb[v] = hbn[v];
      }
    }
  }

  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) a.partials[(int64_t)(k & 3) * kMaxBlocks + blockIdx.x] = tot;
}

// --------------------------------------------------- LDS-tiled kernel

// WRITE: sweep (write u' and evaluate the residual of u); else residual only.
// ZERO_INT: read the field with its interior replaced by 0 (residual of u^0).
template <typename T, int R, bool HAS_F, bool WRITE, bool ZERO_INT>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepK<T> a) {
  constexpr int kTileY = kWavesY * R;
  __shared__ T lds[2][kTileY + 2][kTileX + 2];
  __shared__ double red[kWavesY];
  __shared__ int s_done;

  const int64_t k = (a.ctl ? a.ctl->base : 0) + a.k_off;
  if (!sweep_prologue<T, WRITE>(a, k, red, &s_done)) return;

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

  const int slot = WRITE ? (int)(k & 3) : a.slot;
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
        __builtin_nontemporal_store(v, dst + (int64_t)(kk + 1) * sz + coff[r]);
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
  if (threadIdx.x == 0) a.partials[(int64_t)slot * kMaxBlocks + blockIdx.x] = tot;
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

// ------------------------------------------- two-sweep temporal blocking

// A block owns a 64 x 8 output tile and marches a z-chunk, applying two
// sweeps per pass. Stage A computes u_{k+1} on the tile plus a one-cell ring
// (66 x 10) from u_k staged in LDS with a two-cell ring (68 x 12); stage B
// computes u_{k+2} on the tile from u_{k+1} staged in LDS. Stage A runs one
// level ahead of stage B. Both stages use the single-sweep arithmetic, so
// the results are bit-identical to two plain sweeps; ring cells that are
// Dirichlet halo keep their value, as a plain sweep never writes the halo.
// Four LDS buffers per stage leave one barrier per level. Stage A adds the
// residual of u_k on the tile, stage B the residual of u_{k+1}.
//
// RB: one red-black Gauss-Seidel sweep per launch instead. Red cells are
// those with i + j + k even (interior coordinates). Stage A then updates only
// the red cells of the ring region (black ones keep u_k), which is the first
// half-sweep; stage B updates only the black cells of the tile from that
// half-swept field (red ones keep it), which is the second. All six
// neighbours of a cell have the other colour, so each half-sweep is the
// Jacobi update restricted to one colour. Launch L reads u_L and writes
// u_{L+1}; stage A adds the residual of u_L, and block 0 judges u_{L-1}.
constexpr int kTbX = 64, kTbY = 8;
constexpr int kTbAX = kTbX + 4, kTbAY = kTbY + 4;  // u_k region (68 x 12)
constexpr int kTbBX = kTbX + 2, kTbBY = kTbY + 2;  // u_{k+1} region (66 x 10)
constexpr int kTbACells = kTbAX * kTbAY;           // 816 -> 4 per thread
constexpr int kTbBCells = kTbBX * kTbBY;           // 660 -> 3 per thread
constexpr int kTbOut = kTbX * kTbY;                // 512 -> 2 per thread

template <typename T, bool HAS_F, bool RB>
__global__ __launch_bounds__(kThreads) void sweep_tb2_kernel(SweepK<T> a) {
  __shared__ T A[4][kTbAY][kTbAX];
  __shared__ T B[4][kTbBY][kTbBX];
  __shared__ double red[kWavesY];
  __shared__ int s_done;

  const int64_t L = (a.ctl ? a.ctl->base : 0) + a.k_off;
  const int64_t k0 = RB ? L : 2 * L;  // iterate read by this launch
  // Block 0 finalises the iterates of the previous launch, in order.
  if (blockIdx.x == 0 && L >= 1 && (a.hist || a.ctl)) {
#pragma unroll
    for (int d = RB ? 1 : 2; d >= 1; --d) {
      if (!a.ctl || a.ctl->done == RUNNING) {
        const double t = sum_partials(a.partials + ((k0 - d) & 3) * (int64_t)kMaxBlocks,
                                      a.nblocks, red);
        if (threadIdx.x == 0) judge(a.ctl, a.hist, k0 - d, sqrt(t));
        __syncthreads();
      }
    }
  }
  if (a.ctl) {
    if (threadIdx.x == 0) s_done = a.ctl->done;
    __syncthreads();
    if (s_done != RUNNING) return;
  }

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int i0 = txi * kTbX, j0 = tyi * kTbY;
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t sy = a.sy, sz = a.sz;
  const T* __restrict__ src = a.buf[L % a.nbuf];
  T* __restrict__ dst = a.buf[(L + 1) % a.nbuf];
  const T* __restrict__ f = a.f;
  const int t = threadIdx.x;
  auto off = [&](int i, int j, int k) {
    return (int64_t)(k + 1) * sz + (int64_t)(j + 1) * sy + (i + 1);
  };
  auto abuf = [&](int k) { return (k - z0 + 8) & 3; };

  // u_k region cells owned by this thread (LDS staging): c = t + 256 q.
  constexpr int QA = (kTbACells + kThreads - 1) / kThreads;
  auto a_cell = [&](int q, int& ra, int& ca) {
    const int c = t + q * kThreads;
    ra = c / kTbAX;
    ca = c % kTbAX;
    return c < kTbACells;
  };
  // Loads are unconditional, from coordinates clamped into the field (halo
  // included): cells outside the field feed no output and no residual, and
  // a conditional load would have to complete before its branch joins,
  // which serialises the loads.
  auto clampx = [&](int i) { return min(max(i, -1), nx); };
  auto clampy = [&](int j) { return min(max(j, -1), ny); };
  auto clampz = [&](int k) { return min(max(k, -1), nz); };
  auto load_a = [&](T (&r)[QA], int k) {
    const int kc = clampz(k);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      int ra, ca;
      (void)a_cell(q, ra, ca);
      r[q] = src[off(clampx(i0 - 2 + ca), clampy(j0 - 2 + ra), kc)];
    }
  };
  auto store_a = [&](const T (&r)[QA], int k) {
    const int b = abuf(k);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      int ra, ca;
      if (a_cell(q, ra, ca)) A[b][ra][ca] = r[q];
    }
  };

  // Prologue: levels z0-2 .. z0 into LDS, z0+1 into registers.
  {
    T r[QA];
    for (int k = z0 - 2; k <= z0; ++k) {
      if (k < -1) continue;
      load_a(r, k);
      store_a(r, k);
    }
  }
  // Two register sets of prefetched u_k levels: at step z the set of parity
  // (z - z0 + 1) holds level z+2, is stored to LDS and refilled with level
  // z+4, so two levels of loads are in flight behind the compute.
  T preA[QA], preB[QA];
  const int klast = min(z1 + 1, nz);  // last u_k level stage A needs
  load_a(preA, z0 + 1);               // z0 + 1 <= nz always
  if (z0 + 2 <= klast) load_a(preB, z0 + 2);
  __syncthreads();

  double acc_a = 0.0, acc_b = 0.0;
  const T c6 = C6<T>::v();
  constexpr int QB = (kTbBCells + kThreads - 1) / kThreads;
  constexpr int QO = kTbOut / kThreads;
  // Loop-invariant cell bookkeeping. Stage A: cells of the 66 x 10 region.
  int arb[QB], acb[QB], apar[QB];  // apar: parity of i + j
  int64_t aoff[QB];  // clamped into the field (for the f loads)
  bool aown[QB], ain[QB], atile[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int c = t + q * kThreads;
    aown[q] = c < kTbBCells;
    arb[q] = c / kTbBX;
    acb[q] = c % kTbBX;
    apar[q] = (arb[q] + acb[q]) & 1;  // i0 and j0 are even
    const int i = i0 - 1 + acb[q], j = j0 - 1 + arb[q];
    ain[q] = aown[q] && i >= 0 && i < nx && j >= 0 && j < ny;
    atile[q] = arb[q] >= 1 && arb[q] <= kTbY && acb[q] >= 1 && acb[q] <= kTbX;
    aoff[q] = (int64_t)(clampy(j) + 1) * sy + (clampx(i) + 1);
  }
  // Stage B: cells of the 64 x 8 tile.
  int brt[QO], bct[QO], bpar[QO];
  int64_t boff[QO];
  bool bin[QO];
#pragma unroll
  for (int q = 0; q < QO; ++q) {
    const int c = t + q * kThreads;
    brt[q] = c / kTbX;
    bct[q] = c % kTbX;
    bpar[q] = (brt[q] + bct[q]) & 1;
    const int i = i0 + bct[q], j = j0 + brt[q];
    bin[q] = i < nx && j < ny;
    boff[q] = (int64_t)(clampy(j) + 1) * sy + (clampx(i) + 1);  // clamped
  }
  auto zin = [&](int z) { return z >= 0 && z < nz; };
  // f for stage A at level z and for stage B at level z-1, prefetched one
  // step ahead.
  // (unconditional and clamped as above; only interior cells use them)
  auto ld_fa = [&](T (&d)[QB], int z) {
    const int64_t pz = (int64_t)(clampz(z) + 1) * sz;
#pragma unroll
    for (int q = 0; q < QB; ++q) d[q] = HAS_F ? f[pz + aoff[q]] : T(0);
  };
  auto ld_fb = [&](T (&d)[QO], int z) {
    const int64_t pz = (int64_t)(clampz(z) + 1) * sz;
#pragma unroll
    for (int q = 0; q < QO; ++q) d[q] = HAS_F ? f[pz + boff[q]] : T(0);
  };
  T fa[QB], fb[QO];
  ld_fa(fa, z0 - 1);
#pragma unroll
  for (int q = 0; q < QO; ++q) fb[q] = T(0);

  auto step = [&](int z, T (&pre)[QA]) {
    // 1. publish level z+2 of u_k (read from step z+1 on), prefetch z+4
    if (z + 2 <= klast) {
      store_a(pre, z + 2);
      if (z + 4 <= klast) load_a(pre, z + 4);
    }
    T fa_n[QB], fb_n[QO];
    ld_fa(fa_n, z + 1);
    ld_fb(fb_n, z);
    // 2. stage A at level z: u_{k+1} on the 66 x 10 region
    {
      const int bm = abuf(z - 1), bc = abuf(z), bp = abuf(z + 1);
      const bool zz = zin(z);
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        if (!aown[q]) continue;
        const int ra = arb[q] + 1, ca = acb[q] + 1;
        const T uc = A[bc][ra][ca];
        T v = uc;  // halo cells keep their Dirichlet value
        if (ain[q] && zz) {
          const T xp = A[bc][ra][ca + 1], xm = A[bc][ra][ca - 1];
          const T yp = A[bc][ra + 1][ca], ym = A[bc][ra - 1][ca];
          const T zp = A[bp][ra][ca], zm = A[bm][ra][ca];
          const T s = ((((xp + xm) + yp) + ym) + zp) + zm;
          if (!RB || ((apar[q] + z) & 1) == 0) v = HAS_F ? (s - fa[q]) * c6 : s * c6;
          if (atile[q] && z >= z0 && z < z1) {
            const double res = cell_residual(xp, xm, yp, ym, zp, zm, uc, fa[q], HAS_F);
            acc_a += res * res;
          }
        }
        B[bc][arb[q]][acb[q]] = v;
      }
    }
    __syncthreads();
    // 3. stage B at level z-1: u_{k+2} on the tile
    const int zb = z - 1;
    if (zb >= z0 && zb < z1) {
      const int bm = abuf(zb - 1), bc = abuf(zb), bp = abuf(zb + 1);
#pragma unroll
      for (int q = 0; q < QO; ++q) {
        if (!bin[q]) continue;
        const int rb = brt[q] + 1, cb = bct[q] + 1;
        const T uc = B[bc][rb][cb];
        const T xp = B[bc][rb][cb + 1], xm = B[bc][rb][cb - 1];
        const T yp = B[bc][rb + 1][cb], ym = B[bc][rb - 1][cb];
        const T zp = B[bp][rb][cb], zm = B[bm][rb][cb];
        const T s = ((((xp + xm) + yp) + ym) + zp) + zm;
        const bool upd = !RB || ((bpar[q] + zb) & 1) == 1;
        const T v = upd ? (HAS_F ? (s - fb[q]) * c6 : s * c6) : uc;
        __builtin_nontemporal_store(v, dst + (int64_t)(zb + 1) * sz + boff[q]);
        if (!RB) {
          const double res = cell_residual(xp, xm, yp, ym, zp, zm, uc, fb[q], HAS_F);
          acc_b += res * res;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) fa[q] = fa_n[q];
#pragma unroll
    for (int q = 0; q < QO; ++q) fb[q] = fb_n[q];
  };
  for (int z = z0 - 1; z <= z1; z += 2) {
    step(z, preA);
    if (z + 1 <= z1) step(z + 1, preB);
  }

  const double ta = block_sum(acc_a, red);
  const double tb = RB ? 0.0 : block_sum(acc_b, red);
  if (threadIdx.x == 0) {
    a.partials[(int64_t)(k0 & 3) * kMaxBlocks + blockIdx.x] = ta;
    if (!RB) a.partials[(int64_t)((k0 + 1) & 3) * kMaxBlocks + blockIdx.x] = tb;
  }
}

// ------------------------------- two-stage pass, one column per lane

// The same two stages (two Jacobi sweeps, or one red-black Gauss-Seidel
// sweep) with the work laid out so that almost every neighbour is a
// register. A block of kTwWaves waves covers a staging region of 64 columns
// (one per lane) x kTwWaves * kTwRows rows; a lane keeps its column's rows in
// registers across three z levels. x neighbours come from the adjacent lane
// (DPP moves), y neighbours from the thread's own rows, z neighbours from
// its level queue; only the rows just above and below a wave's group cross
// waves, through LDS (two rows per wave and level, one barrier per level).
// Stage A (u_k -> h) covers columns 1..62 and rows 1..R-2 of the region,
// stage B (h -> output) columns 2..61 and rows 2..R-3 (the 60-wide output
// tile), one level behind stage A. f is loaded once per cell and kept for
// stage B. The per-cell arithmetic is the single sweep's, so the results
// are bit-identical to the other kernels.
// Blocks of 8 waves: region 64 x 24, output tile 60 x 20. (16-wave blocks,
// 60 x 44 output tiles with fewer re-read halo rows, measured 3-9% slower:
// the per-level barrier then waits on twice as many waves.)
constexpr int kTwWaves = 8, kTwRows = 3;  // 121 VGPRs (FP64): four waves per SIMD
constexpr int kTwThreads = 64 * kTwWaves;
constexpr int kTwRegionY = kTwWaves * kTwRows;  // 24 rows
constexpr int kTwTileX = 60, kTwTileY = kTwRegionY - 4;

template <typename T, bool HAS_F, bool RB>
__global__ __launch_bounds__(kTwThreads) __attribute__((amdgpu_waves_per_eu(4))) void sweep_tbw_kernel(SweepK<T> a) {
  __shared__ T xu[2][kTwWaves][2][64];  // u_k rows 0 and R-1 of every wave group
  __shared__ T xh[2][kTwWaves][2][64];  // h rows 0 and R-1
  __shared__ double red[kTwWaves];
  __shared__ int s_done;

  const int64_t L = (a.ctl ? a.ctl->base : 0) + a.k_off;
  const int64_t k0 = RB ? L : 2 * L;  // iterate read by this launch
  if (blockIdx.x == 0 && L >= 1 && (a.hist || a.ctl)) {
#pragma unroll
    for (int d = RB ? 1 : 2; d >= 1; --d) {
      if (!a.ctl || a.ctl->done == RUNNING) {
        const double t = sum_partials(a.partials + ((k0 - d) & 3) * (int64_t)kMaxBlocks,
                                      a.nblocks, red);
        if (threadIdx.x == 0) judge(a.ctl, a.hist, k0 - d, sqrt(t));
        __syncthreads();
      }
    }
  }
  if (a.ctl) {
    if (threadIdx.x == 0) s_done = a.ctl->done;
    __syncthreads();
    if (s_done != RUNNING) return;
  }

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  const int64_t sy = a.sy, sz = a.sz;
  const T* __restrict__ src = a.buf[L % a.nbuf];
  T* __restrict__ dst = a.buf[(L + 1) % a.nbuf];
  const T* __restrict__ f = a.f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = txi * kTwTileX - 2 + lane;            // this lane's column
  const int jr0 = tyi * kTwTileY - 2 + w * kTwRows;   // its first row
  const int wup = min(w + 1, kTwWaves - 1), wdn = max(w - 1, 0);
  const int ic = min(max(i, -1), nx);
  const bool colA = lane >= 1 && lane <= 62, colB = lane >= 2 && lane <= 61;
  const bool xin = i >= 0 && i < nx;
  int64_t off[kTwRows];
  bool inA[kTwRows], outB[kTwRows];
#pragma unroll
  for (int s = 0; s < kTwRows; ++s) {
    const int j = jr0 + s, row = w * kTwRows + s;
    off[s] = (int64_t)(min(max(j, -1), ny) + 1) * sy + (ic + 1);
    const bool yin = j >= 0 && j < ny;
    inA[s] = colA && row >= 1 && row <= kTwRegionY - 2 && xin && yin;
    outB[s] = colB && row >= 2 && row <= kTwRegionY - 3 && xin && yin;
  }
  auto plane = [&](int z) { return (int64_t)(min(max(z, -1), nz) + 1) * sz; };
  auto load_u = [&](T (&r)[kTwRows], int z) {
    const int64_t p = plane(z);
#pragma unroll
    for (int s = 0; s < kTwRows; ++s) r[s] = src[p + off[s]];
  };
  auto load_f = [&](T (&r)[kTwRows], int z) {
    const int64_t p = plane(z);
#pragma unroll
    for (int s = 0; s < kTwRows; ++s) r[s] = HAS_F ? f[p + off[s]] : T(0);
  };
  // colour parity of (i + j) for row 0 (RB): red cells have i + j + z even
  const int par0 = (i + jr0) & 1;

  T um[kTwRows], uc[kTwRows], up[kTwRows];  // u_k at z-1, z, z+1
  T hm2[kTwRows], hm1[kTwRows];             // h at z-2, z-1
  T fa[kTwRows], fb[kTwRows];               // f at z (stage A), z-1 (stage B)
  T pu0[kTwRows], pu1[kTwRows], pf0[kTwRows], pf1[kTwRows];
  load_u(um, z0 - 2);
  load_u(uc, z0 - 1);
  load_u(up, z0);
  load_u(pu0, z0 + 1);
  load_u(pu1, z0 + 2);
  load_f(fa, z0 - 1);
  load_f(pf0, z0);
  load_f(pf1, z0 + 1);
#pragma unroll
  for (int s = 0; s < kTwRows; ++s) {
    hm2[s] = T(0);
    hm1[s] = T(0);
    fb[s] = T(0);
  }

  double acc_a = 0.0, acc_b = 0.0;
  const T c6 = C6<T>::v();
  // One level: stage A at z (u_k -> h(z)), stage B at z - 1 (h -> output).
  // pu / pf hold u_k(z+2) / f(z+1) on entry and take u_k(z+4) / f(z+3).
  auto step = [&](int z, int b, T (&pu)[kTwRows], T (&pf)[kTwRows]) {
    // publish the group's edge rows of u_k(z) and h(z-1)
    xu[b][w][0][lane] = uc[0];
    xu[b][w][1][lane] = uc[kTwRows - 1];
    xh[b][w][0][lane] = hm1[0];
    xh[b][w][1][lane] = hm1[kTwRows - 1];
    __syncthreads();
    const bool zA = z >= 0 && z < nz, zres = z >= z0 && z < z1;
    T hn[kTwRows];
#pragma unroll
    for (int s = 0; s < kTwRows; ++s) {
      const T xp = lane_from_right(uc[s], uc[s]), xm = lane_from_left(uc[s], uc[s]);
      const T yp = s < kTwRows - 1 ? uc[s + 1] : xu[b][wup][0][lane];
      const T ym = s > 0 ? uc[s - 1] : xu[b][wdn][1][lane];
      const T sum = ((((xp + xm) + yp) + ym) + up[s]) + um[s];
      const bool upd = !RB || ((par0 + s + z) & 1) == 0;
      hn[s] = inA[s] && zA && upd ? (HAS_F ? (sum - fa[s]) * c6 : sum * c6) : uc[s];
      if (outB[s] && zres) {
        const double r = cell_residual(xp, xm, yp, ym, up[s], um[s], uc[s], fa[s], HAS_F);
        acc_a += r * r;
      }
    }
    const int zb = z - 1;
    if (zb >= z0 && zb < z1) {
      const int64_t pb = (int64_t)(zb + 1) * sz;
#pragma unroll
      for (int s = 0; s < kTwRows; ++s) {
        const T xp = lane_from_right(hm1[s], hm1[s]), xm = lane_from_left(hm1[s], hm1[s]);
        const T yp = s < kTwRows - 1 ? hm1[s + 1] : xh[b][wup][0][lane];
        const T ym = s > 0 ? hm1[s - 1] : xh[b][wdn][1][lane];
        const T sum = ((((xp + xm) + yp) + ym) + hn[s]) + hm2[s];
        const bool upd = !RB || ((par0 + s + zb) & 1) == 1;
        const T v = upd ? (HAS_F ? (sum - fb[s]) * c6 : sum * c6) : hm1[s];
        if (outB[s]) {
          __builtin_nontemporal_store(v, dst + pb + off[s]);
          if (!RB) {
            const double r = cell_residual(xp, xm, yp, ym, hn[s], hm2[s], hm1[s], fb[s], HAS_F);
            acc_b += r * r;
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kTwRows; ++s) {
      um[s] = uc[s];
      uc[s] = up[s];
      up[s] = pu[s];
      hm2[s] = hm1[s];
      hm1[s] = hn[s];
      fb[s] = fa[s];
      fa[s] = pf[s];
    }
    load_u(pu, z + 4);
    load_f(pf, z + 3);
  };
  for (int z = z0 - 1; z <= z1; z += 2) {
    step(z, 0, pu0, pf0);
    if (z + 1 > z1) break;
    step(z + 1, 1, pu1, pf1);
  }

  const double ta = block_sum(acc_a, red);
  const double tb = RB ? 0.0 : block_sum(acc_b, red);
  if (threadIdx.x == 0) {
    a.partials[(int64_t)(k0 & 3) * kMaxBlocks + blockIdx.x] = ta;
    if (!RB) a.partials[(int64_t)((k0 + 1) & 3) * kMaxBlocks + blockIdx.x] = tb;
  }
}

// ------------------------- two-stage pass, one column per lane, no LDS

// Two Jacobi sweeps per pass with every value in registers and no barrier
// inside the march: each wave works alone. A wave owns 64 columns (one per
// lane; its output tile is the middle 60) and kTrRows output rows, and
// keeps the rows j0-2 .. j0+kTrRows+1 of u_k of its column, three z levels
// deep, in registers. x neighbours come from the adjacent lanes (DPP), y
// neighbours from the lane's own rows, z neighbours from its level queue.
// Stage A computes h = u_{k+1} on rows j0-1 .. j0+kTrRows (lanes 1..62) at
// level z; stage B computes u_{k+2} on the output rows (lanes 2..61) at
// level z-1 from h at z-2, z-1, z. Blocks hold four waves stacked in y
// (they share the L2 lines of their halo rows). The per-cell arithmetic is
// the single sweep's, so the results are bit-identical to it; ring cells
// that are Dirichlet halo keep their value.
constexpr int kTrRows = 4;
constexpr int kTrWaves = 4;
constexpr int kTrTileX = 60;
constexpr int kTrTileY = kTrRows * kTrWaves;

template <typename T, bool HAS_F>
__global__ __launch_bounds__(64 * kTrWaves) void sweep_tbr_kernel(SweepK<T> a) {
  __shared__ double red[kTrWaves];
  __shared__ int s_done;

  const int64_t L = (a.ctl ? a.ctl->base : 0) + a.k_off;
  const int64_t k0 = 2 * L;  // iterate read by this launch
  if (blockIdx.x == 0 && L >= 1 && (a.hist || a.ctl)) {
#pragma unroll
    for (int d = 2; d >= 1; --d) {
      if (!a.ctl || a.ctl->done == RUNNING) {
        const double t = sum_partials(a.partials + ((k0 - d) & 3) * (int64_t)kMaxBlocks,
                                      a.nblocks, red);
        if (threadIdx.x == 0) judge(a.ctl, a.hist, k0 - d, sqrt(t));
        __syncthreads();
      }
    }
  }
  if (a.ctl) {
    if (threadIdx.x == 0) s_done = a.ctl->done;
    __syncthreads();
    if (s_done != RUNNING) return;
  }

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = tyi * kTrTileY + w * kTrRows;  // first output row of this wave
  double acc_a = 0.0, acc_b = 0.0;
  two_sweep_march<T, HAS_F, kTrRows>(a.buf[L % a.nbuf], a.buf[(L + 1) % a.nbuf], a.f, a.nx,
                                     a.ny, a.nz, a.sy, a.sz, txi * kTrTileX - 2 + lane, j0, z0,
                                     z1, C6<T>::v(), acc_a, acc_b);

  const double ta = block_sum(acc_a, red);
  const double tb = block_sum(acc_b, red);
  if (threadIdx.x == 0) {
    a.partials[(int64_t)(k0 & 3) * kMaxBlocks + blockIdx.x] = ta;
    a.partials[(int64_t)((k0 + 1) & 3) * kMaxBlocks + blockIdx.x] = tb;
  }
}

template <typename T, bool HAS_F, bool WRITE, bool ZERO_INT>
int launch_lds(const SweepK<T>& a, const SweepGeom& geo, hipStream_t s) {
  const dim3 grid(geo.nblocks), block(kThreads);
  if (geo.rows == 8)
    hipLaunchKernelGGL((sweep_kernel<T, 8, HAS_F, WRITE, ZERO_INT>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((sweep_kernel<T, 4, HAS_F, WRITE, ZERO_INT>), grid, block, 0, s, a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

template <typename T, int V, bool HAS_F>
void launch_rt_v(const SweepK<T>& a, const SweepGeom& geo, hipStream_t s) {
  const dim3 grid(geo.nblocks), block(kThreads);
  switch (geo.rows) {
    case 2:
      hipLaunchKernelGGL((sweep_rt_kernel<T, V, 2, HAS_F>), grid, block, 0, s, a);
      break;
    case 8:
      hipLaunchKernelGGL((sweep_rt_kernel<T, V, 8, HAS_F>), grid, block, 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((sweep_rt_kernel<T, V, 4, HAS_F>), grid, block, 0, s, a);
      break;
  }
}

template <typename T, bool HAS_F>
int launch_rt(const SweepK<T>& a, const SweepGeom& geo, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (geo.vec == 2) launch_rt_v<T, 2, HAS_F>(a, geo, s);
    else launch_rt_v<T, 1, HAS_F>(a, geo, s);
  } else {
    if (geo.vec == 4) launch_rt_v<T, 4, HAS_F>(a, geo, s);
    else if (geo.vec == 2) launch_rt_v<T, 2, HAS_F>(a, geo, s);
    else launch_rt_v<T, 1, HAS_F>(a, geo, s);
  }
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
  a.wx = geo.wx;
  return a;
}

template <typename T>
int sweep_typed(const ms_grid& g, void* const bufs[3], int nbuf, const void* f,
                double* partials, double* hist, Ctl* ctl, int64_t k_off, const SweepGeom& geo,
                hipStream_t s) {
  auto a = make_args<T>(g, geo);
  for (int q = 0; q < 3; ++q) a.buf[q] = static_cast<T*>(bufs[q]);
  a.f = static_cast<const T*>(f);
  a.partials = partials; a.hist = hist; a.ctl = ctl; a.k_off = k_off; a.nbuf = nbuf;
  if (geo.variant == kVariantRegister)
    return f ? launch_rt<T, true>(a, geo, s) : launch_rt<T, false>(a, geo, s);
  return f ? launch_lds<T, true, true, false>(a, geo, s)
           : launch_lds<T, false, true, false>(a, geo, s);
}

template <typename T>
int residual_typed(const ms_grid& g, const void* u, const void* f, bool zero_interior,
                   double* partials, int slot, const SweepGeom& geo, hipStream_t s) {
  auto a = make_args<T>(g, geo);
  a.buf[0] = const_cast<T*>(static_cast<const T*>(u));
  a.f = static_cast<const T*>(f);
  a.partials = partials; a.slot = slot; a.nbuf = 1;
  if (zero_interior)
    return f ? launch_lds<T, true, false, true>(a, geo, s)
             : launch_lds<T, false, false, true>(a, geo, s);
  return f ? launch_lds<T, true, false, false>(a, geo, s)
           : launch_lds<T, false, false, false>(a, geo, s);
}

}  // namespace

int launch_sweep(const ms_grid& g, int dtype, void* const bufs[3], int nbuf, const void* f,
                 double* partials, double* hist, Ctl* ctl, int64_t k_off,
                 const SweepGeom& geo, hipStream_t s) {
  if (geo.nblocks > kMaxBlocks || geo.nblocks < 1)
    return set_error(MS_EUNSUPPORTED, "sweep geometry with %d blocks", geo.nblocks);
  if (dtype == MS_F64)
    return sweep_typed<double>(g, bufs, nbuf, f, partials, hist, ctl, k_off, geo, s);
  return sweep_typed<float>(g, bufs, nbuf, f, partials, hist, ctl, k_off, geo, s);
}

int launch_residual(const ms_grid& g, int dtype, const void* u, const void* f,
                    bool zero_interior, double* partials, int slot, hipStream_t s) {
  // The standalone residual always runs the LDS-tiled kernel, 4 rows/thread.
  const SweepGeom geo = sweep_geom_lds(g);
  if (geo.nblocks > kMaxBlocks)
    return set_error(MS_EUNSUPPORTED, "residual geometry with %d blocks", geo.nblocks);
  if (dtype == MS_F64)
    return residual_typed<double>(g, u, f, zero_interior, partials, slot, geo, s);
  return residual_typed<float>(g, u, f, zero_interior, partials, slot, geo, s);
}

int residual_blocks(const ms_grid& g) { return sweep_geom_lds(g).nblocks; }

// Variants of the two-stage pass: kTbLds (LDS-staged 64 x 8 tiles),
// kTbColumns (one column per lane) and kTbRegisters (one wave per tile, no
// barrier). Measured kernel times per pass, FP64: 512^3 columns 776 us,
// LDS 825, registers 810 (red-black: columns 772, LDS 827); 256^3 columns
// 106.5, LDS 118.7, registers 117.3; 128^3 LDS 15% faster than columns
// (less padding: 64 x 8 tiles against 60 x 20). FP32: 128^3 registers 16.5
// against 18.3 with columns (a pass is short and latency-bound), 256^3 76.0
// against 80.2, 512^3 even.
// Default: FP64 LDS tiles up to 2^22 cells and columns above; FP32 the
// register march up to 2^25 cells and columns above (red-black sweeps have
// no register form and take columns for FP32, the FP64 rule otherwise);
// MS_TB_VARIANT=0, 2 or 3 forces one.
constexpr int kTbLds = 0, kTbColumns = 2, kTbRegisters = 3;

SweepGeom tb2_geom(const ms_grid& g, int dtype, bool rb) {
  SweepGeom s{};
  const char* ev_var = getenv("MS_TB_VARIANT");
  const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
  const int def = dtype == MS_F64 ? (cells <= ((int64_t)1 << 22) ? kTbLds : kTbColumns)
                                  : (cells <= ((int64_t)1 << 25) && !rb ? kTbRegisters : kTbColumns);
  s.variant = ev_var ? (atoi(ev_var) == 0 ? kTbLds : atoi(ev_var) == 3 ? kTbRegisters : kTbColumns)
                     : def;
  if (rb && s.variant == kTbRegisters) s.variant = kTbLds;  // Jacobi only
  // the register march indexes within a z plane with 32-bit offsets
  if (s.variant == kTbRegisters && g.sz >= INT32_MAX)
    s.variant = kTbLds;
  s.vec = 1;
  s.wx = 1;
  s.rows = 2;
  const bool cols = s.variant == kTbColumns, regs = s.variant == kTbRegisters;
  s.tiles_x = regs   ? (g.nx + kTrTileX - 1) / kTrTileX
              : cols ? (g.nx + kTwTileX - 1) / kTwTileX
                     : (g.nx + kTbX - 1) / kTbX;
  s.tiles_y = regs   ? (g.ny + kTrTileY - 1) / kTrTileY
              : cols ? (g.ny + kTwTileY - 1) / kTwTileY
                     : (g.ny + kTbY - 1) / kTbY;
  const int64_t tiles2d = (int64_t)s.tiles_x * s.tiles_y;
  // Block targets measured at 512^3. LDS tiles: 2048 (FP64) / 1024 (FP32)
  // blocks of 256 threads, three or four resident per CU. Columns: 4096
  // blocks of 512 threads (two resident per CU; 256 to 4096 were within 3%
  // for FP64, 4096 best for FP32). Marches of at least 8 levels.
  // MS_TB_BLOCKS overrides the target for tuning.
  const char* ev = getenv("MS_TB_BLOCKS");
  const int64_t want = ev && atoi(ev) > 0 ? atoi(ev)
                       : cols              ? 4096
                                           : (dtype == MS_F64 ? 2048 : 1024);
  int64_t chunks = (want + tiles2d - 1) / tiles2d;
  int zc = (int)((g.nz + chunks - 1) / chunks);
  if (zc < 8) zc = 8;
  if (zc > g.nz) zc = g.nz;
  while (tiles2d * ((g.nz + zc - 1) / zc) > kMaxBlocks && zc < g.nz) zc *= 2;
  if (zc > g.nz) zc = g.nz;
  s.zc = zc;
  s.chunks_z = (g.nz + zc - 1) / zc;
  const int64_t nb = tiles2d * s.chunks_z;
  s.nblocks = nb > kMaxBlocks ? kMaxBlocks + 1 : (int)nb;
  return s;
}

int tb2_blocks(const ms_grid& g, int dtype, bool rb) { return tb2_geom(g, dtype, rb).nblocks; }

namespace {

template <typename T, bool RB>
void launch_tb2_typed(const ms_grid& g, const SweepGeom& geo, void* const bufs[3], int nbuf,
                      const void* f, double* partials, double* hist, Ctl* ctl, int64_t k_off,
                      hipStream_t s) {
  auto a = make_args<T>(g, geo);
  for (int q = 0; q < 3; ++q) a.buf[q] = static_cast<T*>(bufs[q]);
  a.f = static_cast<const T*>(f);
  a.partials = partials; a.hist = hist; a.ctl = ctl; a.k_off = k_off; a.nbuf = nbuf;
  const dim3 grid(geo.nblocks);
  if (geo.variant == kTbRegisters && !RB) {
    if (f) hipLaunchKernelGGL((sweep_tbr_kernel<T, true>), grid, dim3(64 * kTrWaves), 0, s, a);
    else hipLaunchKernelGGL((sweep_tbr_kernel<T, false>), grid, dim3(64 * kTrWaves), 0, s, a);
  } else if (geo.variant == kTbColumns) {
    if (f) hipLaunchKernelGGL((sweep_tbw_kernel<T, true, RB>), grid, dim3(kTwThreads), 0, s, a);
    else hipLaunchKernelGGL((sweep_tbw_kernel<T, false, RB>), grid, dim3(kTwThreads), 0, s, a);
  } else {
    if (f) hipLaunchKernelGGL((sweep_tb2_kernel<T, true, RB>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((sweep_tb2_kernel<T, false, RB>), grid, dim3(kThreads), 0, s, a);
  }
}

template <bool RB>
int launch_tb2_any(const ms_grid& g, int dtype, void* const bufs[3], int nbuf, const void* f,
                   double* partials, double* hist, Ctl* ctl, int64_t k_off, hipStream_t s) {
  const SweepGeom geo = tb2_geom(g, dtype, RB);
  if (geo.nblocks > kMaxBlocks || geo.nblocks < 1)
    return set_error(MS_EUNSUPPORTED, "two-stage sweep geometry with %d blocks", geo.nblocks);
  if (dtype == MS_F64)
    launch_tb2_typed<double, RB>(g, geo, bufs, nbuf, f, partials, hist, ctl, k_off, s);
  else
    launch_tb2_typed<float, RB>(g, geo, bufs, nbuf, f, partials, hist, ctl, k_off, s);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

}  // namespace

int launch_sweep_tb2(const ms_grid& g, int dtype, void* const bufs[3], int nbuf,
                     const void* f, double* partials, double* hist, Ctl* ctl, int64_t k_off,
                     hipStream_t s) {
  return launch_tb2_any<false>(g, dtype, bufs, nbuf, f, partials, hist, ctl, k_off, s);
}

int launch_rbgs(const ms_grid& g, int dtype, void* const bufs[3], int nbuf, const void* f,
                double* partials, double* hist, Ctl* ctl, int64_t k_off, hipStream_t s) {
  return launch_tb2_any<true>(g, dtype, bufs, nbuf, f, partials, hist, ctl, k_off, s);
}

int launch_finalize(const double* partials, int slot, int nblocks, double* out_norm, Ctl* ctl,
                    double* hist, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s,
                     partials + (int64_t)slot * kMaxBlocks, nblocks, out_norm, ctl, hist, k);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

}  // namespace ms
