// Fused three-field advection source term (the Piacsek-Williams benchmark of
// the paper's evaluation, Section 4.1: three stencils over u, v, w fused
// into one region, 63 flops per cell).
//
// Staggered C-grid: u sits at (i+1/2, j, k), v at (i, j+1/2, k), w at
// (i, j, k+1/2). For phi in (u, v, w):
//   s_phi = (tcx*(Px- - Px+) + tcy*(Py- - Py+)) + (tzc1[k]*Pz- - tzc2[k]*Pz+)
// where P on each side is phi at the neighbour on that side times the sum of
// the two samples of the advecting velocity that straddle that face.
//
// Staged kernel (default): a block of eight waves owns a 64 x 8 (x, y) tile,
// one row per thread (four-wave blocks with 64 x 4 tiles, or 64 x 8 with two
// rows per thread, are the alternatives), and marches a z-chunk. Planes of u, v, w (tile plus a one-cell ring, corners included)
// pass through a ring of four LDS buffers: at level k the block reads level
// k (all in-plane neighbours) and level k+1 (the four off-column values the
// upper face needs), writes level k+2 that it loaded into registers two
// steps earlier, and issues the global loads of level k+4, so two levels of
// loads are in flight behind the compute. Four buffers leave one barrier
// per level. The level-(k-1) values (five per cell) are
// carried in registers from the previous level. Every input element is read
// from HBM once per z-chunk plus the ring; outputs are nontemporal stores.
//
// Direct kernel (cross-check): one thread per column, all neighbours read
// from global memory through the caches.
#include "ms_internal.hpp"

#pragma clang fp contract(off)

namespace ms {
namespace {

struct AdvK {
  const double* u;
  const double* v;
  const double* w;
  const double* t1;
  const double* t2;
  double* su;
  double* sv;
  double* sw;
  double tcx, tcy;
  int nx, ny, nz, zc;
  int64_t sy, sz;
  int tiles_x, tiles_y, nblocks;
};

// s_phi from its six face products, in the order of the definition.
__device__ __forceinline__ double combine(double tcx, double tcy, double c1, double c2,
                                          double pxm, double pxp, double pym, double pyp,
                                          double pzm, double pzp) {
  return (tcx * (pxm - pxp) + tcy * (pym - pyp)) + (c1 * pzm - c2 * pzp);
}

// ------------------------------------------------------------ staged kernel

constexpr int kAdvTX = 64;
constexpr int kAdvLX = kAdvTX + 2;  // 66

// kAdvRows rows per thread: tile 64 x 4*kAdvRows, LDS 4 x 3 x (tile + ring).
// GUARD: centre loads predicated on the cell lying inside the field (the
// earlier form, kept as a cross-check); otherwise they are unconditional
// loads of clamped addresses.
// W waves per block, stacked in y: the tile is 64 x (W * kAdvRows).
template <int kAdvRows, bool GUARD, int W>
__global__ __launch_bounds__(64 * W) void advect_staged_kernel(AdvK a) {
  constexpr int kAdvTY = W * kAdvRows;
  constexpr int kAdvLY = kAdvTY + 2;
  constexpr int kAdvRing = 2 * kAdvLX + 2 * kAdvTY;  // ring cells per field
  static_assert(kAdvRing <= 64 * W, "one ring cell per thread");
  // Up to eight waves the staging buffers are static LDS (at most 63 KB);
  // sixteen-wave blocks take theirs (114 KB) from dynamic LDS.
  constexpr int kStatic = W <= 8 ? 4 * 3 * kAdvLY * kAdvLX : 1;
  __shared__ double l_static[kStatic];
  extern __shared__ double l_dynamic[];
  typedef double Plane[3][kAdvLY][kAdvLX];
  Plane* L = reinterpret_cast<Plane*>(W <= 8 ? l_static : l_dynamic);

  const int tile = xcd_tile(blockIdx.x, a.nblocks);
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int tzi = rest / a.tiles_y;
  const int i0 = txi * kAdvTX, j0 = tyi * kAdvTY;
  const int z0 = tzi * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
  const int nx = a.nx, ny = a.ny;
  const int64_t sy = a.sy, sz = a.sz;
  const double* __restrict__ fld[3] = {a.u, a.v, a.w};
  double* __restrict__ out[3] = {a.su, a.sv, a.sw};

  // Centre cells of this thread: column i, rows j0 + wy*R + r.
  // Centre loads are unconditional: a cell outside the field (i > nx or
  // j > ny, which only inactive cells read) loads its clamped neighbour
  // instead, so no load waits behind an execution-mask branch. Ring loads
  // stay predicated on ring ownership, which is wave-uniform for most waves
  // (the last wave owns no ring cell and issues no ring load).
  const int i = i0 + lane;
  int64_t coff[kAdvRows], aoff[kAdvRows];
  bool cld[kAdvRows], cact[kAdvRows];
#pragma unroll
  for (int r = 0; r < kAdvRows; ++r) {
    const int j = j0 + wy * kAdvRows + r;
    coff[r] = (int64_t)(min(j, ny) + 1) * sy + (min(i, nx) + 1);
    aoff[r] = (int64_t)(min(j, ny - 1) + 1) * sy + (min(i, nx - 1) + 1);
    cld[r] = i <= nx && j <= ny;
    cact[r] = i < nx && j < ny;
  }
  // Ring cell of this thread (threads 0..147): rows 0 and LY-1 in full, then
  // columns 0 and LX-1 of the rows in between.
  int rrow = 0, rcol = 0;
  bool rown = false;
  {
    const int t = threadIdx.x;
    if (t < kAdvLX) {
      rrow = 0; rcol = t; rown = true;
    } else if (t < 2 * kAdvLX) {
      rrow = kAdvLY - 1; rcol = t - kAdvLX; rown = true;
    } else if (t < 2 * kAdvLX + kAdvTY) {
      rrow = t - 2 * kAdvLX + 1; rcol = 0; rown = true;
    } else if (t < kAdvRing) {
      rrow = t - 2 * kAdvLX - kAdvTY + 1; rcol = kAdvLX - 1; rown = true;
    }
  }
  const int ri = rown ? min(i0 - 1 + rcol, nx) : -1;
  const int rj = rown ? min(j0 - 1 + rrow, ny) : -1;
  const int64_t roff = (int64_t)(rj + 1) * sy + (ri + 1);

  auto plane = [&](int k) { return (int64_t)(k + 1) * sz; };
  // registers of one staged level: centre rows and the ring cell, per field
  auto load_level = [&](double (&c)[3][kAdvRows], double (&rg)[3], int k) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
      for (int r = 0; r < kAdvRows; ++r)
        c[q][r] = (!GUARD || cld[r]) ? fld[q][plane(k) + coff[r]] : 0.0;
      rg[q] = rown ? fld[q][plane(k) + roff] : 0.0;
    }
  };
  auto store_level = [&](const double (&c)[3][kAdvRows], const double (&rg)[3], int b) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
      for (int r = 0; r < kAdvRows; ++r) L[b][q][wy * kAdvRows + r + 1][lane + 1] = c[q][r];
      if (rown) L[b][q][rrow][rcol] = rg[q];
    }
  };

  // Level z0-1 values each cell needs: u, v, w at the cell, w at (i+1, j)
  // and at (i, j+1).
  double um1[kAdvRows], vm1[kAdvRows], wm1[kAdvRows], wm1x[kAdvRows], wm1y[kAdvRows];
#pragma unroll
  for (int r = 0; r < kAdvRows; ++r) {
    const int64_t p = plane(z0 - 1) + aoff[r];
    const bool ld = !GUARD || cact[r];
    um1[r] = ld ? a.u[p] : 0.0;
    vm1[r] = ld ? a.v[p] : 0.0;
    wm1[r] = ld ? a.w[p] : 0.0;
    wm1x[r] = ld ? a.w[p + 1] : 0.0;
    wm1y[r] = ld ? a.w[p + sy] : 0.0;
  }
  {
    double c[3][kAdvRows], rg[3];
    load_level(c, rg, z0);
    store_level(c, rg, 0);
    load_level(c, rg, z0 + 1);
    store_level(c, rg, 1);
  }
  // Two register sets of prefetched levels: at step k the set of parity
  // (k - z0) holds level k+2 (stored to LDS at step k, then refilled with
  // level k+4); the other set's level k+3 is in flight meanwhile.
  double pa[3][kAdvRows], pra[3], pb[3][kAdvRows], prb[3];
  if (z0 + 2 <= z1) load_level(pa, pra, z0 + 2);
  if (z0 + 3 <= z1) load_level(pb, prb, z0 + 3);

  const double tcx = a.tcx, tcy = a.tcy;
  auto step = [&](int k, double (&pc)[3][kAdvRows], double (&prg)[3]) {
    const int b = (k - z0) & 3, nb = (b + 1) & 3, wb = (b + 2) & 3;
    if (k + 2 <= z1) store_level(pc, prg, wb);
    if (k + 4 <= z1) load_level(pc, prg, k + 4);
    __syncthreads();
    const double c1 = a.t1[k], c2 = a.t2[k];
#pragma unroll
    for (int r = 0; r < kAdvRows; ++r) {
      const int y = wy * kAdvRows + r + 1, x = lane + 1;
      auto Lu = [&](int dy, int dx) { return L[b][0][y + dy][x + dx]; };
      auto Lv = [&](int dy, int dx) { return L[b][1][y + dy][x + dx]; };
      auto Lw = [&](int dy, int dx) { return L[b][2][y + dy][x + dx]; };
      const double u0 = Lu(0, 0), v0 = Lv(0, 0), w0 = Lw(0, 0);
      const double up = L[nb][0][y][x], upxm = L[nb][0][y][x - 1];
      const double vp = L[nb][1][y][x], vpym = L[nb][1][y - 1][x];
      const double wp = L[nb][2][y][x];
      if (cact[r]) {
        const int64_t p = plane(k) + coff[r];
        const double su = combine(
            tcx, tcy, c1, c2,
            Lu(0, -1) * (Lu(0, -1) + u0), Lu(0, 1) * (u0 + Lu(0, 1)),
            Lu(-1, 0) * (Lv(-1, 0) + Lv(-1, 1)), Lu(1, 0) * (v0 + Lv(0, 1)),
            um1[r] * (wm1[r] + wm1x[r]), up * (w0 + Lw(0, 1)));
        const double sv = combine(
            tcx, tcy, c1, c2,
            Lv(0, -1) * (Lu(0, -1) + Lu(1, -1)), Lv(0, 1) * (u0 + Lu(1, 0)),
            Lv(-1, 0) * (Lv(-1, 0) + v0), Lv(1, 0) * (v0 + Lv(1, 0)),
            vm1[r] * (wm1[r] + wm1y[r]), vp * (w0 + Lw(1, 0)));
        const double sw = combine(
            tcx, tcy, c1, c2,
            Lw(0, -1) * (Lu(0, -1) + upxm), Lw(0, 1) * (u0 + up),
            Lw(-1, 0) * (Lv(-1, 0) + vpym), Lw(1, 0) * (v0 + vp),
            wm1[r] * (wm1[r] + w0), wp * (w0 + wp));
        __builtin_nontemporal_store(su, out[0] + p);
        __builtin_nontemporal_store(sv, out[1] + p);
        __builtin_nontemporal_store(sw, out[2] + p);
      }
      um1[r] = u0;
      vm1[r] = v0;
      wm1[r] = w0;
      wm1x[r] = Lw(0, 1);
      wm1y[r] = Lw(1, 0);
    }
  };
  for (int k = z0; k < z1; k += 2) {
    step(k, pa, pra);
    if (k + 1 < z1) step(k + 1, pb, prb);
  }
}

// ------------------------------------------------------------ direct kernel

__global__ __launch_bounds__(256) void advect_kernel(AdvK a) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= a.nx || j >= a.ny) return;
  const int z0 = blockIdx.z * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int64_t X = 1, Y = a.sy, Z = a.sz;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double* __restrict__ w = a.w;
  const double tcx = a.tcx, tcy = a.tcy;
  int64_t p = (int64_t)(z0 + 1) * Z + (int64_t)(j + 1) * Y + (i + 1);
  for (int k = z0; k < z1; ++k, p += Z) {
    const double c1 = a.t1[k], c2 = a.t2[k];
    const double u0 = u[p], v0 = v[p], w0 = w[p];
    a.su[p] = combine(tcx, tcy, c1, c2, u[p - X] * (u[p - X] + u0), u[p + X] * (u0 + u[p + X]),
                      u[p - Y] * (v[p - Y] + v[p - Y + X]), u[p + Y] * (v0 + v[p + X]),
                      u[p - Z] * (w[p - Z] + w[p - Z + X]), u[p + Z] * (w0 + w[p + X]));
    a.sv[p] = combine(tcx, tcy, c1, c2, v[p - X] * (u[p - X] + u[p - X + Y]),
                      v[p + X] * (u0 + u[p + Y]), v[p - Y] * (v[p - Y] + v0),
                      v[p + Y] * (v0 + v[p + Y]), v[p - Z] * (w[p - Z] + w[p - Z + Y]),
                      v[p + Z] * (w0 + w[p + Y]));
    a.sw[p] = combine(tcx, tcy, c1, c2, w[p - X] * (u[p - X] + u[p - X + Z]),
                      w[p + X] * (u0 + u[p + Z]), w[p - Y] * (v[p - Y] + v[p - Y + Z]),
                      w[p + Y] * (v0 + v[p + Z]), w[p - Z] * (w[p - Z] + w0),
                      w[p + Z] * (w0 + w[p + Z]));
  }
}

int env_int(const char* name) {
  const char* v = getenv(name);
  return v ? atoi(v) : 0;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int advect_source(const ms_grid* g, const double* u, const double* v,
                             const double* w, const double* tzc1, const double* tzc2,
                             double tcx, double tcy, double* su, double* sv, double* sw,
                             void* stream) {
  clear_error();
  if (int rc = check_grid(g, "advect_source")) return rc;
  if (!u || !v || !w || !tzc1 || !tzc2 || !su || !sv || !sw)
    return set_error(MS_EINVAL, "advect_source: NULL field or coefficient array");
  const size_t bytes = (size_t)field_span(*g) * 8;
  const void* ins[3] = {u, v, w};
  void* outs[3] = {su, sv, sw};
  for (int q = 0; q < 3; ++q) {
    for (int b = 0; b < 3; ++b)
      if (overlaps(outs[q], bytes, ins[b], bytes))
        return set_error(MS_EINVAL, "advect_source: an output aliases an input field");
    for (int b = q + 1; b < 3; ++b)
      if (overlaps(outs[q], bytes, outs[b], bytes))
        return set_error(MS_EINVAL, "advect_source: outputs overlap");
  }
  AdvK a{u, v, w, tzc1, tzc2, su, sv, sw, tcx, tcy, g->nx, g->ny, g->nz, 0, g->sy, g->sz};
  hipStream_t s = static_cast<hipStream_t>(stream);
  // MS_ADVECT_VARIANT=0 selects the direct kernel (a cross-check).
  if (getenv("MS_ADVECT_VARIANT") && env_int("MS_ADVECT_VARIANT") == 0) {
    if (g->ny > 4 * 65535) return set_error(MS_EUNSUPPORTED, "advect_source: ny too large");
    const int tiles = ((g->nx + 63) / 64) * ((g->ny + 3) / 4);
    int chunks = (4096 + tiles - 1) / tiles;
    if (chunks > g->nz) chunks = g->nz;
    a.zc = (g->nz + chunks - 1) / chunks;
    chunks = (g->nz + a.zc - 1) / a.zc;
    if (chunks > 65535) return set_error(MS_EUNSUPPORTED, "advect_source: nz too large");
    const dim3 grid((g->nx + 63) / 64, (g->ny + 3) / 4, chunks);
    hipLaunchKernelGGL(advect_kernel, grid, dim3(256), 0, s, a);
    MS_LAUNCH_CHECK();
    return MS_OK;
  }
  // Staged kernel: one block round of long z marches. Default: blocks of
  // eight waves (64 x 8 tiles, one row per thread; 63 KB of LDS, two blocks
  // per CU) on 512 blocks. Measured at 512 x 512 x 256 on one box: 675 us,
  // against 692 us on 1024 blocks and 728 us for four-wave blocks (64 x 4
  // tiles: more ring cells per cell). MS_ADVECT_WAVES (4 or 8),
  // MS_ADVECT_ROWS (1 or 2 rows per thread, four-wave blocks) and
  // MS_ADVECT_BLOCKS (target grid) select the alternatives.
  const int rows = env_int("MS_ADVECT_ROWS") == 2 ? 2 : 1;
  const int ew = env_int("MS_ADVECT_WAVES");
  const int waves = (ew == 4 || rows == 2) ? 4 : ew == 16 ? 16 : 8;
  const int64_t want = env_int("MS_ADVECT_BLOCKS") > 0 ? env_int("MS_ADVECT_BLOCKS")
                       : waves == 16                   ? 256
                       : waves == 8                    ? 512
                                                       : 1024;
  a.tiles_x = (g->nx + kAdvTX - 1) / kAdvTX;
  a.tiles_y = (g->ny + waves * rows - 1) / (waves * rows);
  const int64_t tiles2d = (int64_t)a.tiles_x * a.tiles_y;
  int zc = env_int("MS_ADVECT_ZC");
  if (zc <= 0) {
    int64_t chunks = (want + tiles2d - 1) / tiles2d;
    zc = (int)((g->nz + chunks - 1) / chunks);
    if (zc < 4) zc = 4;
  }
  if (zc > g->nz) zc = g->nz;
  const int64_t nb = tiles2d * ((g->nz + zc - 1) / zc);
  if (nb > 0x7fffffffLL) return set_error(MS_EUNSUPPORTED, "advect_source: grid too large");
  a.zc = zc;
  a.nblocks = (int)nb;
  // MS_ADVECT_GUARD=1: the predicated centre loads (cross-check)
  const bool guard = env_int("MS_ADVECT_GUARD") == 1;
  void (*kern)(AdvK);
  size_t dyn = 0;
  if (waves == 16) {
    kern = guard ? advect_staged_kernel<1, true, 16> : advect_staged_kernel<1, false, 16>;
    dyn = sizeof(double) * 4 * 3 * (16 + 2) * kAdvLX;
    MS_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
  } else if (waves == 8)
    kern = guard ? advect_staged_kernel<1, true, 8> : advect_staged_kernel<1, false, 8>;
  else if (rows == 1)
    kern = guard ? advect_staged_kernel<1, true, 4> : advect_staged_kernel<1, false, 4>;
  else
    kern = guard ? advect_staged_kernel<2, true, 4> : advect_staged_kernel<2, false, 4>;
  hipLaunchKernelGGL(kern, dim3(a.nblocks), dim3(64 * waves), dyn, s, a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}
