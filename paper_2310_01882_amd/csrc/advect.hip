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
// One thread owns an (i, j) column of a tile and marches up a z-chunk. The
// values of u, v, w on the column at levels k-1, k, k+1 rotate through
// registers; in-plane neighbours are read from global memory and served by
// the L1/L2 caches (neighbouring lanes touch the same lines).
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
};

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
    {
      const double pxm = u[p - X] * (u[p - X] + u0);
      const double pxp = u[p + X] * (u0 + u[p + X]);
      const double pym = u[p - Y] * (v[p - Y] + v[p - Y + X]);
      const double pyp = u[p + Y] * (v0 + v[p + X]);
      const double pzm = u[p - Z] * (w[p - Z] + w[p - Z + X]);
      const double pzp = u[p + Z] * (w0 + w[p + X]);
      a.su[p] = (tcx * (pxm - pxp) + tcy * (pym - pyp)) + (c1 * pzm - c2 * pzp);
    }
    {
      const double pxm = v[p - X] * (u[p - X] + u[p - X + Y]);
      const double pxp = v[p + X] * (u0 + u[p + Y]);
      const double pym = v[p - Y] * (v[p - Y] + v0);
      const double pyp = v[p + Y] * (v0 + v[p + Y]);
      const double pzm = v[p - Z] * (w[p - Z] + w[p - Z + Y]);
      const double pzp = v[p + Z] * (w0 + w[p + Y]);
      a.sv[p] = (tcx * (pxm - pxp) + tcy * (pym - pyp)) + (c1 * pzm - c2 * pzp);
    }
    {
      const double pxm = w[p - X] * (u[p - X] + u[p - X + Z]);
      const double pxp = w[p + X] * (u0 + u[p + Z]);
      const double pym = w[p - Y] * (v[p - Y] + v[p - Y + Z]);
      const double pyp = w[p + Y] * (v0 + v[p + Z]);
      const double pzm = w[p - Z] * (w[p - Z] + w0);
      const double pzp = w[p + Z] * (w0 + w[p + Z]);
      a.sw[p] = (tcx * (pxm - pxp) + tcy * (pym - pyp)) + (c1 * pzm - c2 * pzp);
    }
  }
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
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      if (overlaps(outs[a], bytes, ins[b], bytes))
        return set_error(MS_EINVAL, "advect_source: an output aliases an input field");
    for (int b = a + 1; b < 3; ++b)
      if (overlaps(outs[a], bytes, outs[b], bytes))
        return set_error(MS_EINVAL, "advect_source: outputs overlap");
  }
  if (g->ny > 4 * 65535) return set_error(MS_EUNSUPPORTED, "advect_source: ny too large");
  AdvK a{u, v, w, tzc1, tzc2, su, sv, sw, tcx, tcy, g->nx, g->ny, g->nz, 0, g->sy, g->sz};
  const int tiles = ((g->nx + 63) / 64) * ((g->ny + 3) / 4);
  int chunks = (4096 + tiles - 1) / tiles;
  if (chunks > g->nz) chunks = g->nz;
  a.zc = (g->nz + chunks - 1) / chunks;
  chunks = (g->nz + a.zc - 1) / a.zc;
  if (chunks > 65535) return set_error(MS_EUNSUPPORTED, "advect_source: nz too large");
  const dim3 grid((g->nx + 63) / 64, (g->ny + 3) / 4, chunks);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(advect_kernel, grid, dim3(256), 0, s, a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}
