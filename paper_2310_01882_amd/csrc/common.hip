// Error reporting, grid validation and launch geometry shared by the
// mistencil entry points.
#include "ms_internal.hpp"

#include <cstring>

namespace ms {

namespace {
thread_local char g_err[512] = {0};
}

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

const char* last_error() { return g_err; }

int check_grid(const ms_grid* g, const char* who) {
  if (!g) return set_error(MS_EINVAL, "%s: grid descriptor is NULL", who);
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return set_error(MS_EINVAL, "%s: extents must be >= 1 (got %d x %d x %d)", who,
                     g->nx, g->ny, g->nz);
  if (g->reserved != 0) return set_error(MS_EINVAL, "%s: grid.reserved must be 0", who);
  if (g->sy < (int64_t)g->nx + 2)
    return set_error(MS_EINVAL, "%s: sy = %lld < nx + 2 = %d", who, (long long)g->sy,
                     g->nx + 2);
  if (g->sz < g->sy * ((int64_t)g->ny + 2))
    return set_error(MS_EINVAL, "%s: sz = %lld < sy * (ny + 2) = %lld", who,
                     (long long)g->sz, (long long)(g->sy * ((int64_t)g->ny + 2)));
  // Offsets are formed in 64-bit arithmetic; extents stay below 2^30 so that
  // every per-axis index fits a 32-bit int with room for the halo.
  if (g->nx > (1 << 30) || g->ny > (1 << 30) || g->nz > (1 << 30))
    return set_error(MS_EINVAL, "%s: extent above 2^30", who);
  return MS_OK;
}

SweepGeom sweep_geom(const ms_grid& g, int zc_hint) {
  SweepGeom s;
  s.tiles_x = (g.nx + kTileX - 1) / kTileX;
  s.tiles_y = (g.ny + kTileY - 1) / kTileY;
  const int64_t tiles2d = (int64_t)s.tiles_x * s.tiles_y;
  int zc = zc_hint;
  if (zc <= 0) {
    // Enough z-chunks for ~8 blocks per CU over 256 CUs, but at least 4
    // planes per chunk so that the two re-read boundary planes stay cheap.
    const int64_t want_blocks = 2048;
    int64_t chunks = (want_blocks + tiles2d - 1) / tiles2d;
    if (chunks < 1) chunks = 1;
    zc = (int)((g.nz + chunks - 1) / chunks);
    if (zc < 4) zc = 4;
  }
  if (zc > g.nz) zc = g.nz;
  s.zc = zc;
  s.chunks_z = (g.nz + zc - 1) / zc;
  s.nblocks = (int)(tiles2d * s.chunks_z);
  return s;
}

}  // namespace ms

extern "C" const char* ms_last_error(void) { return ms::last_error(); }

extern "C" const char* ms_version(void) { return "mistencil 0.1 (gfx950)"; }
