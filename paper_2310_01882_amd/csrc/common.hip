// Error reporting, grid validation and launch geometry shared by the
// mistencil entry points.
#include "ms_internal.hpp"

#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

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

namespace {
int env_int(const char* name) {
  const char* v = getenv(name);
  return v ? atoi(v) : 0;
}
}  // namespace

int vec_alignment(const ms_grid& g, int dtype, const void* const* ptrs, int n) {
  const int esz = dtype == MS_F64 ? 8 : 4;
  int v = 16 / esz;
  for (; v > 1; v >>= 1) {
    bool ok = (g.sy % v == 0) && (g.sz % v == 0);
    for (int q = 0; q < n && ok; ++q) {
      if (!ptrs[q]) continue;
      const uintptr_t p = reinterpret_cast<uintptr_t>(ptrs[q]);
      ok = (p % esz == 0) && ((p / esz + 1) % v == 0);
    }
    if (ok) break;
  }
  return v;
}

namespace {

// Two resident blocks per CU over 256 CUs: measured on 512^3 FP64 and FP32
// sweeps, a grid that is exactly resident once (no second round, long z
// marches, few concurrent DRAM streams) beats deeper oversubscription.
constexpr int64_t kTargetBlocks = 512;

// Splits z so that the grid has about `want` blocks, at least 4 planes per
// chunk, and never more than kMaxBlocks blocks.
void split_z(SweepGeom& s, const ms_grid& g, int zc_hint, int64_t want) {
  const int64_t tiles2d = (int64_t)s.tiles_x * s.tiles_y;
  int zc = zc_hint;
  if (zc <= 0) {
    int64_t chunks = (want + tiles2d - 1) / tiles2d;
    if (chunks < 1) chunks = 1;
    zc = (int)((g.nz + chunks - 1) / chunks);
    if (zc < 4) zc = 4;
  }
  if (zc > g.nz) zc = g.nz;
  while (tiles2d * ((g.nz + zc - 1) / zc) > kMaxBlocks && zc < g.nz) zc *= 2;
  if (zc > g.nz) zc = g.nz;
  s.zc = zc;
  s.chunks_z = (g.nz + zc - 1) / zc;
  const int64_t nb = tiles2d * s.chunks_z;
  s.nblocks = nb > kMaxBlocks ? kMaxBlocks + 1 : (int)nb;  // > kMaxBlocks is rejected at launch
}

}  // namespace

SweepGeom sweep_geom_lds(const ms_grid& g) {
  SweepGeom s{};
  s.variant = kVariantLds;
  s.vec = 1;
  s.wx = 1;
  s.rows = 4;
  s.tiles_x = (g.nx + kTileX - 1) / kTileX;
  s.tiles_y = (g.ny + kWavesY * s.rows - 1) / (kWavesY * s.rows);
  split_z(s, g, 0, kTargetBlocks);
  return s;
}

SweepGeom geom_register(const ms_grid& g, int dtype, int vec_ok, int vec, int wx, int rows,
                        int zc_hint, int64_t target_blocks) {
  SweepGeom s{};
  s.variant = kVariantRegister;
  const int vmax = dtype == MS_F64 ? 2 : 4;
  if (vec != 1 && vec != 2 && vec != 4) vec = vmax;
  if (vec > vmax) vec = vmax;
  while (vec > vec_ok) vec >>= 1;
  // Narrow grids: do not let a lane hold cells that do not exist.
  while (vec > 1 && 64 * vec > g.nx + 64) vec >>= 1;
  s.vec = vec;
  if (wx != 1 && wx != 2 && wx != 4) {
    const int waves_x = (g.nx + 64 * vec - 1) / (64 * vec);
    wx = waves_x >= 2 ? 2 : 1;
  }
  s.wx = wx;
  s.rows = (rows == 2 || rows == 4 || rows == 8) ? rows : 2;
  s.tiles_x = (g.nx + 64 * vec * wx - 1) / (64 * vec * wx);
  const int tile_y = (kWavesY / wx) * s.rows;
  s.tiles_y = (g.ny + tile_y - 1) / tile_y;
  split_z(s, g, zc_hint, target_blocks > 0 ? target_blocks : kTargetBlocks);
  return s;
}

// ------------------------------------------------------------ tuning table

namespace {
struct TuneKey {
  int dtype, nx, ny, nz, vec_ok;
  bool operator<(const TuneKey& o) const {
    return std::tie(dtype, nx, ny, nz, vec_ok) < std::tie(o.dtype, o.nx, o.ny, o.nz, o.vec_ok);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, ms_tuning> g_tune;
}  // namespace

bool tuned_lookup(const ms_grid& g, int dtype, int vec_ok, ms_tuning* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey{dtype, g.nx, g.ny, g.nz, vec_ok});
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void tuned_store(const ms_tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey{t.dtype, t.nx, t.ny, t.nz, t.vec_ok}] = t;
}

int tuned_export(ms_tuning* out, int cap) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int n = 0;
  for (const auto& kv : g_tune) {
    if (out && n < cap) out[n] = kv.second;
    ++n;
  }
  return n;
}

void tuned_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

SweepGeom sweep_geom(const ms_grid& g, int dtype, int vec_ok) {
  const int ev = env_int("MS_SWEEP_VARIANT");
  const bool forced = getenv("MS_SWEEP_VARIANT") || getenv("MS_SWEEP_VEC") ||
                      getenv("MS_SWEEP_ROWS") || getenv("MS_SWEEP_WX") || getenv("MS_SWEEP_ZC");
  if (getenv("MS_SWEEP_VARIANT") && ev == 0) {
    SweepGeom s{};
    s.variant = kVariantLds;
    s.vec = 1;
    s.wx = 1;
    const int rows = env_int("MS_SWEEP_ROWS");
    s.rows = (rows == 8) ? 8 : 4;
    s.tiles_x = (g.nx + kTileX - 1) / kTileX;
    s.tiles_y = (g.ny + kWavesY * s.rows - 1) / (kWavesY * s.rows);
    split_z(s, g, env_int("MS_SWEEP_ZC"), kTargetBlocks);
    return s;
  }
  ms_tuning t{};
  if (!forced && tuned_lookup(g, dtype, vec_ok, &t))
    return geom_register(g, dtype, vec_ok, t.vec, t.wx, t.rows, 0, t.target_blocks);
  return geom_register(g, dtype, vec_ok, env_int("MS_SWEEP_VEC"), env_int("MS_SWEEP_WX"),
                       env_int("MS_SWEEP_ROWS"), env_int("MS_SWEEP_ZC"), kTargetBlocks);
}

}  // namespace ms

extern "C" const char* ms_last_error(void) { return ms::last_error(); }

extern "C" const char* ms_version(void) { return "mistencil 0.1 (gfx950)"; }
