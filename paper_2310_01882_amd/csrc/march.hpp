// Device code shared by the sweep kernels and the batched solve: lane
// shifts across a wave and the two-sweep march of one wave over a column
// tile (internal; not installed).
#pragma once

#include "ms_internal.hpp"

namespace ms {

// Lane shifts (DPP).

// Lane l receives lane l-1's value (wave_shr:1); lane 0 keeps `old`.
__device__ __forceinline__ float lane_from_left(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v),
                                                    0x138, 0xf, 0xf, false));
}
// Lane l receives lane l+1's value (wave_shl:1); lane 63 keeps `old`.
__device__ __forceinline__ float lane_from_right(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v),
                                                    0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_from_left(double old, double v) {
  const long long o = __double_as_longlong(old), s = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x138, 0xf, 0xf,
                                             false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double old, double v) {
  const long long o = __double_as_longlong(old), s = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x130, 0xf, 0xf,
                                             false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Residual of one cell in FP64: r = f - (S - c*6) as written (FP32 values are
// widened exactly first); -(S - c*6) without f.
__device__ __forceinline__ double march_residual(double xp, double xm, double yp, double ym,
                                                 double zp, double zm, double c, double f,
                                                 bool has_f) {
  const double s = ((((xp + xm) + yp) + ym) + zp) + zm;
  const double lap = s - c * 6.0;
  return has_f ? f - lap : -lap;
}

// Two Jacobi sweeps of one wave's column tile, everything in registers and
// no barrier. Lane l owns column i (the caller passes i0 - 2 + l); stage A
// computes h = u_{k+1} on rows j0-1 .. j0+R at lanes 1..62, stage B writes
// u_{k+2} on rows j0 .. j0+R-1 at lanes 2..61, for levels z0 .. z1-1; all
// loads are clamped into the field (halo included), so any lane and row may
// lie outside it. acc_a / acc_b receive this lane's sums of r(u_k)^2 and
// r(u_{k+1})^2 over its output cells. Every lane of the wave must call it
// (the lane shifts read neighbours). Per-cell arithmetic is the single
// sweep's: (S - f) * c6 with S in the order x+, x-, y+, y-, z+, z-.
// Offsets within a z plane are 32-bit: the caller guarantees sz < 2^31.
// The fields are device (global) memory: the pointers are taken as such, so
// that loads and stores are global rather than flat instructions even when
// the caller read the pointers from memory (flat ones also count against
// the LDS counter, and need a 64-bit address per lane).
template <typename T, bool HAS_F, int R>
__device__ __forceinline__ void two_sweep_march(const T* __restrict__ src_any,
                                                T* __restrict__ dst_any,
                                                const T* __restrict__ f_any, int nx, int ny,
                                                int nz, int64_t sy, int64_t sz, int i, int j0,
                                                int z0, int z1, T c6, double& acc_a,
                                                double& acc_b) {
  using GT = __attribute__((address_space(1))) T;
  const GT* __restrict__ src = (const GT*)src_any;
  GT* __restrict__ dst = (GT*)dst_any;
  const GT* __restrict__ f = (const GT*)f_any;
  const int lane = threadIdx.x & 63;
  const bool colA = lane >= 1 && lane <= 62, colB = lane >= 2 && lane <= 61;
  const bool xin = i >= 0 && i < nx;
  const int col = min(max(i, -1), nx) + 1;
  const int sy32 = (int)sy;
  // offsets within a plane (clamped into the field) of rows j0-2 .. j0+R+1
  int roff[R + 4];
  bool yin[R + 4];
#pragma unroll
  for (int q = 0; q < R + 4; ++q) {
    const int j = j0 - 2 + q;
    roff[q] = (min(max(j, -1), ny) + 1) * sy32 + col;
    yin[q] = j >= 0 && j < ny;
  }
  auto plane = [&](int z) { return (int64_t)(min(max(z, -1), nz) + 1) * sz; };
  // u_k rows j0-2 .. j0+R+1 (q = 0 .. R+3) at level z
  auto load_u = [&](T (&r)[R + 4], int z) {
    const GT* pl = src + plane(z);
#pragma unroll
    for (int q = 0; q < R + 4; ++q) r[q] = pl[roff[q]];
  };
  // f rows j0-1 .. j0+R (q = 1 .. R+2) at level z
  auto load_f = [&](T (&r)[R + 2], int z) {
    const GT* pl = HAS_F ? f + plane(z) : f;
#pragma unroll
    for (int q = 0; q < R + 2; ++q) r[q] = HAS_F ? pl[roff[q + 1]] : T(0);
  };

  T um[R + 2];        // u_k at z-1, rows j0-1 .. j0+R
  T uc[R + 4];        // u_k at z, rows j0-2 .. j0+R+1
  T up[R + 4];        // u_k at z+1
  T fa[R + 2];        // f at z, rows j0-1 .. j0+R (stage A)
  T fb[R];            // f at z-1, rows j0 .. j0+R-1 (stage B)
  T hm2[R], hm1[R + 2];  // h at z-2 (output rows) and z-1 (rows j0-1 .. j0+R)
  {
    T t[R + 4];
    load_u(t, z0 - 2);
#pragma unroll
    for (int q = 0; q < R + 2; ++q) um[q] = t[q + 1];
  }
  load_u(uc, z0 - 1);
  load_u(up, z0);
  load_f(fa, z0 - 1);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    fb[q] = T(0);
    hm2[q] = T(0);
  }
#pragma unroll
  for (int q = 0; q < R + 2; ++q) hm1[q] = T(0);

  const bool wave_live = j0 < ny;
  for (int z = z0 - 1; z <= z1 && wave_live; ++z) {
    // next level's loads first: u_k at z+2, f at z+1. Unconditional (past
    // the chunk they read clamped levels whose values are never used): a
    // load under a branch makes the wait after the join count as if the
    // branch had not been taken, i.e. wait for the loads just issued.
    T un[R + 4], fn[R + 2];
    load_u(un, z + 2);
    load_f(fn, z + 1);
    // stage A at level z: h on rows j0-1 .. j0+R
    const bool zA = z >= 0 && z < nz, zres = z >= z0 && z < z1;
    T hn[R + 2];
#pragma unroll
    for (int q = 0; q < R + 2; ++q) {
      const T c = uc[q + 1];
      const T xp = lane_from_right(c, c), xm = lane_from_left(c, c);
      const T yp = uc[q + 2], ym = uc[q];
      const T zp = up[q + 1], zm = um[q];
      const T sum = ((((xp + xm) + yp) + ym) + zp) + zm;
      hn[q] = (colA && xin && yin[q + 1] && zA) ? (HAS_F ? (sum - fa[q]) * c6 : sum * c6) : c;
      if (q >= 1 && q <= R && colB && xin && yin[q + 1] && zres) {
        const double r = march_residual(xp, xm, yp, ym, zp, zm, c, fa[q], HAS_F);
        acc_a += r * r;
      }
    }
    // stage B at level z-1: output rows j0 .. j0+R-1
    const int zb = z - 1;
    if (zb >= z0 && zb < z1) {
      const int64_t pb = (int64_t)(zb + 1) * sz;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const T c = hm1[q + 1];
        const T xp = lane_from_right(c, c), xm = lane_from_left(c, c);
        const T yp = hm1[q + 2], ym = hm1[q];
        const T zp = hn[q + 1], zm = hm2[q];
        const T sum = ((((xp + xm) + yp) + ym) + zp) + zm;
        const T v = HAS_F ? (sum - fb[q]) * c6 : sum * c6;
        if (colB && xin && yin[q + 2]) {
          __builtin_nontemporal_store(v, dst + pb + roff[q + 2]);
          const double r = march_residual(xp, xm, yp, ym, zp, zm, c, fb[q], HAS_F);
          acc_b += r * r;
        }
      }
    }
    // shift the queues
#pragma unroll
    for (int q = 0; q < R; ++q) {
      hm2[q] = hm1[q + 1];
      fb[q] = fa[q + 1];
    }
#pragma unroll
    for (int q = 0; q < R + 2; ++q) {
      hm1[q] = hn[q];
      um[q] = uc[q + 1];
    }
#pragma unroll
    for (int q = 0; q < R + 4; ++q) {
      uc[q] = up[q];
      up[q] = un[q];
    }
#pragma unroll
    for (int q = 0; q < R + 2; ++q) fa[q] = fn[q];
  }

}

}  // namespace ms
