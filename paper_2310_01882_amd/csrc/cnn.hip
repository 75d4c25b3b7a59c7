// Learned warm start: 3x3x3 convolutions on BF16 MFMA with FP32
// accumulation (forward, input gradient, weight gradient), the MSE loss,
// Adam, and the feature / guess kernels.
//
// Activations are channels-last with a one-voxel zero halo ("same" zero
// padding): element (x, y, z, c) of an X x Y x Z volume with C channels is
// at ((((z+1)*(Y+2) + (y+1))*(X+2) + (x+1))*C + c). C is 8 (input features)
// or 32 (hidden layers); output channels are always padded to 32.
//
// Every convolution is an implicit GEMM on v_mfma_f32_32x32x16_bf16: a wave
// owns 32 consecutive voxels along x (M) times 32 channels (N) and walks K
// = 27 taps x input channels in steps of 16; the lane layout (checked on
// the device) is A[m = l%32][k = 8(l/32)+e], B[k = 8(l/32)+e][n = l%32],
// D[m = 8(r/4) + 4(l/32) + r%4][n = l%32].
//  * forward:  A = input at voxel + tap offset, B = W[tap][co][ci] (LDS);
//    epilogue adds the bias, applies ReLU (hidden layers) and stores BF16,
//    or stores channel 0 in FP32 (last layer).
//  * dgrad:    A = output gradient at voxel - tap offset, B = W[tap][ci][co];
//    epilogue multiplies by the ReLU mask of the layer input (post > 0).
//  * wgrad:    dW[tap][co][ci] = sum over voxels of dPre[v][co] in[v+d][ci];
//    M = co, N = ci (or, for 8 input channels, N = (dx, ci)), K = voxels
//    in steps of 16, operands staged and transposed through LDS, block tasks
//    of 32 voxels x 4 rows; per-block partials are summed by a second kernel
//    in a fixed order (deterministic).
#include "ms_internal.hpp"

#include <hip/hip_bf16.h>

#include <algorithm>

namespace ms {
namespace {

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kTaps = 27;
constexpr int kCo = 32;  // padded output channels

__device__ __forceinline__ void tap_offset(int t, int& dx, int& dy, int& dz) {
  dx = t % 3 - 1;
  dy = (t / 3) % 3 - 1;
  dz = t / 9 - 1;
}

struct Vol {
  int X, Y, Z;
  __device__ __forceinline__ int64_t vox(int x, int y, int z) const {
    return (((int64_t)(z + 1) * (Y + 2) + (y + 1)) * (X + 2) + (x + 1));
  }
};

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int e = 0; e < 8; ++e) z[e] = (bf16)0.0f;
  return z;
}

// ------------------------------------------------------------- forward

struct FwdK {
  Vol v;
  const bf16* in;      // C = CIN
  const bf16* w;       // [27][32][CIN]
  const float* bias;   // [32]
  bf16* out;           // C = 32 (hidden layers)
  float* out32;        // channel 0 in FP32 (last layer), field layout
  int relu;
  int nseg;
};

template <int CIN>
__global__ __launch_bounds__(256) void conv_fwd_kernel(FwdK a) {
  __shared__ bf16x8 wl[kTaps * kCo * CIN / 8];
  for (int t = threadIdx.x; t < kTaps * kCo * CIN / 8; t += blockDim.x)
    wl[t] = reinterpret_cast<const bf16x8*>(a.w)[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + 31) / 32;
  constexpr int KS = (kTaps * CIN + 15) / 16;
  const float bj = a.bias[m];
  for (int seg = blockIdx.x * 4 + w; seg < a.nseg; seg += gridDim.x * 4) {
    const int x0 = (seg % sx) * 32, y = (seg / sx) % a.v.Y, z = seg / (sx * a.v.Y);
    f32x16 acc = {};
#pragma unroll 2
    for (int s = 0; s < KS; ++s) {
      const int k0 = s * 16 + 8 * h;
      const int t = k0 / CIN, c0 = k0 % CIN;
      // Unconditional load from a clamped tap and x (a lane past the interior
      // feeds only outputs that are not stored; a tap past the last gets a
      // zero weight), so that the loads pipeline.
      int dx, dy, dz;
      tap_offset(t < kTaps ? t : kTaps - 1, dx, dy, dz);
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(
          a.in + a.v.vox(min(x0 + m + dx, a.v.X), y + dy, z + dz) * CIN + c0);
      const bf16x8 bv = t < kTaps ? wl[((t * kCo + m) * CIN + c0) / 8] : zero8();
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      const int x = x0 + i;
      if (x >= a.v.X) continue;
      float val = acc[r] + bj;
      if (a.relu) val = fmaxf(val, 0.0f);
      const int64_t p = a.v.vox(x, y, z);
      if (a.out) a.out[p * kCo + m] = (bf16)val;
      if (a.out32 && m == 0) a.out32[p] = val;
    }
  }
}

// --------------------------------------------------------------- dgrad

struct DgK {
  Vol v;
  const bf16* dout;  // C = 32 (gradient w.r.t. the layer's pre-activation)
  const bf16* wd;    // [27][CIN][32]
  const bf16* mask;  // layer input (post-ReLU of the previous layer), C = CIN
  bf16* din;         // C = CIN: gradient w.r.t. the previous pre-activation
  int nseg;
};

template <int CIN>
__global__ __launch_bounds__(256) void conv_dgrad_kernel(DgK a) {
  __shared__ bf16x8 wl[kTaps * CIN * kCo / 8];
  for (int t = threadIdx.x; t < kTaps * CIN * kCo / 8; t += blockDim.x)
    wl[t] = reinterpret_cast<const bf16x8*>(a.wd)[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + 31) / 32;
  constexpr int KS = kTaps * kCo / 16;
  for (int seg = blockIdx.x * 4 + w; seg < a.nseg; seg += gridDim.x * 4) {
    const int x0 = (seg % sx) * 32, y = (seg / sx) % a.v.Y, z = seg / (sx * a.v.Y);
    const bool mok = x0 + m < a.v.X;
    f32x16 acc = {};
#pragma unroll 2
    for (int s = 0; s < KS; ++s) {
      const int k0 = s * 16 + 8 * h;
      const int t = k0 / kCo, c0 = k0 % kCo;
      int dx, dy, dz;
      tap_offset(t, dx, dy, dz);
      bf16x8 av = zero8(), bv = zero8();
      // input voxel q feeds output q - d through tap d
      if (mok)
        av = *reinterpret_cast<const bf16x8*>(a.dout + a.v.vox(x0 + m - dx, y - dy, z - dz) * kCo +
                                              c0);
      if (m < CIN) bv = wl[((t * CIN + m) * kCo + c0) / 8];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    if (m >= CIN) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      const int x = x0 + i;
      if (x >= a.v.X) continue;
      const int64_t p = a.v.vox(x, y, z);
      float g = acc[r];
      if (a.mask && !((float)a.mask[p * CIN + m] > 0.0f)) g = 0.0f;
      a.din[p * CIN + m] = (bf16)g;
    }
  }
}

// ------------------------------------------- row-blocked 32-channel kernel
//
// Forward (kDgrad = false) and input gradient (kDgrad = true) of a layer
// with 32 input channels, register-blocked over kRows output rows: a wave
// owns 32 voxels along x (M) on kRows consecutive rows y0..y0+kRows-1 of
// one z level, all 32 output channels (N), with one accumulator per row.
// K is walked in 18 groups (dz, dx, half of the channels); a group loads
// the kRows+2 input rows that its rows can reach (one 16-byte load per lane
// each) and the three weight fragments of dy = -1, 0, 1 (from LDS), then
// issues 3 kRows MFMAs: input row k feeds output row r through
// dy = sgn*(k - 1 - r), so each load serves up to three MFMAs and each
// weight fragment all kRows rows. The next group's input rows are loaded
// while the current group's MFMAs run. Forward reads input voxel
// v + d for tap d, the input gradient reads output-gradient voxel q - d
// (sgn = -1). Epilogues as in the one-row kernels above.
struct RowK {
  Vol v;
  const bf16* src;    // forward: layer input; dgrad: gradient of the pre-activation
  const bf16* w;      // forward: [27][32][32] (tap, co, ci); dgrad: [27][32][32] (tap, ci, co)
  const float* bias;  // forward only
  bf16* out;          // forward hidden layers: output, C = 32
  float* out32;       // forward last layer: channel 0 in FP32
  const bf16* mask;   // dgrad: the layer input (ReLU mask), C = 32, or null
  bf16* din;          // dgrad: output, C = 32
  int relu;
  int nseg;           // (X/32 rounded up) * (Y/kRows rounded up) * Z
};

constexpr int kConvRows = 4;

template <bool kDgrad>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_rows_kernel(RowK a) {
  constexpr int C = 32;
  constexpr int R = kConvRows;
  constexpr int sgn = kDgrad ? -1 : 1;
  // Weights in LDS as 16-byte chunks ordered [tap][channel half][m][h]
  // (global order: [tap][m][c8], c8 = 2 * half + h), so that the 64 lanes
  // of one operand read (fixed tap and half; m = lane % 32, h = lane / 32)
  // take 64 consecutive chunks: no two lanes of a read share a bank.
  __shared__ bf16x8 wl[kTaps * kCo * C / 8];
  for (int gi = threadIdx.x; gi < kTaps * kCo * C / 8; gi += blockDim.x) {
    const int t = gi / (kCo * 4), co = (gi / 4) % kCo, c8 = gi % 4;
    wl[((t * 2 + c8 / 2) * kCo + co) * 2 + c8 % 2] = reinterpret_cast<const bf16x8*>(a.w)[gi];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + 31) / 32, sy = (a.v.Y + R - 1) / R;
  const float bj = kDgrad ? 0.0f : a.bias[m];
  for (int seg = blockIdx.x * 4 + w; seg < a.nseg; seg += gridDim.x * 4) {
    const int x0 = (seg % sx) * 32, y0 = ((seg / sx) % sy) * R, z = seg / (sx * sy);
    f32x16 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = f32x16{};
    // input rows y0 - 1 + k, k = 0 .. R+1, of group g = (dz, dx, channel half).
    // The loads are unconditional, from coordinates clamped into the volume
    // (halo included): a clamped lane (x past the interior) or row (y past
    // the halo) feeds only outputs that are not stored, and a conditional
    // load would have to complete before its branch joins.
    auto load_rows = [&](bf16x8 (&av)[R + 2], int g) {
      const int dz = g / 6 - 1, dx = (g / 2) % 3 - 1, c0 = (g % 2) * 16 + 8 * h;
      const int x = min(x0 + m + sgn * dx, a.v.X);
#pragma unroll
      for (int k = 0; k < R + 2; ++k) {
        const int yy = min(y0 - 1 + k, a.v.Y);
        av[k] = *reinterpret_cast<const bf16x8*>(a.src + a.v.vox(x, yy, z + sgn * dz) * C + c0);
      }
    };
    bf16x8 cur[R + 2], nxt[R + 2];
    load_rows(cur, 0);
#pragma unroll
    for (int g = 0; g < 18; ++g) {
      if (g + 1 < 18) load_rows(nxt, g + 1);
      const int dz = g / 6 - 1, dx = (g / 2) % 3 - 1;
      bf16x8 bv[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int t = (dx + 1) + 3 * d + 9 * (dz + 1);  // dy = d - 1
        bv[d] = wl[((t * 2 + g % 2) * kCo + m) * 2 + h];
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int k = r + 1 + sgn * (d - 1);  // input row feeding row r at dy = d - 1
          acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur[k], bv[d], acc[r], 0, 0, 0);
        }
#pragma unroll
      for (int k = 0; k < R + 2; ++k) cur[k] = nxt[k];
    }
    // keep the epilogue's loads (the ReLU mask) below the MFMA chain
    __builtin_amdgcn_sched_barrier(0);
    // dgrad: all R x 16 mask values of the task first (the operand buffers
    // are dead by now), so that their loads share one round trip
    // Loads are unconditional (coordinates past the interior are clamped to
    // the halo, whose outputs are not stored): a conditional load would
    // have to complete before its branch joins, one round trip per value.
    bf16 mk[kDgrad ? R : 1][16];
    if constexpr (kDgrad) {
      if (a.mask) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int x = min(x0 + 8 * (q / 4) + 4 * h + (q % 4), a.v.X);
            const int y = min(y0 + r, a.v.Y);
            mk[r][q] = a.mask[a.v.vox(x, y, z) * C + m];
          }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 16; ++q) mk[r][q] = (bf16)1.0f;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = y0 + r;
      if (y >= a.v.Y) break;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 8 * (q / 4) + 4 * h + (q % 4);
        const int x = x0 + i;
        if (x >= a.v.X) continue;
        const int64_t p = a.v.vox(x, y, z);
        if constexpr (kDgrad) {
          const float gv = (float)mk[r][q] > 0.0f ? acc[r][q] : 0.0f;
          a.din[p * C + m] = (bf16)gv;
        } else {
          float val = acc[r][q] + bj;
          if (a.relu) val = fmaxf(val, 0.0f);
          if (a.out) a.out[p * kCo + m] = (bf16)val;
          if (a.out32 && m == 0) a.out32[p] = val;
        }
      }
    }
  }
}

// ------------------------------------------ lane-shifted 32-channel kernel
//
// The row-blocked kernel's work with a third of its L1 data: a wave's 32
// lanes (per K half) hold input voxels x0-1 .. x0+30 and it stores the 30
// outputs x0 .. x0+29. The dx = -1 and +1 neighbours of a loaded row are the
// adjacent lanes' values (DPP shift of the whole wave by one lane), so the
// rows of a z level are loaded once, both channel halves, for all three dx
// taps. Lanes 0 and 31 of each half are halo voxels: the shift fills them
// with a neighbour half's value or zero, and their outputs are not stored.
// The MFMAs run in the row-blocked kernel's order (dz, dx, channel half;
// rows; dy), so every accumulator sums the same products in the same order.
constexpr int kShiftVox = 30;

// s = +1: lane l receives lane l+1's value; s = -1: lane l-1's; 0 elsewhere.
__device__ __forceinline__ bf16x8 shift_lanes(bf16x8 v, int s) {
  typedef __attribute__((ext_vector_type(4))) int i32x4;
  const i32x4 x = __builtin_bit_cast(i32x4, v);
  i32x4 y;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    y[e] = s > 0 ? __builtin_amdgcn_update_dpp(0, x[e], 0x130, 0xf, 0xf, false)
                 : __builtin_amdgcn_update_dpp(0, x[e], 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(bf16x8, y);
}

template <bool kDgrad>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_shift_kernel(RowK a) {
  constexpr int C = 32;
  constexpr int R = kConvRows;
  constexpr int sgn = kDgrad ? -1 : 1;
  __shared__ bf16x8 wl[kTaps * kCo * C / 8];  // layout as in conv_rows_kernel
  for (int gi = threadIdx.x; gi < kTaps * kCo * C / 8; gi += blockDim.x) {
    const int t = gi / (kCo * 4), co = (gi / 4) % kCo, c8 = gi % 4;
    wl[((t * 2 + c8 / 2) * kCo + co) * 2 + c8 % 2] = reinterpret_cast<const bf16x8*>(a.w)[gi];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + kShiftVox - 1) / kShiftVox, sy = (a.v.Y + R - 1) / R;
  const float bj = kDgrad ? 0.0f : a.bias[m];
  for (int seg = blockIdx.x * 4 + w; seg < a.nseg; seg += gridDim.x * 4) {
    const int x0 = (seg % sx) * kShiftVox, y0 = ((seg / sx) % sy) * R, z = seg / (sx * sy);
    f32x16 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = f32x16{};
    // rows y0-1 .. y0+R of level z + sgn*dz, both channel halves, at this
    // lane's voxel x0-1+m; coordinates clamped into the volume (halo
    // included), unconditional loads as in conv_rows_kernel
    auto load_level = [&](bf16x8 (&av)[2][R + 2], int dz) {
      const int x = min(x0 - 1 + m, a.v.X);
#pragma unroll
      for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int k = 0; k < R + 2; ++k) {
          const int yy = min(y0 - 1 + k, a.v.Y);
          av[half][k] = *reinterpret_cast<const bf16x8*>(
              a.src + a.v.vox(x, yy, z + sgn * dz) * C + half * 16 + 8 * h);
        }
    };
    bf16x8 cur[2][R + 2], nxt[2][R + 2];
    load_level(cur, -1);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int dz = l - 1;
      if (l + 1 < 3) load_level(nxt, dz + 1);  // in flight while this level computes
      // keep those loads ahead of this level's MFMAs (left to itself the
      // scheduler sinks them to just before their first use: 175 -> 143 us
      // forward, 203 -> 171 us input gradient at 128^3 with this barrier)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi) {
        const int dx = dxi - 1;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          bf16x8 rows[R + 2];
#pragma unroll
          for (int k = 0; k < R + 2; ++k)
            rows[k] = dx == 0 ? cur[half][k] : shift_lanes(cur[half][k], sgn * dx);
          bf16x8 bv[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int t = (dx + 1) + 3 * d + 9 * (dz + 1);  // dy = d - 1
            bv[d] = wl[((t * 2 + half) * kCo + m) * 2 + h];
          }
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const int k = r + 1 + sgn * (d - 1);
              acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rows[k], bv[d], acc[r], 0, 0, 0);
            }
        }
      }
      if (l + 1 < 3) {
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
          for (int k = 0; k < R + 2; ++k) cur[half][k] = nxt[half][k];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    bf16 mk[kDgrad ? R : 1][16];
    if constexpr (kDgrad) {
      if (a.mask) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int x = min(x0 - 1 + 8 * (q / 4) + 4 * h + (q % 4), a.v.X);
            const int y = min(y0 + r, a.v.Y);
            mk[r][q] = a.mask[a.v.vox(x, y, z) * C + m];
          }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 16; ++q) mk[r][q] = (bf16)1.0f;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = y0 + r;
      if (y >= a.v.Y) break;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 8 * (q / 4) + 4 * h + (q % 4);  // lane voxel x0-1+i
        const int x = x0 - 1 + i;
        if (i < 1 || i > kShiftVox || x >= a.v.X) continue;
        const int64_t p = a.v.vox(x, y, z);
        if constexpr (kDgrad) {
          const float gv = (float)mk[r][q] > 0.0f ? acc[r][q] : 0.0f;
          a.din[p * C + m] = (bf16)gv;
        } else {
          float val = acc[r][q] + bj;
          if (a.relu) val = fmaxf(val, 0.0f);
          if (a.out) a.out[p * kCo + m] = (bf16)val;
          if (a.out32 && m == 0) a.out32[p] = val;
        }
      }
    }
  }
}

// ------------------------------------ lane-shifted 8-channel forward
//
// The first layer (8 input channels) in the lane-shifted form: K = 16 is
// two taps of 8 channels, the lane half h taking one of them. The taps of
// an MFMA share (dx, dy) and differ in dz: pair 0 holds dz = -1 (h = 0) and
// dz = 0 (h = 1), pair 1 dz = +1 (h = 0) and a zero weight (h = 1). A wave
// loads, per pair, the rows y0-1 .. y0+4 of its two planes at voxels
// x0-1 .. x0+30 (one 16-byte load per lane and row), takes dx = +-1 from
// the neighbouring lanes and dy from the row index, and issues 3 x 3 x 2 x 4
// MFMAs for its 4 x 30 outputs; the next task's rows are loaded while this
// one computes. (The one-row kernel issues one load per MFMA.)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_shift8_kernel(RowK a) {
  constexpr int CIN = 8, R = kConvRows;
  __shared__ bf16x8 wl[kTaps * kCo];  // [tap][co], 8 input channels each
  for (int t = threadIdx.x; t < kTaps * kCo; t += blockDim.x)
    wl[t] = reinterpret_cast<const bf16x8*>(a.w)[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + kShiftVox - 1) / kShiftVox, sy = (a.v.Y + R - 1) / R;
  const float bj = a.bias[m];
  // rows y0-1 .. y0+R of the task's planes for both pairs, at voxel x0-1+m
  // (clamped into the volume, halo included; unconditional loads)
  auto load_task = [&](bf16x8 (&av)[2][R + 2], int seg) {
    const int x0 = (seg % sx) * kShiftVox, y0 = ((seg / sx) % sy) * R, z = seg / (sx * sy);
    const int x = min(x0 - 1 + m, a.v.X);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int zz = p == 0 ? z - 1 + h : z + 1;
#pragma unroll
      for (int k = 0; k < R + 2; ++k)
        av[p][k] = *reinterpret_cast<const bf16x8*>(
            a.src + a.v.vox(x, min(y0 - 1 + k, a.v.Y), zz) * CIN);
    }
  };
  const int stride = gridDim.x * 4;
  int seg = blockIdx.x * 4 + w;
  bf16x8 cur[2][R + 2], nxt[2][R + 2];
  if (seg < a.nseg) load_task(cur, seg);
  for (; seg < a.nseg; seg += stride) {
    if (seg + stride < a.nseg) load_task(nxt, seg + stride);
    __builtin_amdgcn_sched_barrier(0);  // keep those loads ahead of this task's MFMAs
    const int x0 = (seg % sx) * kShiftVox, y0 = ((seg / sx) % sy) * R, z = seg / (sx * sy);
    f32x16 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = f32x16{};
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi) {
        const int dx = dxi - 1;
        bf16x8 rows[R + 2];
#pragma unroll
        for (int k = 0; k < R + 2; ++k) rows[k] = dx == 0 ? cur[p][k] : shift_lanes(cur[p][k], dx);
        bf16x8 bv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          // tap (dx, dy = d - 1, dz): pair 0 dz = h - 1, pair 1 dz = +1 (h = 0 only)
          const int dz = p == 0 ? h - 1 : 1;
          const int t = (dx + 1) + 3 * d + 9 * (dz + 1);
          bv[d] = (p == 1 && h == 1) ? zero8() : wl[t * kCo + m];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int d = 0; d < 3; ++d)
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rows[r + d], bv[d], acc[r], 0, 0, 0);
      }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = y0 + r;
      if (y >= a.v.Y) break;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 8 * (q / 4) + 4 * h + (q % 4);  // lane voxel x0-1+i
        const int x = x0 - 1 + i;
        if (i < 1 || i > kShiftVox || x >= a.v.X) continue;
        float val = acc[r][q] + bj;
        if (a.relu) val = fmaxf(val, 0.0f);
        const int64_t pv = a.v.vox(x, y, z);
        if (a.out) a.out[pv * kCo + m] = (bf16)val;
        if (a.out32 && m == 0) a.out32[pv] = val;
      }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int k = 0; k < R + 2; ++k) cur[p][k] = nxt[p][k];
  }
}

// --------------------------------------------------------------- wgrad

struct WgK {
  Vol v;
  const bf16* in;    // C = CIN
  const bf16* dpre;  // C = 32
  float* part;       // per block: [27][32][CIN] then [32] bias
  int nseg16;        // segments of 16 voxels along x
};

template <int CIN>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(WgK a) {
  __shared__ bf16 dp[16][kCo];
  __shared__ bf16 inr[9][18][CIN];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + 15) / 16;
  f32x16 acc[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q] = f32x16{};
  float dbacc = 0.0f;
  // Operands of one segment, 16-byte chunks spread over the block: dPre
  // (16 voxels x 32 channels, 64 chunks) and the input rows of the 9 (dy, dz)
  // offsets (18 voxels from x0 - 1, CIN channels). The next segment's chunks
  // are loaded into registers while the current segment computes.
  constexpr int ND = 16 * kCo / 8, NI = 9 * 18 * CIN / 8;
  constexpr int QD = (ND + 255) / 256, QI = (NI + 255) / 256;
  bf16x8 pd[QD], pi[QI];
  auto load_seg = [&](int seg) {
    const int x0 = (seg % sx) * 16, y = (seg / sx) % a.v.Y, z = seg / (sx * a.v.Y);
#pragma unroll
    for (int q = 0; q < QD; ++q) {
      const int e = threadIdx.x + q * 256;
      pd[q] = zero8();
      if (e < ND && seg < a.nseg16) {
        const int vx = e / (kCo / 8), c8 = (e % (kCo / 8)) * 8;
        if (x0 + vx < a.v.X)  // voxels past X read as 0
          pd[q] = *reinterpret_cast<const bf16x8*>(a.dpre + a.v.vox(x0 + vx, y, z) * kCo + c8);
      }
    }
#pragma unroll
    for (int q = 0; q < QI; ++q) {
      const int e = threadIdx.x + q * 256;
      pi[q] = zero8();
      if (e < NI && seg < a.nseg16) {
        const int c8 = (e % (CIN / 8)) * 8;
        const int vx = (e / (CIN / 8)) % 18;
        const int row = e / (CIN / 8) / 18;
        const int dy = row % 3 - 1, dz = row / 3 - 1;
        const int x = x0 - 1 + vx;
        if (x <= a.v.X)  // the halo voxel x = X exists (zero)
          pi[q] = *reinterpret_cast<const bf16x8*>(a.in + a.v.vox(x, y + dy, z + dz) * CIN + c8);
      }
    }
  };
  auto store_seg = [&]() {
#pragma unroll
    for (int q = 0; q < QD; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < ND) *reinterpret_cast<bf16x8*>(&dp[e / (kCo / 8)][(e % (kCo / 8)) * 8]) = pd[q];
    }
#pragma unroll
    for (int q = 0; q < QI; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < NI) {
        const int c8 = (e % (CIN / 8)) * 8;
        const int vx = (e / (CIN / 8)) % 18;
        const int row = e / (CIN / 8) / 18;
        *reinterpret_cast<bf16x8*>(&inr[row][vx][c8]) = pi[q];
      }
    }
  };
  load_seg(blockIdx.x);
  for (int seg = blockIdx.x; seg < a.nseg16; seg += gridDim.x) {
    __syncthreads();  // the previous segment's LDS reads are done
    store_seg();
    __syncthreads();
    load_seg(seg + gridDim.x);  // in flight while this segment computes
    bf16x8 av;
#pragma unroll
    for (int e = 0; e < 8; ++e) av[e] = dp[8 * h + e][m];  // A[co = m][voxel]
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int t = w + 4 * q;
      if (t >= kTaps) break;
      int dx, dy, dz;
      tap_offset(t, dx, dy, dz);
      const int row = (dz + 1) * 3 + (dy + 1);
      bf16x8 bv = zero8();
      if (m < CIN) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = inr[row][8 * h + e + 1 + dx][m];  // B[voxel][ci = m]
      }
      acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[q], 0, 0, 0);
    }
    if (w == 0 && h == 0) {
#pragma unroll
      for (int e = 0; e < 16; ++e) dbacc += (float)dp[e][m];
    }
  }
  // block partials: D[i = co][j = ci]
  float* out = a.part + (int64_t)blockIdx.x * (kTaps * kCo * CIN + kCo);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int t = w + 4 * q;
    if (t >= kTaps) break;
    if (m < CIN) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int co = 8 * (r / 4) + 4 * h + (r % 4);
        out[(t * kCo + co) * CIN + m] = acc[q][r];
      }
    }
  }
  if (w == 0 && h == 0) out[kTaps * kCo * CIN + m] = dbacc;
}

// ---------------------------------------------- row-blocked 32-channel wgrad
//
// Weight gradient of a layer with 32 input channels. A block task is 32
// voxels along x on kWgRows consecutive rows y0.. of one z level: K = 128
// voxels, eight MFMA K-steps of 16. The block stages the task's dPre rows and
// the input rows they reach (3 dz x (kWgRows + 2) rows of 34 voxels, from
// x0 - 1) in LDS; the next task's chunks are loaded into registers while the
// current task computes, so one barrier pair serves 7 x 8 MFMAs per wave.
// Taps are split so that a wave owns whole (dy, dz) rows of three dx taps:
// wave w takes rows 2w and 2w + 1 (taps 6w .. 6w + 5) and, for w < 3, tap
// 24 + w of row 8. For a row, lane (ci, h) reads the 10 input voxels
// 16kk + 8h + j (j = 0..9) of its channel once and forms the operands of
// dx = -1, 0, 1 from the windows j = e + dx + 1. A = dPre[16kk + 8h + e][co]
// is read once per K-step and shared by the wave's taps; wave 3 (six taps)
// also multiplies it by a ones column, which sums dPre for the bias.
//
// LDS voxel slots are 64 bytes with 64 bytes of padding after every 8
// voxels: the two lane halves read voxels 8 apart, 576 bytes, i.e. disjoint
// bank ranges. dPre values of voxels past X or rows past Y are stored as
// zero (their loads are clamped into the interior), so the dPre halo is never
// read; input loads are clamped into the input's zero halo.
constexpr int kWgRows = 4;
constexpr int kWgVox = 32;
constexpr int kWgInVox = kWgVox + 2;
__host__ __device__ constexpr int wg_slot(int x) { return 32 * x + 32 * (x >> 3); }
constexpr int kWgDpRow = wg_slot(kWgVox - 1) + 32;    // bf16 elements per dPre row
constexpr int kWgInRow = wg_slot(kWgInVox - 1) + 32;  // per input row
constexpr int kWgInRows = 3 * (kWgRows + 2);
constexpr int kWgDpChunks = kWgRows * kWgVox * 4;         // 16-byte chunks per task
constexpr int kWgInChunks = kWgInRows * kWgInVox * 4;
constexpr int kWgChunks = kWgDpChunks + kWgInChunks;
constexpr int kWgPerThread = (kWgChunks + 255) / 256;
static_assert(kWgDpChunks % 256 == 0, "dPre chunks fill whole load rounds");
constexpr int kWgBlocks = 512;

// Tasks of a block: blocks are dispatched round-robin over the XCDs (8, each
// with its own L2), so XCD k = b % 8 gets the contiguous task range
// [k ntask / 8, (k + 1) ntask / 8), walked by its blocks in stride. The
// blocks of one XCD then work on neighbouring rows and planes at the same
// time and share their halo rows in that XCD's L2.
struct TaskWalk {
  int first, step, end;
};
__device__ __forceinline__ TaskWalk xcd_tasks(int ntask) {
  const int G = min(8, (int)gridDim.x);
  const int k = blockIdx.x % G, slot = blockIdx.x / G;
  const int nk = ((int)gridDim.x - k + G - 1) / G;  // blocks of group k
  return {(int)((int64_t)k * ntask / G) + slot, nk, (int)((int64_t)(k + 1) * ntask / G)};
}

struct WgRowK {
  Vol v;
  const bf16* in;    // C = 32
  const bf16* dpre;  // C = 32
  float* part;       // per block: [27][32][32] then [32] bias
  int ntask;         // (X/32 rounded up) * (Y/kWgRows rounded up) * Z
};

// Two transposing LDS reads (ds_read_b64_tr_b16) giving a lane the 8
// values an MFMA operand needs along K from a channels-last tile (all 64
// lanes must take part: a lane's result comes from other lanes' fetches):
// within each 16-lane group, lane 4a + b receives element b of the 8-byte
// chunks fetched by lanes a, a + 4, a + 8 and a + 12 (checked on the
// device). So
// if lane l fetches channels 16((l/16)%2) + 4((l%16)%4) .. +3 of voxel
// v0 + 8(l/32) + (l%16)/4 (p0) and of the voxel 4 further on (p1), lane
// m + 32h receives channel m of voxels v0 + 8h .. v0 + 8h + 7.
typedef __attribute__((ext_vector_type(4))) short i16x4;
typedef __attribute__((ext_vector_type(8))) short i16x8;
__device__ __forceinline__ bf16x8 lds_tr8(const bf16* p0, const bf16* p1) {
  typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
  const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)const_cast<bf16*>(p0));
  const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)const_cast<bf16*>(p1));
  const i16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}

// kTr: operands through transposing LDS reads (2 per operand) instead of
// one 2-byte read per element (8 for A, 10 per row for B); the same values,
// so the same sums.
template <bool kTr>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_wgrad_rows_kernel(WgRowK a) {
  constexpr int C = 32, R = kWgRows;
  __shared__ __attribute__((aligned(16))) bf16 dp[R * kWgDpRow];
  __shared__ __attribute__((aligned(16))) bf16 inr[kWgInRows * kWgInRow];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + kWgVox - 1) / kWgVox, sy = (a.v.Y + R - 1) / R;
  bf16x8 pre[kWgPerThread];
  auto origin = [&](int t, int& x0, int& y0, int& z) {
    x0 = (t % sx) * kWgVox;
    y0 = ((t / sx) % sy) * R;
    z = t / (sx * sy);
  };
  // Chunk e < kWgDpChunks: dPre row e / 128, voxel (e % 128) / 4, channels
  // 8 (e % 4). Otherwise input row ri = e' / 136 (dz = ri / (R+2) - 1, row
  // y0 - 1 + ri % (R+2)), voxel x0 - 1 + (e' % 136) / 4.
  auto load_task = [&](int t) {
    int x0, y0, z;
    origin(t, x0, y0, z);
#pragma unroll
    for (int q = 0; q < kWgPerThread; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (q * 256 + 255 >= kWgChunks && e >= kWgChunks) continue;
      const int c8 = (e & 3) * 8;
      int64_t p;
      if (q * 256 < kWgDpChunks) {
        const int x = min(x0 + (e % (kWgVox * 4)) / 4, a.v.X - 1);
        const int y = min(y0 + e / (kWgVox * 4), a.v.Y - 1);
        p = a.v.vox(x, y, z) * C + c8;
        pre[q] = *reinterpret_cast<const bf16x8*>(a.dpre + p);
      } else {
        const int f = e - kWgDpChunks, ri = f / (kWgInVox * 4);
        const int x = min(x0 - 1 + (f % (kWgInVox * 4)) / 4, a.v.X);
        const int y = min(y0 - 1 + ri % (R + 2), a.v.Y);
        p = a.v.vox(x, y, z + ri / (R + 2) - 1) * C + c8;
        pre[q] = *reinterpret_cast<const bf16x8*>(a.in + p);
      }
    }
  };
  auto store_task = [&](int t) {
    int x0, y0, z;
    origin(t, x0, y0, z);
#pragma unroll
    for (int q = 0; q < kWgPerThread; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (q * 256 + 255 >= kWgChunks && e >= kWgChunks) continue;
      const int c8 = (e & 3) * 8;
      if (q * 256 < kWgDpChunks) {
        const int r = e / (kWgVox * 4), vx = (e % (kWgVox * 4)) / 4;
        const bool ok = x0 + vx < a.v.X && y0 + r < a.v.Y;
        *reinterpret_cast<bf16x8*>(&dp[r * kWgDpRow + wg_slot(vx) + c8]) = ok ? pre[q] : zero8();
      } else {
        const int f = e - kWgDpChunks, ri = f / (kWgInVox * 4), vx = (f % (kWgInVox * 4)) / 4;
        *reinterpret_cast<bf16x8*>(&inr[ri * kWgInRow + wg_slot(vx) + c8]) = pre[q];
      }
    }
  };
  f32x16 acc[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q] = f32x16{};
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (bf16)1.0f;
  // the wave's full rows (dy, dz) and its single tap of row 8 (dx = w - 1)
  const int rowA = 2 * w, rowB = 2 * w + 1;
  const bool extra = w < 3;
  const TaskWalk tw = xcd_tasks(a.ntask);
  load_task(min(tw.first, a.ntask - 1));
  for (int t = tw.first; t < tw.end; t += tw.step) {
    __syncthreads();  // the previous task's LDS reads are done
    store_task(t);
    __syncthreads();
    load_task(min(t + tw.step, a.ntask - 1));  // in flight while this task computes
#pragma unroll 1
    for (int r = 0; r < R; ++r)
#pragma unroll 1
      for (int kk = 0; kk < 2; ++kk) {
        const int vb = 16 * kk + 8 * h;  // first voxel of the lane's K-slice
        // transposing reads: this lane fetches channels tc .. tc+3 of voxel
        // tv (+ shift) and tv + 4 (+ shift)
        const int tv = 16 * kk + 8 * (lane >> 5) + ((lane & 15) >> 2);
        const int tc = 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
        bf16x8 av;
        if constexpr (kTr) {
          av = lds_tr8(&dp[r * kWgDpRow + wg_slot(tv) + tc], &dp[r * kWgDpRow + wg_slot(tv + 4) + tc]);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) av[e] = dp[r * kWgDpRow + wg_slot(vb + e) + m];
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int row = half ? rowB : rowA;
          const int dz = row / 3 - 1, dy = row % 3 - 1;
          const int rbase = ((dz + 1) * (R + 2) + r + 1 + dy) * kWgInRow;
          const bf16* src = &inr[rbase + m];
          bf16 s[10];
          if constexpr (!kTr) {
#pragma unroll
            for (int j = 0; j < 10; ++j) s[j] = src[wg_slot(vb + j)];
          }
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            bf16x8 bv;
            if constexpr (kTr) {
              bv = lds_tr8(&inr[rbase + wg_slot(tv + d) + tc], &inr[rbase + wg_slot(tv + d + 4) + tc]);
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) bv[e] = s[e + d];
            }
            acc[3 * half + d] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[3 * half + d], 0, 0, 0);
          }
        }
        if (extra) {
          // row 8: dz = dy = +1, dx = w - 1
          const int rbase = (2 * (R + 2) + r + 2) * kWgInRow;
          bf16x8 bv;
          if constexpr (kTr) {
            bv = lds_tr8(&inr[rbase + wg_slot(tv + w) + tc], &inr[rbase + wg_slot(tv + w + 4) + tc]);
          } else {
            const bf16* src = &inr[rbase + m];
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = src[wg_slot(vb + e + w)];
          }
          acc[6] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[6], 0, 0, 0);
        } else {
          // wave 3 (six taps) sums dPre over the voxels: A times a ones column
          acc[6] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, ones, acc[6], 0, 0, 0);
        }
      }
  }
  // block partials: D[i = co][j = ci]
  float* out = a.part + (int64_t)blockIdx.x * (kTaps * kCo * C + kCo);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    if (q == 6 && !extra) break;
    const int t = q < 6 ? 6 * w + q : 24 + w;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = 8 * (r / 4) + 4 * h + (r % 4);
      out[(t * kCo + co) * C + m] = acc[q][r];
    }
  }
  // bias: every column of wave 3's last accumulator holds sum_v dPre[v][co]
  if (!extra && m == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) out[kTaps * kCo * C + 8 * (r / 4) + 4 * h + (r % 4)] = acc[6][r];
  }
}

// ------------------------------------------ row-blocked 8-channel wgrad
//
// Weight gradient of the first layer (8 input channels: the two features
// and six zero channels), staged like the kernel above but with tasks of
// kWg8Rows rows (this layer has a third of the MFMAs per voxel, so a task
// needs more rows to cover the latency of the next task's loads). One
// MFMA covers the three dx taps of a (dy, dz) row: its columns are
// n = 8 (dx + 1) + ci for n < 24, so lane (n, h) reads input voxel
// 16kk + 8h + e + dx + 1 of the row's window, channel ci. Column 24 of row
// 0's MFMA reads ones (the bias: dPre summed over the voxels); the other
// spare columns are never stored, and their lanes read the addresses of
// lanes n - 24 (same-address reads share a bank access). Wave w takes dPre
// rows w, w + 4, ... of the task and all nine (dy, dz) rows (nine
// accumulators); the four waves' sums are added through LDS in wave order
// at the end.
__host__ __device__ constexpr int wg8_slot(int x) { return 8 * x + 32 * (x >> 3); }
constexpr int kWg8Rows = 8;
constexpr int kWg8InRows = 3 * (kWg8Rows + 2);
constexpr int kWg8InRow = wg8_slot(kWgInVox - 1) + 8;
constexpr int kWg8DpChunks = kWg8Rows * kWgVox * 4;
constexpr int kWg8InChunks = kWg8InRows * kWgInVox;  // one 16-byte chunk per voxel
constexpr int kWg8Chunks = kWg8DpChunks + kWg8InChunks;
constexpr int kWg8PerThread = (kWg8Chunks + 255) / 256;
static_assert(kWg8DpChunks % 256 == 0 && kWg8Rows % 4 == 0, "whole load rounds and row sets");

// kTr: operands through transposing LDS reads (as in the 32-channel
// kernel); lane (n, h) of B receives channel n & 7 of voxels shifted by
// dx + 1 = n >> 3, the ones column (n = 24 of row 0) from the ones slot, the
// other spare columns from dx + 1 = 0. The same values in every stored
// column, so the same sums.
template <bool kTr>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_wgrad_rows8_kernel(WgRowK a) {
  constexpr int C = 8, R = kWg8Rows;
  __shared__ __attribute__((aligned(16))) bf16 dp[R * kWgDpRow];
  __shared__ __attribute__((aligned(16))) bf16 inr[kWg8InRows * kWg8InRow + 8];
  __shared__ float red[9 * 32 * 32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int sx = (a.v.X + kWgVox - 1) / kWgVox, sy = (a.v.Y + R - 1) / R;
  constexpr int kOnes = kWg8InRows * kWg8InRow;
  if (threadIdx.x < 8) inr[kOnes + threadIdx.x] = (bf16)1.0f;
  bf16x8 pre[kWg8PerThread];
  auto origin = [&](int t, int& x0, int& y0, int& z) {
    x0 = (t % sx) * kWgVox;
    y0 = ((t / sx) % sy) * R;
    z = t / (sx * sy);
  };
  // chunk e < kWg8DpChunks: dPre as in the 32-channel kernel; otherwise
  // input row ri = e' / 34, voxel x0 - 1 + e' % 34 (all 8 channels)
  auto load_task = [&](int t) {
    int x0, y0, z;
    origin(t, x0, y0, z);
#pragma unroll
    for (int q = 0; q < kWg8PerThread; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (q * 256 + 255 >= kWg8Chunks && e >= kWg8Chunks) continue;
      if (q * 256 < kWg8DpChunks) {
        const int x = min(x0 + (e % (kWgVox * 4)) / 4, a.v.X - 1);
        const int y = min(y0 + e / (kWgVox * 4), a.v.Y - 1);
        pre[q] = *reinterpret_cast<const bf16x8*>(a.dpre + a.v.vox(x, y, z) * kCo + (e & 3) * 8);
      } else {
        const int f = e - kWg8DpChunks, ri = f / kWgInVox;
        const int x = min(x0 - 1 + f % kWgInVox, a.v.X);
        const int y = min(y0 - 1 + ri % (R + 2), a.v.Y);
        pre[q] = *reinterpret_cast<const bf16x8*>(a.in + a.v.vox(x, y, z + ri / (R + 2) - 1) * C);
      }
    }
  };
  auto store_task = [&](int t) {
    int x0, y0, z;
    origin(t, x0, y0, z);
#pragma unroll
    for (int q = 0; q < kWg8PerThread; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (q * 256 + 255 >= kWg8Chunks && e >= kWg8Chunks) continue;
      if (q * 256 < kWg8DpChunks) {
        const int r = e / (kWgVox * 4), vx = (e % (kWgVox * 4)) / 4;
        const bool ok = x0 + vx < a.v.X && y0 + r < a.v.Y;
        *reinterpret_cast<bf16x8*>(&dp[r * kWgDpRow + wg_slot(vx) + (e & 3) * 8]) =
            ok ? pre[q] : zero8();
      } else {
        const int f = e - kWg8DpChunks;
        *reinterpret_cast<bf16x8*>(&inr[(f / kWgInVox) * kWg8InRow + wg8_slot(f % kWgInVox)]) =
            pre[q];
      }
    }
  };
  f32x16 acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = f32x16{};
  // column n = m < 24: tap dx = dx1 - 1, channel ci; spare columns alias n - 24
  const int dx1 = m < 24 ? m >> 3 : 0, ci = m & 7;
  const TaskWalk tw = xcd_tasks(a.ntask);
  load_task(min(tw.first, a.ntask - 1));
  for (int t = tw.first; t < tw.end; t += tw.step) {
    __syncthreads();  // the previous task's LDS reads are done
    store_task(t);
    __syncthreads();
    load_task(min(t + tw.step, a.ntask - 1));  // in flight while this task computes
#pragma unroll 1
    for (int rk = 0; rk < 2 * R / 4; ++rk) {
      const int r = w + 4 * (rk >> 1);        // the wave's dPre row
      const int vb = 16 * (rk & 1) + 8 * h;  // first voxel of the lane's K-slice
      // transposing reads (see lds_tr8): voxel tv (+ 4), channels tc (A) or
      // 4 (ta & 1) at shift tdx1 (B)
      const int tv = 16 * (rk & 1) + 8 * (lane >> 5) + ((lane & 15) >> 2);
      const int tc = 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
      const int ta = lane & 3, todd = (lane >> 4) & 1;
      const int tdx1 = todd ? (ta >= 2 ? 0 : 2) : (ta >> 1);
      const bool tones = todd && ta == 2;
      bf16x8 av;
      if constexpr (kTr) {
        av = lds_tr8(&dp[r * kWgDpRow + wg_slot(tv) + tc], &dp[r * kWgDpRow + wg_slot(tv + 4) + tc]);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = dp[r * kWgDpRow + wg_slot(vb + e) + m];
      }
#pragma unroll
      for (int row = 0; row < 9; ++row) {
        const int dz = row / 3 - 1, dy = row % 3 - 1;
        const int ri = (dz + 1) * (R + 2) + r + 1 + dy;
        bf16x8 bv;
        if constexpr (kTr) {
          // one read for every lane (a transposing read takes its values from
          // the other lanes of its group, so it must not run under a branch):
          // the ones lanes select their address instead
          const int rb = ri * kWg8InRow + 4 * (ta & 1);
          const bool one = row == 0 && tones;
          const int q0 = one ? kOnes : rb + wg8_slot(tv + tdx1);
          const int q1 = one ? kOnes + 4 : rb + wg8_slot(tv + tdx1 + 4);
          bv = lds_tr8(&inr[q0], &inr[q1]);
        } else {
          const bool ones = row == 0 && m == 24;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            bv[e] = inr[ones ? kOnes : ri * kWg8InRow + wg8_slot(vb + e + dx1) + ci];
        }
        acc[row] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[row], 0, 0, 0);
      }
    }
  }
  // the four waves' sums, added in wave order: red[row][co][n]
#pragma unroll 1
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int row = 0; row < 9; ++row)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int co = 8 * (r / 4) + 4 * h + (r % 4);
          float& d = red[(row * 32 + co) * 32 + m];
          d = ww == 0 ? acc[row][r] : d + acc[row][r];
        }
    }
    __syncthreads();
  }
  float* out = a.part + (int64_t)blockIdx.x * (kTaps * kCo * C + kCo);
  for (int i = threadIdx.x; i < 9 * 32 * 32; i += blockDim.x) {
    const int row = i >> 10, co = (i >> 5) & 31, n = i & 31;
    if (n < 24) out[((3 * row + (n >> 3)) * kCo + co) * C + (n & 7)] = red[i];
    else if (n == 24 && row == 0) out[kTaps * kCo * C + co] = red[i];
  }
}

// Sums block partials: dw[27*32*CIN], db[32]. Eight interleaved running
// sums (block b goes to sum b % 8) keep eight loads in flight per thread;
// they are combined in a fixed order, so the result does not depend on the
// launch.
__global__ void wgrad_reduce_kernel(const float* part, int nblocks, int n, float* dw, float* db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n + kCo) return;
  const int64_t stride = n + kCo;
  float s[8] = {};
  int b = 0;
  for (; b + 8 <= nblocks; b += 8)
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += part[(int64_t)(b + e) * stride + i];
  for (int e = 0; b < nblocks; ++b, ++e) s[e] += part[(int64_t)b * stride + i];
  const float t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  if (i < n) dw[i] = t;
  else db[i - n] = t;
}

// First pass of the row-blocked kernels' reduction: slice y of the grid
// sums block partials [y per, (y + 1) per) in the order above into
// slices[y]; wgrad_reduce_kernel then sums the slices (as if they were
// blocks). Sixteen slices give the reduction sixteen times the parallelism
// of one pass over the blocks.
constexpr int kWgSlices = 16;

__global__ void wgrad_slice_kernel(const float* part, int nblocks, int n, int per,
                                   float* slices) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n + kCo) return;
  const int64_t stride = n + kCo;
  const int b0 = blockIdx.y * per, b1 = min(nblocks, b0 + per);
  float s[8] = {};
  int b = b0;
  for (; b + 8 <= b1; b += 8)
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += part[(int64_t)(b + e) * stride + i];
  for (int e = 0; b < b1; ++b, ++e) s[e] += part[(int64_t)b * stride + i];
  slices[blockIdx.y * stride + i] =
      ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// ------------------------------------------------- loss, Adam, features

// loss partials and dPre of the last layer: d = 2 (pred - target) / N in
// channel 0 (BF16), channels 1..31 zero. Interior voxels only.
__global__ __launch_bounds__(256) void mse_kernel(Vol v, const float* pred, const float* target,
                                                  double inv_n, bf16* dpre, double* part) {
  __shared__ double red[kWavesY];
  double acc = 0.0;
  const int64_t n = (int64_t)v.X * v.Y * v.Z;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(t % v.X), y = (int)((t / v.X) % v.Y), z = (int)(t / ((int64_t)v.X * v.Y));
    const int64_t p = v.vox(x, y, z);
    const double d = (double)pred[p] - (double)target[p];
    acc += d * d;
    dpre[p * kCo] = (bf16)(float)(2.0 * d * inv_n);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Adam on FP32 master weights; writes both BF16 layouts.
struct AdamK {
  float* w;       // [27][32][cin] master
  float* b;       // [32]
  float* mw;
  float* vw;
  float* mb;
  float* vb;
  const float* gw;
  const float* gb;
  bf16* wf;       // [27][32][cin]
  bf16* wd;       // [27][cin][32]
  int cin;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__global__ void adam_kernel(AdamK a) {
  const int n = kTaps * kCo * a.cin;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float g = a.gw[i];
    const float mm = a.b1 * a.mw[i] + (1.0f - a.b1) * g;
    const float vv = a.b2 * a.vw[i] + (1.0f - a.b2) * g * g;
    a.mw[i] = mm;
    a.vw[i] = vv;
    const float wv = a.w[i] - a.lr * (mm / a.c1) / (sqrtf(vv / a.c2) + a.eps);
    a.w[i] = wv;
    const int t = i / (kCo * a.cin), co = (i / a.cin) % kCo, ci = i % a.cin;
    a.wf[i] = (bf16)wv;
    a.wd[(t * a.cin + ci) * kCo + co] = (bf16)wv;
  } else if (i < n + kCo) {
    const int j = i - n;
    const float g = a.gb[j];
    const float mm = a.b1 * a.mb[j] + (1.0f - a.b1) * g;
    const float vv = a.b2 * a.vb[j] + (1.0f - a.b2) * g * g;
    a.mb[j] = mm;
    a.vb[j] = vv;
    a.b[j] = a.b[j] - a.lr * (mm / a.c1) / (sqrtf(vv / a.c2) + a.eps);
  }
}

// BF16 copies of FP32 master weights in both layouts (initialisation).
__global__ void pack_weights_kernel(const float* w, int cin, bf16* wf, bf16* wd) {
  const int n = kTaps * kCo * cin;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = i / (kCo * cin), co = (i / cin) % kCo, ci = i % cin;
  wf[i] = (bf16)w[i];
  wd[(t * cin + ci) * kCo + co] = (bf16)w[i];
}

// max(|f|, |g|) partials over the interior; g = sum of Dirichlet neighbours.
__device__ __forceinline__ double lift(const double* u, const ms_grid& g, int i, int j, int k) {
  const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
  double s = 0.0;
  if (i == g.nx - 1) s += u[p + 1];
  if (i == 0) s += u[p - 1];
  if (j == g.ny - 1) s += u[p + g.sy];
  if (j == 0) s += u[p - g.sy];
  if (k == g.nz - 1) s += u[p + g.sz];
  if (k == 0) s += u[p - g.sz];
  return s;
}

__global__ __launch_bounds__(256) void feat_max_kernel(ms_grid g, const double* u,
                                                       const double* f, double* part) {
  __shared__ double red[kWavesY];
  double mx = 0.0;
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    mx = fmax(mx, fabs(lift(u, g, i, j, k)));
    if (f) mx = fmax(mx, fabs(f[p]));
  }
  // block max (order-independent)
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    part[blockIdx.x] = r;
  }
}

// One block of 256 threads: the max over the block partials (max is exact
// and order-independent).
__global__ __launch_bounds__(256) void feat_scale_kernel(const double* part, int nb,
                                                         double* scale) {
  __shared__ double red[kWavesY];
  double r = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) r = fmax(r, part[b]);
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_down(r, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    *scale = m > 0.0 ? m : 1.0;
  }
}

// Feature channels (BF16, 8 per voxel): 0 f/s, 1 g/s, 2..5 cube means of
// f/s of half-widths kBoxHalf[0..3], 6 the slowest Jacobi mode
// phi = prod sin(pi (i+1)/(n+1)), 7 the cube mean of half-width kBoxHalf[4].
constexpr int kBoxHalf[5] = {2, 5, 11, 23, 47};
constexpr int kBoxChannel[5] = {2, 3, 4, 5, 7};

__device__ __forceinline__ double mode_factor(int i, int n) {
  return sin((M_PI * (double)(i + 1)) / (double)(n + 1));
}

// Channels 0, 1 and 6 (the cube means are written by box_z_kernel).
__global__ void feat_write_kernel(ms_grid g, const double* u, const double* f,
                                  const double* scale, Vol v, bf16* feat) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const double s = *scale;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    bf16x8 val = zero8();
    val[0] = (bf16)(float)((f ? f[p] : 0.0) / s);
    val[1] = (bf16)(float)(lift(u, g, i, j, k) / s);
    const double phi = (mode_factor(k, g.nz) * mode_factor(j, g.ny)) * mode_factor(i, g.nx);
    val[6] = (bf16)(float)phi;
    *reinterpret_cast<bf16x8*>(feat + v.vox(i, j, k) * 8) = val;
  }
}

// Separable cube sums of f/s over the interior (zero outside), each pass a
// sum over offsets -h .. h in increasing order. x pass: from the field f;
// y pass: between dense interior volumes t[(k * ny + j) * nx + i]; z pass:
// divides by the cube's volume and writes one feature channel.
__global__ void box_x_kernel(ms_grid g, const double* f, const double* scale, int h,
                             double* out) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const double s = *scale;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    double acc = 0.0;
    if (f) {
      const int lo = max(-h, -i), hi = min(h, g.nx - 1 - i);
      for (int d = lo; d <= hi; ++d) acc = acc + f[p + d] / s;
    }
    out[t] = acc;
  }
}

__global__ void box_y_kernel(int nx, int ny, int nz, int h, const double* in, double* out) {
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)((t / nx) % ny);
    const int lo = max(-h, -j), hi = min(h, ny - 1 - j);
    double acc = 0.0;
    for (int d = lo; d <= hi; ++d) acc = acc + in[t + (int64_t)d * nx];
    out[t] = acc;
  }
}

__global__ void box_z_kernel(int nx, int ny, int nz, int h, const double* in, Vol v, int ch,
                             bf16* feat) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t pl = (int64_t)nx * ny;
  const double vol = (double)((2 * h + 1) * (2 * h + 1) * (2 * h + 1));
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / pl);
    const int lo = max(-h, -k), hi = min(h, nz - 1 - k);
    double acc = 0.0;
    for (int d = lo; d <= hi; ++d) acc = acc + in[t + (int64_t)d * pl];
    feat[v.vox(i, j, k) * 8 + ch] = (bf16)(float)(acc / vol);
  }
}

// Box sums through LDS: a block stages the lines it sums along (the x
// kernel dividing by the scale once per element instead of once per use),
// then each output adds its window from LDS in increasing offset -- the
// same additions in the same order as the kernels above, which stay for
// lines longer than kBoxLds.
constexpr int kBoxLds = 8192;  // doubles of LDS per block (64 KiB)

// x: T = max(1, 256 / nx) rows of x per round.
__global__ __launch_bounds__(256) void box_x_lds_kernel(ms_grid g, const double* f,
                                                        const double* scale, int h,
                                                        double* out) {
  extern __shared__ double lds_line[];
  const int nx = g.nx, T = max(1, 256 / nx);
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const double s = *scale;
  for (int64_t r0 = (int64_t)blockIdx.x * T; r0 < nrows; r0 += (int64_t)gridDim.x * T) {
    const int rows = (int)min((int64_t)T, nrows - r0);
    __syncthreads();  // the previous round's reads are done
    for (int e = threadIdx.x; e < rows * nx; e += blockDim.x) {
      const int64_t row = r0 + e / nx;
      const int i = e % nx, j = (int)(row % g.ny), k = (int)(row / g.ny);
      lds_line[e] = f ? f[(int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1)] / s : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * nx; e += blockDim.x) {
      const int rr = e / nx, i = e % nx;
      const int lo = max(-h, -i), hi = min(h, nx - 1 - i);
      double acc = 0.0;
      if (f)
        for (int d = lo; d <= hi; ++d) acc = acc + lds_line[rr * nx + i + d];
      out[(r0 + rr) * nx + i] = acc;
    }
  }
}

// y (kZ false: out) or z (kZ true: the feature channel): tiles of W
// consecutive x by the whole line, at one position of the third axis.
template <bool kZ>
__global__ __launch_bounds__(256) void box_line_lds_kernel(int nx, int ny, int nz, int h, int W,
                                                           const double* in, double* out, Vol v,
                                                           int ch, bf16* feat) {
  extern __shared__ double lds_line[];
  const int n = kZ ? nz : ny;
  const int64_t S = kZ ? (int64_t)nx * ny : nx;  // stride along the line
  const int other = kZ ? ny : nz;
  const int cx = (nx + W - 1) / W;
  const int64_t ntiles = (int64_t)cx * other;
  const double vol = (double)((2 * h + 1) * (2 * h + 1) * (2 * h + 1));
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (int)(tile % cx) * W, o = (int)(tile / cx);
    const int w = min(W, nx - x0);
    // element (x0, 0, o) for y lines, (x0, o, 0) for z lines
    const int64_t base = kZ ? (int64_t)o * nx + x0 : (int64_t)o * nx * ny + x0;
    __syncthreads();
    for (int e = threadIdx.x; e < n * W; e += blockDim.x) {
      const int q = e / W, x = e % W;
      lds_line[e] = x < w ? in[base + q * S + x] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * W; e += blockDim.x) {
      const int q = e / W, x = e % W;
      if (x >= w) continue;
      const int lo = max(-h, -q), hi = min(h, n - 1 - q);
      double acc = 0.0;
      for (int d = lo; d <= hi; ++d) acc = acc + lds_line[(q + d) * W + x];
      if constexpr (kZ)
        feat[v.vox(x0 + x, o, q) * 8 + ch] = (bf16)(float)(acc / vol);
      else
        out[base + q * S + x] = acc;
    }
  }
}

// guess: x interior = s * lambda * uhat (FP64), halo untouched.
__global__ void guess_kernel(ms_grid g, const float* uhat, Vol v, const double* scale,
                             double lambda, double* x) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const double s = *scale * lambda;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    x[p] = s * (double)uhat[v.vox(i, j, k)];
  }
}

// target: uhat = u / (s * lambda) in FP32 on the interior (training data).
__global__ void target_kernel(ms_grid g, const double* u, Vol v, const double* scale,
                              double lambda, float* out) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const double s = *scale * lambda;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    out[v.vox(i, j, k)] = (float)(u[p] / s);
  }
}

constexpr int conv_grid_blocks() { return 1024; }

// 32-channel layers use the row-blocked kernels; MS_CONV_ROWS=0 selects the
// one-row kernels instead (a cross-check).
bool row_blocked() {
  const char* e = getenv("MS_CONV_ROWS");
  return !(e && atoi(e) == 0);
}

bool cin_ok(int cin) { return cin == 8 || cin == 32; }

// Weight gradients: operands through transposing LDS reads; MS_WGRAD_TR=0
// keeps the element-wise reads (the same values).
bool wgrad_tr() {
  const char* e = getenv("MS_WGRAD_TR");
  return !(e && atoi(e) == 0);
}

// Lane-shifted kernels for the 32-channel layers and the 8-channel forward;
// MS_CONV_SHIFT=0 keeps the row-blocked 32-channel kernels (the same sums
// bit for bit) and the one-row 8-channel forward (the same products, summed
// in another order).
bool conv_shift() {
  const char* e = getenv("MS_CONV_SHIFT");
  return !(e && atoi(e) == 0);
}

}  // namespace
}  // namespace ms

using namespace ms;

// ------------------------------------------------------------- C ABI

extern "C" int conv3d_bf16_fwd(int X, int Y, int Z, int cin, const void* in, const void* w,
                               const float* bias, void* out, float* out32, int relu,
                               void* stream) {
  clear_error();
  if (X < 1 || Y < 1 || Z < 1 || !cin_ok(cin) || !in || !w || !bias || (!out && !out32))
    return set_error(MS_EINVAL, "conv3d_bf16_fwd: bad arguments");
  FwdK a{{X, Y, Z}, static_cast<const bf16*>(in), static_cast<const bf16*>(w), bias,
         static_cast<bf16*>(out), out32, relu, ((X + 31) / 32) * Y * Z};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cin == 8 && conv_shift()) {
    const RowK r{{X, Y, Z}, static_cast<const bf16*>(in), static_cast<const bf16*>(w), bias,
                 static_cast<bf16*>(out), out32, nullptr, nullptr, relu,
                 ((X + kShiftVox - 1) / kShiftVox) * ((Y + kConvRows - 1) / kConvRows) * Z};
    hipLaunchKernelGGL(conv_shift8_kernel, dim3(conv_grid_blocks()), dim3(256), 0, s, r);
  } else if (cin == 8) {
    hipLaunchKernelGGL(conv_fwd_kernel<8>, dim3(conv_grid_blocks()), dim3(256), 0, s, a);
  } else if (row_blocked()) {
    RowK r{{X, Y, Z}, static_cast<const bf16*>(in), static_cast<const bf16*>(w), bias,
           static_cast<bf16*>(out), out32, nullptr, nullptr, relu,
           ((X + 31) / 32) * ((Y + kConvRows - 1) / kConvRows) * Z};
    if (conv_shift()) {
      r.nseg = ((X + kShiftVox - 1) / kShiftVox) * ((Y + kConvRows - 1) / kConvRows) * Z;
      hipLaunchKernelGGL(conv_shift_kernel<false>, dim3(conv_grid_blocks()), dim3(256), 0, s, r);
    } else {
      hipLaunchKernelGGL(conv_rows_kernel<false>, dim3(conv_grid_blocks()), dim3(256), 0, s, r);
    }
  } else {
    hipLaunchKernelGGL(conv_fwd_kernel<32>, dim3(conv_grid_blocks()), dim3(256), 0, s, a);
  }
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int conv3d_bf16_dgrad(int X, int Y, int Z, int cin, const void* dout, const void* wd,
                                 const void* mask, void* din, void* stream) {
  clear_error();
  if (X < 1 || Y < 1 || Z < 1 || !cin_ok(cin) || !dout || !wd || !din)
    return set_error(MS_EINVAL, "conv3d_bf16_dgrad: bad arguments");
  DgK a{{X, Y, Z}, static_cast<const bf16*>(dout), static_cast<const bf16*>(wd),
        static_cast<const bf16*>(mask), static_cast<bf16*>(din), ((X + 31) / 32) * Y * Z};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cin == 8) {
    hipLaunchKernelGGL(conv_dgrad_kernel<8>, dim3(conv_grid_blocks()), dim3(256), 0, s, a);
  } else if (row_blocked()) {
    RowK r{{X, Y, Z}, static_cast<const bf16*>(dout), static_cast<const bf16*>(wd),
           nullptr, nullptr, nullptr, static_cast<const bf16*>(mask),
           static_cast<bf16*>(din), 0,
           ((X + 31) / 32) * ((Y + kConvRows - 1) / kConvRows) * Z};
    if (conv_shift()) {
      r.nseg = ((X + kShiftVox - 1) / kShiftVox) * ((Y + kConvRows - 1) / kConvRows) * Z;
      hipLaunchKernelGGL(conv_shift_kernel<true>, dim3(conv_grid_blocks()), dim3(256), 0, s, r);
    } else {
      hipLaunchKernelGGL(conv_rows_kernel<true>, dim3(conv_grid_blocks()), dim3(256), 0, s, r);
    }
  } else {
    hipLaunchKernelGGL(conv_dgrad_kernel<32>, dim3(conv_grid_blocks()), dim3(256), 0, s, a);
  }
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" size_t conv3d_bf16_wgrad_workspace_bytes(int cin) {
  if (!cin_ok(cin)) return 0;
  return (size_t)conv_grid_blocks() * (kTaps * kCo * cin + kCo) * sizeof(float);
}

extern "C" int conv3d_bf16_wgrad(int X, int Y, int Z, int cin, const void* in, const void* dpre,
                                 float* dw, float* db, void* work, size_t work_bytes,
                                 void* stream) {
  clear_error();
  if (X < 1 || Y < 1 || Z < 1 || !cin_ok(cin) || !in || !dpre || !dw || !db)
    return set_error(MS_EINVAL, "conv3d_bf16_wgrad: bad arguments");
  const size_t need = conv3d_bf16_wgrad_workspace_bytes(cin);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "conv3d_bf16_wgrad: workspace needs %zu bytes", need);
  WgK a{{X, Y, Z}, static_cast<const bf16*>(in), static_cast<const bf16*>(dpre),
        static_cast<float*>(work), ((X + 15) / 16) * Y * Z};
  hipStream_t s = static_cast<hipStream_t>(stream);
  int nb = conv_grid_blocks();
  if (row_blocked()) {
    const int rows = cin == 8 ? kWg8Rows : kWgRows;
    const int ntask = ((X + kWgVox - 1) / kWgVox) * ((Y + rows - 1) / rows) * Z;
    nb = std::min(kWgBlocks, ntask);
    const WgRowK r{{X, Y, Z}, static_cast<const bf16*>(in), static_cast<const bf16*>(dpre),
                   static_cast<float*>(work), ntask};
    if (cin == 8)
      if (wgrad_tr())
        hipLaunchKernelGGL(conv_wgrad_rows8_kernel<true>, dim3(nb), dim3(256), 0, s, r);
      else
        hipLaunchKernelGGL(conv_wgrad_rows8_kernel<false>, dim3(nb), dim3(256), 0, s, r);
    else
      if (wgrad_tr())
        hipLaunchKernelGGL(conv_wgrad_rows_kernel<true>, dim3(nb), dim3(256), 0, s, r);
      else
        hipLaunchKernelGGL(conv_wgrad_rows_kernel<false>, dim3(nb), dim3(256), 0, s, r);
  } else if (cin == 8) {
    hipLaunchKernelGGL(conv_wgrad_kernel<8>, dim3(nb), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(conv_wgrad_kernel<32>, dim3(nb), dim3(256), 0, s, a);
  }
  MS_LAUNCH_CHECK();
  const int n = kTaps * kCo * cin;
  const int64_t stride = n + kCo;
  const dim3 rgrid((unsigned)((stride + 255) / 256));
  if (row_blocked()) {
    // the row-blocked kernels use at most kWgBlocks of the workspace's
    // conv_grid_blocks() partial slots; the slices go after them
    static_assert(kWgBlocks + kWgSlices <= conv_grid_blocks(), "slices fit the workspace");
    float* slices = static_cast<float*>(work) + (int64_t)nb * stride;
    hipLaunchKernelGGL(wgrad_slice_kernel, dim3(rgrid.x, kWgSlices), dim3(256), 0, s,
                       static_cast<const float*>(work), nb, n, (nb + kWgSlices - 1) / kWgSlices,
                       slices);
    MS_LAUNCH_CHECK();
    hipLaunchKernelGGL(wgrad_reduce_kernel, rgrid, dim3(256), 0, s, slices, kWgSlices, n, dw, db);
  } else {
    hipLaunchKernelGGL(wgrad_reduce_kernel, rgrid, dim3(256), 0, s,
                       static_cast<const float*>(work), nb, n, dw, db);
  }
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int cnn_mse_grad(int X, int Y, int Z, const float* pred, const float* target,
                            void* dpre, double* loss_part, int nparts, void* stream) {
  clear_error();
  if (X < 1 || Y < 1 || Z < 1 || !pred || !target || !dpre || !loss_part || nparts < 1)
    return set_error(MS_EINVAL, "cnn_mse_grad: bad arguments");
  const double inv_n = 1.0 / ((double)X * Y * Z);
  hipLaunchKernelGGL(mse_kernel, dim3(nparts), dim3(256), 0, static_cast<hipStream_t>(stream),
                     Vol{X, Y, Z}, pred, target, inv_n, static_cast<bf16*>(dpre), loss_part);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int cnn_adam(int cin, float* w, float* b, float* mw, float* vw, float* mb, float* vb,
                        const float* gw, const float* gb, void* wf, void* wd, float lr, int t,
                        void* stream) {
  clear_error();
  if (!cin_ok(cin) || t < 1) return set_error(MS_EINVAL, "cnn_adam: bad arguments");
  AdamK a{w, b, mw, vw, mb, vb, gw, gb, static_cast<bf16*>(wf), static_cast<bf16*>(wd), cin,
          lr, 0.9f, 0.999f, 1e-8f, 1.0f - powf(0.9f, (float)t), 1.0f - powf(0.999f, (float)t)};
  const int n = kTaps * kCo * cin + kCo;
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int cnn_pack_weights(int cin, const float* w, void* wf, void* wd, void* stream) {
  clear_error();
  if (!cin_ok(cin) || !w || !wf || !wd) return set_error(MS_EINVAL, "cnn_pack_weights");
  const int n = kTaps * kCo * cin;
  hipLaunchKernelGGL(pack_weights_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w, cin, static_cast<bf16*>(wf),
                     static_cast<bf16*>(wd));
  MS_LAUNCH_CHECK();
  return MS_OK;
}

namespace ms {
namespace {
constexpr int kFeatParts = 1024;
}  // namespace
}  // namespace ms

extern "C" size_t cnn_features_workspace_bytes(const ms_grid* g) {
  if (check_grid(g, "cnn_features_workspace_bytes")) return 0;
  const size_t vol = (size_t)g->nx * g->ny * g->nz * sizeof(double);
  return align_up(kFeatParts * sizeof(double), 256) + 2 * align_up(vol, 256);
}

extern "C" int cnn_features(const ms_grid* g, const double* u, const double* f, void* feat,
                            double* scale, void* work, size_t work_bytes, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "cnn_features")) return rc;
  if (!u || !feat || !scale) return set_error(MS_EINVAL, "cnn_features: bad arguments");
  const size_t need = cnn_features_workspace_bytes(g);
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "cnn_features: workspace needs %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws{static_cast<char*>(work), work_bytes};
  double* part = ws.take<double>(kFeatParts);
  const size_t nvox = (size_t)g->nx * g->ny * g->nz;
  double* t1 = ws.take<double>(nvox);
  double* t2 = ws.take<double>(nvox);
  const Vol v{g->nx, g->ny, g->nz};
  bf16* fb = static_cast<bf16*>(feat);
  hipLaunchKernelGGL(feat_max_kernel, dim3(kFeatParts), dim3(256), 0, s, *g, u, f, part);
  MS_LAUNCH_CHECK();
  hipLaunchKernelGGL(feat_scale_kernel, dim3(1), dim3(256), 0, s, part, kFeatParts, scale);
  MS_LAUNCH_CHECK();
  hipLaunchKernelGGL(feat_write_kernel, dim3(1024), dim3(256), 0, s, *g, u, f, scale, v, fb);
  MS_LAUNCH_CHECK();
  // LDS forms where a line fits (MS_BOX_LDS=0: the global-memory forms)
  const char* ev = getenv("MS_BOX_LDS");
  const bool lds = !(ev && atoi(ev) == 0);
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  // tiles of at most 16 x by 2048 doubles: many small blocks, since each
  // output's sum is a chain of dependent adds and latency wants many waves
  const int wy = std::max(1, std::min(16, 2048 / ny)), wz = std::max(1, std::min(16, 2048 / nz));
  const int64_t ty = (int64_t)((nx + wy - 1) / wy) * nz, tz = (int64_t)((nx + wz - 1) / wz) * ny;
  for (int b = 0; b < 5; ++b) {
    const int h = kBoxHalf[b];
    if (lds && nx <= kBoxLds) {
      const size_t bytes = (size_t)std::max(256, nx) * sizeof(double);
      hipLaunchKernelGGL(box_x_lds_kernel, dim3(2048), dim3(256), bytes, s, *g, f, scale, h, t1);
    } else {
      hipLaunchKernelGGL(box_x_kernel, dim3(2048), dim3(256), 0, s, *g, f, scale, h, t1);
    }
    MS_LAUNCH_CHECK();
    if (lds && ny <= kBoxLds) {
      hipLaunchKernelGGL(box_line_lds_kernel<false>, dim3((unsigned)std::min<int64_t>(ty, 2048)),
                         dim3(256), (size_t)ny * wy * sizeof(double), s, nx, ny, nz, h, wy, t1,
                         t2, v, 0, fb);
    } else {
      hipLaunchKernelGGL(box_y_kernel, dim3(2048), dim3(256), 0, s, nx, ny, nz, h, t1, t2);
    }
    MS_LAUNCH_CHECK();
    if (lds && nz <= kBoxLds) {
      hipLaunchKernelGGL(box_line_lds_kernel<true>, dim3((unsigned)std::min<int64_t>(tz, 2048)),
                         dim3(256), (size_t)nz * wz * sizeof(double), s, nx, ny, nz, h, wz, t2,
                         nullptr, v, kBoxChannel[b], fb);
    } else {
      hipLaunchKernelGGL(box_z_kernel, dim3(2048), dim3(256), 0, s, nx, ny, nz, h, t2, v,
                         kBoxChannel[b], fb);
    }
    MS_LAUNCH_CHECK();
  }
  return MS_OK;
}

extern "C" int cnn_guess(const ms_grid* g, const float* uhat, const double* scale, double lambda,
                         double* x, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "cnn_guess")) return rc;
  if (!uhat || !scale || !x) return set_error(MS_EINVAL, "cnn_guess: bad arguments");
  hipLaunchKernelGGL(guess_kernel, dim3(1024), dim3(256), 0, static_cast<hipStream_t>(stream),
                     *g, uhat, Vol{g->nx, g->ny, g->nz}, scale, lambda, x);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int cnn_target(const ms_grid* g, const double* u, const double* scale, double lambda,
                          float* out, void* stream) {
  clear_error();
  if (int rc = check_grid(g, "cnn_target")) return rc;
  if (!u || !scale || !out) return set_error(MS_EINVAL, "cnn_target: bad arguments");
  hipLaunchKernelGGL(target_kernel, dim3(1024), dim3(256), 0, static_cast<hipStream_t>(stream),
                     *g, u, Vol{g->nx, g->ny, g->nz}, scale, lambda, out);
  MS_LAUNCH_CHECK();
  return MS_OK;
}
