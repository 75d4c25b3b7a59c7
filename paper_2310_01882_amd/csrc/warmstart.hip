// The learned warm start behind two calls.
//
// warmstart_forward: features of the Poisson problem, the four 3x3x3
// convolutions (BF16 MFMA, FP32 accumulation), the guess x = s * lambda *
// u_hat, a few damped Jacobi sweeps on it, then the start selection: the
// residuals of the guess and of u0 (u with its interior zeroed) are
// measured in one FP64 pass, and x's interior is zeroed again when the
// selection rule prefers u0.
//
// warmstart_train_step: the same forward pass keeping every activation, the
// target u_solved / (s * lambda), the MSE loss reduced on the device, the
// weight and input gradients of every layer, and one Adam step.
//
// Both compose the kernels of cnn.hip (convolutions, features, loss, Adam)
// with the few kernels below (halo clearing, guess smoothing, start
// selection, loss sum).
// Activations live in the caller's workspace; their one-voxel halo is the
// convolution's zero padding, cleared on every call.
#include "ms_internal.hpp"

#pragma clang fp contract(off)

namespace ms {
namespace {

constexpr int kLayers = 4;
constexpr int kCinPad[kLayers] = {8, 32, 32, 32};
constexpr int kWsTaps = 27;
constexpr int kWsCo = 32;
constexpr int kParts = 1024;    // feature-scale and loss partials
constexpr int kSelBlocks = 1024;
constexpr int kSelQ = 6;        // sums of the start selection
constexpr double kSmoothOmega = 2.0 / 3.0;  // damping of the guess smoother

constexpr int64_t layer_wcount(int l) { return (int64_t)kWsTaps * kWsCo * kCinPad[l]; }
constexpr int64_t layer_floats(int l) { return layer_wcount(l) + kWsCo; }

int64_t layer_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += layer_floats(i);
  return o;
}

int64_t param_floats() { return layer_offset(kLayers); }

// Carve of the caller's workspace.
struct WsLayout {
  uint16_t* feat;             // vox x 8 BF16
  uint16_t* h[3];             // vox x 32 BF16 (hidden activations)
  float* out32;               // vox FP32 (u_hat, field layout of the volume)
  uint16_t* wf[kLayers];      // BF16 [27][32][cin]
  uint16_t* wd[kLayers];      // BF16 [27][cin][32]
  double* scale;              // 1
  void* fwork;                // feature workspace
  size_t fwork_bytes;
  double* xs;                 // FP64 field (the smoother's second buffer)
  double* parts;              // kParts
  double* sel;                // kSelBlocks x kSelQ
  int* flag;                  // 1
  // training only
  float* tgt32;               // vox FP32
  uint16_t* dpre[kLayers];    // vox x 32 BF16
  float* gw[kLayers];         // [27][32][cin]
  float* gb[kLayers];         // [32]
  void* wgwork;
  size_t wgwork_bytes;
  size_t total;
};

int64_t vox_count(const ms_grid& g) {
  return (int64_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
}

// Lays the workspace out from `base` (nullptr: sizes only).
WsLayout layout(const ms_grid& g, bool train, char* base) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes, 256);
    return p;
  };
  const int64_t vox = vox_count(g);
  L.feat = reinterpret_cast<uint16_t*>(take((size_t)vox * 8 * 2));
  for (int i = 0; i < 3; ++i) L.h[i] = reinterpret_cast<uint16_t*>(take((size_t)vox * 32 * 2));
  L.out32 = reinterpret_cast<float*>(take((size_t)vox * 4));
  for (int l = 0; l < kLayers; ++l) {
    L.wf[l] = reinterpret_cast<uint16_t*>(take((size_t)layer_wcount(l) * 2));
    L.wd[l] = reinterpret_cast<uint16_t*>(take((size_t)layer_wcount(l) * 2));
  }
  L.scale = reinterpret_cast<double*>(take(sizeof(double)));
  L.fwork_bytes = cnn_features_workspace_bytes(&g);
  L.fwork = take(L.fwork_bytes);
  L.xs = reinterpret_cast<double*>(take((size_t)field_span(g) * sizeof(double)));
  L.parts = reinterpret_cast<double*>(take(kParts * sizeof(double)));
  L.sel = reinterpret_cast<double*>(take((size_t)kSelBlocks * kSelQ * sizeof(double)));
  L.flag = reinterpret_cast<int*>(take(sizeof(int)));
  if (train) {
    L.tgt32 = reinterpret_cast<float*>(take((size_t)vox * 4));
    for (int l = 0; l < kLayers; ++l)
      L.dpre[l] = reinterpret_cast<uint16_t*>(take((size_t)vox * 32 * 2));
    for (int l = 0; l < kLayers; ++l) {
      L.gw[l] = reinterpret_cast<float*>(take((size_t)layer_wcount(l) * 4));
      L.gb[l] = reinterpret_cast<float*>(take(kWsCo * 4));
    }
    L.wgwork_bytes = conv3d_bf16_wgrad_workspace_bytes(32);
    L.wgwork = take(L.wgwork_bytes);
  }
  L.total = off;
  return L;
}

// ------------------------------------------------------------ kernels

// Zeroes the one-voxel halo of an (X+2)(Y+2)(Z+2) volume of `q16` 16-byte
// words per voxel: the z = -1 and z = Z planes, then the y = -1 and y = Y
// rows of every interior plane, then the x = -1 and x = X voxels of every
// interior row.
__global__ __launch_bounds__(256) void halo_zero_kernel(uint4* vol, int X, int Y, int Z,
                                                        int q16) {
  const int64_t px = X + 2, py = Y + 2;
  const int64_t n_planes = 2 * px * py;
  const int64_t n_rows = (int64_t)Z * 2 * px;
  const int64_t n_ends = (int64_t)Z * Y * 2;
  const int64_t n = n_planes + n_rows + n_ends;
  const uint4 zero = make_uint4(0, 0, 0, 0);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * q16;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = t / q16;
    const int w = (int)(t % q16);
    int64_t x, y, z;  // halo-inclusive coordinates (0 .. X+1 etc.)
    if (h < n_planes) {
      z = h < px * py ? 0 : Z + 1;
      const int64_t r = h % (px * py);
      y = r / px;
      x = r % px;
    } else if (h < n_planes + n_rows) {
      const int64_t r = h - n_planes;
      z = 1 + r / (2 * px);
      const int64_t s = r % (2 * px);
      y = s < px ? 0 : Y + 1;
      x = s % px;
    } else {
      const int64_t r = h - n_planes - n_rows;
      z = 1 + r / (2 * (int64_t)Y);
      const int64_t s = r % (2 * (int64_t)Y);
      y = 1 + s / 2;
      x = (s & 1) ? X + 1 : 0;
    }
    vol[((z * py + y) * px + x) * q16 + w] = zero;
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* p, int64_t n16) {
  const uint4 zero = make_uint4(0, 0, 0, 0);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n16;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = zero;
}

// sin(pi (i + 1) / (n + 1)): one axis factor of the slowest mode.
__device__ __forceinline__ double mode_axis(int i, int n) {
  return sinpi((double)(i + 1) / (double)(n + 1));
}

// Per-block sums for the start selection, over interior cells:
//   q0 = sum rg^2, q1 = sum r0^2, q2 = sum rg phi, q3 = sum rg psi,
//   q4 = sum r0 phi, q5 = sum r0 psi,
// rg = f - (S(x) - x*6) (the guess), r0 = f - S(u0) (u's halo, zero
// interior), phi = the product of the three axis sines, psi = (-1)^(i+j+k)
// phi.
__global__ __launch_bounds__(256) void select_partials_kernel(ms_grid g, const double* x,
                                                              const double* u,
                                                              const double* f,
                                                              double* sel) {
  __shared__ double red[kWavesY];
  double q[kSelQ] = {0, 0, 0, 0, 0, 0};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    const double s = ((((x[p + 1] + x[p - 1]) + x[p + g.sy]) + x[p - g.sy]) + x[p + g.sz]) +
                     x[p - g.sz];
    const double lap = s - x[p] * 6.0;
    const double fp = f ? f[p] : 0.0;
    const double rg = f ? fp - lap : -lap;
    // u0: only halo neighbours are non-zero
    const double xp = i == g.nx - 1 ? u[p + 1] : 0.0, xm = i == 0 ? u[p - 1] : 0.0;
    const double yp = j == g.ny - 1 ? u[p + g.sy] : 0.0, ym = j == 0 ? u[p - g.sy] : 0.0;
    const double zp = k == g.nz - 1 ? u[p + g.sz] : 0.0, zm = k == 0 ? u[p - g.sz] : 0.0;
    const double s0 = ((((xp + xm) + yp) + ym) + zp) + zm;
    const double r0 = f ? fp - s0 : -s0;
    const double phi = (mode_axis(k, g.nz) * mode_axis(j, g.ny)) * mode_axis(i, g.nx);
    const double psi = ((i + j + k) & 1) ? -phi : phi;
    q[0] += rg * rg;
    q[1] += r0 * r0;
    q[2] += rg * phi;
    q[3] += rg * psi;
    q[4] += r0 * phi;
    q[5] += r0 * psi;
  }
#pragma unroll
  for (int c = 0; c < kSelQ; ++c) {
    const double v = block_sum(q[c], red);
    if (threadIdx.x == 0) sel[(int64_t)c * kSelBlocks + blockIdx.x] = v;
  }
}

// Sums the partials in a fixed order, applies the rule and publishes the
// choice (flag = 1: keep the guess) and the four measures.
__global__ __launch_bounds__(256) void select_finish_kernel(const double* sel, int rule,
                                                            int* flag, int* used,
                                                            double* measures) {
  __shared__ double red[kWavesY];
  double q[kSelQ];
#pragma unroll
  for (int c = 0; c < kSelQ; ++c) q[c] = sum_partials(sel + (int64_t)c * kSelBlocks,
                                                      kSelBlocks, red);
  if (threadIdx.x != 0) return;
  const double ng = sqrt(q[0]), n0 = sqrt(q[1]);
  const double pg = sqrt(q[2] * q[2] + q[3] * q[3]);
  const double p0 = sqrt(q[4] * q[4] + q[5] * q[5]);
  int keep;
  if (rule == MS_START_FORCE)
    keep = 1;
  else if (rule == MS_START_RESIDUAL)
    keep = ng < n0;
  else
    keep = pg < p0;
  *flag = keep;
  if (used) *used = keep;
  if (measures) {
    measures[0] = ng;
    measures[1] = n0;
    measures[2] = pg;
    measures[3] = p0;
  }
}

// x interior = 0 unless the guess was kept.
__global__ __launch_bounds__(256) void select_apply_kernel(ms_grid g, const int* flag,
                                                           double* x) {
  if (*flag) return;
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    x[(int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1)] = 0.0;
  }
}

__global__ __launch_bounds__(256) void copy_field_kernel(const double* src, double* dst,
                                                         int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

// One damped Jacobi sweep on the interior: out = x + omega * (J(x) - x),
// J(x) = (S(x) - f) * fl(1/6) (S(x) * fl(1/6) without f), in this order.
__global__ __launch_bounds__(256) void damped_sweep_kernel(ms_grid g, const double* x,
                                                           const double* f, double omega,
                                                           double* out) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const double c6 = 1.0 / 6.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny),
              k = (int)(t / ((int64_t)g.nx * g.ny));
    const int64_t p = (int64_t)(k + 1) * g.sz + (int64_t)(j + 1) * g.sy + (i + 1);
    const double s = ((((x[p + 1] + x[p - 1]) + x[p + g.sy]) + x[p - g.sy]) + x[p + g.sz]) +
                     x[p - g.sz];
    const double jac = f ? (s - f[p]) * c6 : s * c6;
    out[p] = x[p] + omega * (jac - x[p]);
  }
}

// loss = (sum of the partials, fixed order) / n.
__global__ __launch_bounds__(256) void loss_sum_kernel(const double* parts, int nparts,
                                                       double n, double* loss) {
  __shared__ double red[kWavesY];
  const double s = sum_partials(parts, nparts, red);
  if (threadIdx.x == 0) *loss = s / n;
}

// ------------------------------------------------------------ host steps

int zero_halo(void* vol, const ms_grid& g, int channels, hipStream_t s) {
  hipLaunchKernelGGL(halo_zero_kernel, dim3(512), dim3(256), 0, s, static_cast<uint4*>(vol),
                     g.nx, g.ny, g.nz, channels * 2 / 16);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

int check_common(const ms_grid* g, const double* u, const float* params, double out_scale,
                 void* work, size_t work_bytes, bool train, const char* who) {
  if (int rc = check_grid(g, who)) return rc;
  if (!u || !params) return set_error(MS_EINVAL, "%s: u and params required", who);
  if (!(out_scale > 0.0) || !std::isfinite(out_scale))
    return set_error(MS_EINVAL, "%s: out_scale must be positive and finite", who);
  const size_t need = layout(*g, train, nullptr).total;
  if (!work || work_bytes < need)
    return set_error(MS_EWORKSPACE, "%s: workspace needs %zu bytes", who, need);
  return MS_OK;
}

// Packs the BF16 weights, clears the activation halos, builds the features
// and runs the four layers (hidden activations kept in L.h, u_hat in
// L.out32).
int forward_pass(const ms_grid& g, const double* u, const double* f, const float* params,
                 const WsLayout& L, hipStream_t s) {
  const int X = g.nx, Y = g.ny, Z = g.nz;
  for (int l = 0; l < kLayers; ++l)
    if (int rc = cnn_pack_weights(kCinPad[l], params + layer_offset(l), L.wf[l], L.wd[l], s))
      return rc;
  if (int rc = zero_halo(L.feat, g, 8, s)) return rc;
  for (int i = 0; i < 3; ++i)
    if (int rc = zero_halo(L.h[i], g, 32, s)) return rc;
  if (int rc = cnn_features(&g, u, f, L.feat, L.scale, L.fwork, L.fwork_bytes, s)) return rc;
  const void* ins[kLayers] = {L.feat, L.h[0], L.h[1], L.h[2]};
  for (int l = 0; l < kLayers; ++l) {
    const bool last = l == kLayers - 1;
    const float* b = params + layer_offset(l) + layer_wcount(l);
    if (int rc = conv3d_bf16_fwd(X, Y, Z, kCinPad[l], ins[l], L.wf[l], b,
                                 last ? nullptr : L.h[l], last ? L.out32 : nullptr,
                                 last ? 0 : 1, s))
      return rc;
  }
  return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" size_t warmstart_params_floats(void) { return (size_t)param_floats(); }

extern "C" size_t warmstart_params_bytes(void) { return (size_t)param_floats() * 3 * 4; }

extern "C" size_t warmstart_layer_offset(int layer) {
  if (layer < 0 || layer > kLayers) return (size_t)-1;
  return (size_t)layer_offset(layer);
}

extern "C" size_t warmstart_workspace_bytes(const ms_grid* g, int train) {
  if (check_grid(g, "warmstart_workspace_bytes")) return 0;
  return layout(*g, train != 0, nullptr).total;
}

extern "C" int warmstart_forward(const ms_grid* g, const double* u, const double* f,
                                 const float* params, double out_scale, int smooth, int rule,
                                 double* x, void* work, size_t work_bytes, int* used,
                                 double* measures, void* stream) {
  clear_error();
  if (int rc = check_common(g, u, params, out_scale, work, work_bytes, false,
                            "warmstart_forward"))
    return rc;
  if (!x) return set_error(MS_EINVAL, "warmstart_forward: x required");
  if (rule != MS_START_RESIDUAL && rule != MS_START_SLOW_MODES && rule != MS_START_FORCE)
    return set_error(MS_EINVAL, "warmstart_forward: unknown start rule %d", rule);
  if (smooth < 0 || smooth > 64 || (smooth & 1))
    return set_error(MS_EINVAL, "warmstart_forward: smooth must be even, 0 .. 64");
  const size_t bytes = (size_t)field_span(*g) * 8;
  if (f && overlaps(f, bytes, x, bytes))
    return set_error(MS_EINVAL, "warmstart_forward: x overlaps f");
  if (u != x && overlaps(u, bytes, x, bytes))
    return set_error(MS_EINVAL, "warmstart_forward: x partly overlaps u");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsLayout L = layout(*g, false, static_cast<char*>(work));
  if (int rc = forward_pass(*g, u, f, params, L, s)) return rc;
  if (int rc = cnn_guess(g, L.out32, L.scale, out_scale, x, s)) return rc;
  if (smooth > 0) {
    const int64_t span = field_span(*g);
    hipLaunchKernelGGL(copy_field_kernel, dim3(1024), dim3(256), 0, s, x, L.xs, span);
    MS_LAUNCH_CHECK();
    for (int m = 0; m < smooth; ++m) {
      const double* src = (m & 1) ? L.xs : x;
      double* dst = (m & 1) ? x : L.xs;
      hipLaunchKernelGGL(damped_sweep_kernel, dim3(1024), dim3(256), 0, s, *g, src, f,
                         kSmoothOmega, dst);
      MS_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(select_partials_kernel, dim3(kSelBlocks), dim3(256), 0, s, *g, x, u, f,
                     L.sel);
  MS_LAUNCH_CHECK();
  hipLaunchKernelGGL(select_finish_kernel, dim3(1), dim3(256), 0, s, L.sel, rule, L.flag, used,
                     measures);
  MS_LAUNCH_CHECK();
  hipLaunchKernelGGL(select_apply_kernel, dim3(1024), dim3(256), 0, s, *g, L.flag, x);
  MS_LAUNCH_CHECK();
  return MS_OK;
}

extern "C" int warmstart_train_step(const ms_grid* g, const double* u, const double* f,
                                    const double* u_solved, float* params, double out_scale,
                                    float lr, int step, void* work, size_t work_bytes,
                                    double* loss, void* stream) {
  clear_error();
  if (int rc = check_common(g, u, params, out_scale, work, work_bytes, true,
                            "warmstart_train_step"))
    return rc;
  if (!u_solved) return set_error(MS_EINVAL, "warmstart_train_step: u_solved required");
  if (!(lr > 0.0f) || !std::isfinite(lr) || step < 1)
    return set_error(MS_EINVAL, "warmstart_train_step: lr must be positive, step >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsLayout L = layout(*g, true, static_cast<char*>(work));
  const int X = g->nx, Y = g->ny, Z = g->nz;
  if (int rc = forward_pass(*g, u, f, params, L, s)) return rc;
  if (int rc = cnn_target(g, u_solved, L.scale, out_scale, L.tgt32, s)) return rc;
  // dpre of the last layer: channel 0 written by the loss, channels 1..31 and
  // the halo zero; the others get their interior from the input gradient
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(L.dpre[kLayers - 1]), vox_count(*g) * 32 * 2 / 16);
  MS_LAUNCH_CHECK();
  for (int l = 0; l < kLayers - 1; ++l)
    if (int rc = zero_halo(L.dpre[l], *g, 32, s)) return rc;
  if (int rc = cnn_mse_grad(X, Y, Z, L.out32, L.tgt32, L.dpre[kLayers - 1], L.parts, kParts, s))
    return rc;
  if (loss) {
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, L.parts, kParts,
                       (double)X * Y * Z, loss);
    MS_LAUNCH_CHECK();
  }
  const void* ins[kLayers] = {L.feat, L.h[0], L.h[1], L.h[2]};
  for (int l = kLayers - 1; l >= 0; --l) {
    if (int rc = conv3d_bf16_wgrad(X, Y, Z, kCinPad[l], ins[l], L.dpre[l], L.gw[l], L.gb[l],
                                   L.wgwork, L.wgwork_bytes, s))
      return rc;
    if (l > 0)
      if (int rc = conv3d_bf16_dgrad(X, Y, Z, kCinPad[l], L.dpre[l], L.wd[l], ins[l],
                                     L.dpre[l - 1], s))
        return rc;
  }
  const int64_t P = param_floats();
  for (int l = 0; l < kLayers; ++l) {
    float* w = params + layer_offset(l);
    float* b = w + layer_wcount(l);
    if (int rc = cnn_adam(kCinPad[l], w, b, w + P, w + 2 * P, b + P, b + 2 * P, L.gw[l],
                          L.gb[l], L.wf[l], L.wd[l], lr, step, s))
      return rc;
  }
  return MS_OK;
}
