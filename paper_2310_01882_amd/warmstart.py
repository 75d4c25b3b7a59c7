"""Learned warm start for the Jacobi solve: argument marshalling and buffers
for the library's warm-start entry points (every arithmetic step runs in
libmistencil).

Network: 3x3x3 convolutions 8 -> 32 -> 32 -> 32 -> 1, ReLU after the first
three, "same" zero padding; input: eight feature channels of the
right-hand side f and the boundary lift g, scaled by s = max(max|f|,
max|g|) (f/s, g/s, cube means of f/s at five scales, the slowest Jacobi
mode as position); output u_hat with the guess u = s * out_scale * u_hat,
then a few damped Jacobi sweeps. 63,169 parameters (stored padded to 32
output channels in the last layer). Trained by MSE against Jacobi
solutions with Adam (betas 0.9 / 0.999), FP32 master weights with BF16
copies.

The product path is two calls: ``guess`` (warmstart_forward: features,
network, guess, start selection) and ``train_step`` (warmstart_train_step:
forward, loss, gradients, Adam). The layer-by-layer methods further down
drive the individual kernels for the tests of each kernel.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import (MS_START_FORCE, MS_START_RESIDUAL, MS_START_SLOW_MODES, Grid, _check,
               _field_check, _ptr, _same_layout, _stream, grid_of, lib)

# (real input channels, padded input channels, real output channels, ReLU)
LAYERS = [(8, 8, 32, True), (32, 32, 32, True), (32, 32, 32, True), (32, 32, 1, False)]
TAPS = 27
CO = 32
RULES = {"residual": MS_START_RESIDUAL, "slow_modes": MS_START_SLOW_MODES,
         "force": MS_START_FORCE}


def default_out_scale(nx, ny, nz):
    """out_scale = max(n)^2 / 4096 (4 at 128^3): the solution of these
    problems grows like the square of the source width, which scales with
    the grid; this keeps the targets u / (s * out_scale) of order one."""
    n = max(nx, ny, nz)
    return n * n / 4096.0


def init_params(seed: int):
    """He-normal weights for the hidden layers, a small last layer, zero
    biases; padded channels are zero. Returns [(w[27][32][cin_pad], b[32])]."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for li, (cin, cinp, cout, _) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (TAPS * cin)) if li < len(LAYERS) - 1 else 0.1 / np.sqrt(TAPS * cin)
        w = np.zeros((TAPS, CO, cinp), np.float32)
        w[:, :cout, :cin] = (std * g.standard_normal((TAPS, cout, cin))).astype(np.float32)
        out.append((w, np.zeros(CO, np.float32)))
    return out


def to_oracle_weights(w, cin, cout):
    """[27][32][cinp] (tap = (dx+1) + 3(dy+1) + 9(dz+1)) -> [cout, cin, 3, 3, 3]
    indexed [.., dz+1, dy+1, dx+1]."""
    w = np.asarray(w, np.float64)[:, :cout, :cin].reshape(3, 3, 3, cout, cin)
    return np.transpose(w, (3, 4, 0, 1, 2))


class WarmStart:
    """Parameters (master weights and Adam moments in one device buffer) and
    workspaces of the warm-start network for one volume size."""

    def __init__(self, nx, ny, nz, seed=0, device="cuda", params=None, out_scale=None):
        self.shape = (nx, ny, nz)
        self.dev = torch.device(device)
        self.out_scale = float(out_scale if out_scale is not None
                               else default_out_scale(nx, ny, nz))
        self.nparam = int(lib.warmstart_params_floats())
        self.pbuf = torch.zeros(3 * self.nparam, dtype=torch.float32, device=self.dev)
        self.offsets = [int(lib.warmstart_layer_offset(li)) for li in range(len(LAYERS) + 1)]
        self.w, self.b, self.mw, self.vw, self.mb, self.vb = [], [], [], [], [], []
        for li, (_, cinp, _, _) in enumerate(LAYERS):
            o, nw = self.offsets[li], TAPS * CO * cinp
            for blk, (lw, lb) in enumerate(((self.w, self.b), (self.mw, self.mb),
                                            (self.vw, self.vb))):
                base = blk * self.nparam + o
                lw.append(self.pbuf[base:base + nw].view(TAPS, CO, cinp))
                lb.append(self.pbuf[base + nw:base + nw + CO])
        self.step = 0
        z = dict(device=self.dev)
        self.used = torch.zeros(1, dtype=torch.int32, **z)
        self.measures = torch.zeros(4, dtype=torch.float64, **z)
        self.loss = torch.zeros(1, dtype=torch.float64, **z)
        self._work = {}
        self._layer_bufs = None
        self.set_params(params if params is not None else init_params(seed))

    # -------------------------------------------------------------- params
    def set_params(self, params):
        """Load [(w[27][32][cinp], b[32])] as master weights; Adam restarts."""
        self.pbuf.zero_()
        for li, (w, b) in enumerate(params):
            self.w[li].copy_(torch.as_tensor(np.asarray(w, np.float32)))
            self.b[li].copy_(torch.as_tensor(np.asarray(b, np.float32)))
        self.step = 0
        if self._layer_bufs is not None:
            self._pack()

    def params(self):
        return [(w.detach().cpu().numpy().copy(), b.detach().cpu().numpy().copy())
                for w, b in zip(self.w, self.b)]

    def save(self, path, meta=None):
        d = {}
        for i, (w, b) in enumerate(self.params()):
            d[f"w{i}"], d[f"b{i}"] = w, b
        d["shape"] = np.array(self.shape)
        d["step"] = np.array(self.step)
        d["out_scale"] = np.array(self.out_scale)
        for k, v in (meta or {}).items():
            d[f"meta_{k}"] = np.array(v)
        np.savez(path, **d)

    @staticmethod
    def load(path):
        """(params, out_scale, meta) from a file written by save()."""
        d = np.load(path)
        params = [(d[f"w{i}"], d[f"b{i}"]) for i in range(len(LAYERS))]
        if "out_scale" in d:
            out_scale = float(d["out_scale"])
        else:  # files written before the scale was stored used max(n)^2 / 8
            out_scale = float(np.max(d["shape"])) ** 2 / 8.0
        meta = {k[5:]: d[k].item() for k in d.files if k.startswith("meta_")}
        return params, out_scale, meta

    @classmethod
    def from_file(cls, path, nx, ny, nz, device="cuda"):
        params, out_scale, _ = cls.load(path)
        return cls(nx, ny, nz, device=device, params=params, out_scale=out_scale)

    def _workspace(self, u, train):
        g = grid_of(u)
        key = (train, tuple(u.shape))
        need = int(lib.warmstart_workspace_bytes(ctypes.byref(g), int(train)))
        ws = self._work.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.dev)
            self._work[key] = ws
        return ws

    def _check_volume(self, u):
        _field_check(u, "u", torch.float64)
        if tuple(u.shape) != (self.shape[2] + 2, self.shape[1] + 2, self.shape[0] + 2):
            raise ValueError("field shape does not match the network's volume")

    # --------------------------------------------------- product entry points
    def guess(self, u, f, x, rule="slow_modes", smooth=4, stream=None):
        """warmstart_forward: the guess for (u's Dirichlet halo, f) in x's
        interior after `smooth` damped Jacobi sweeps, or x's interior zeroed
        when the start rule prefers u0.
        Returns device tensors (used [1] int32, measures [4] float64:
        ||r(x)||, ||r(u0)||, slow(r(x)), slow(r(u0)))."""
        self._check_volume(u)
        _field_check(x, "x", torch.float64)
        _same_layout(u, x, "u/x")
        if f is not None:
            _field_check(f, "f", torch.float64)
            _same_layout(u, f, "u/f")
        g = grid_of(u)
        ws = self._workspace(u, False)
        _check(lib.warmstart_forward(ctypes.byref(g), _ptr(u), _ptr(f), _ptr(self.pbuf),
                                     self.out_scale, int(smooth), RULES[rule], _ptr(x), _ptr(ws),
                                     ws.numel(), _ptr(self.used), _ptr(self.measures),
                                     _stream(stream)))
        return self.used, self.measures

    def train_step(self, u, f, u_solved, lr=1e-3, stream=None):
        """warmstart_train_step on one solved instance; returns the loss (a
        device tensor, before the update)."""
        self._check_volume(u)
        _field_check(u_solved, "u_solved", torch.float64)
        _same_layout(u, u_solved, "u/u_solved")
        if f is not None:
            _field_check(f, "f", torch.float64)
            _same_layout(u, f, "u/f")
        g = grid_of(u)
        ws = self._workspace(u, True)
        self.step += 1
        _check(lib.warmstart_train_step(ctypes.byref(g), _ptr(u), _ptr(f), _ptr(u_solved),
                                        _ptr(self.pbuf), self.out_scale, ctypes.c_float(lr),
                                        self.step, _ptr(ws), ws.numel(), _ptr(self.loss),
                                        _stream(stream)))
        if self._layer_bufs is not None:
            self._pack()
        return self.loss

    # ---------------------------------------- layer-by-layer (kernel tests)
    def _bufs(self):
        if self._layer_bufs is None:
            X, Y, Z = self.shape
            vox = (X + 2) * (Y + 2) * (Z + 2)
            z = dict(device=self.dev)
            self.feat = torch.zeros(vox * 8, dtype=torch.bfloat16, **z)
            self.h = [torch.zeros(vox * CO, dtype=torch.bfloat16, **z) for _ in range(3)]
            self.out32 = torch.zeros((Z + 2, Y + 2, X + 2), dtype=torch.float32, **z)
            self.dpre = [torch.zeros(vox * CO, dtype=torch.bfloat16, **z) for _ in range(4)]
            self.scale = torch.zeros(1, dtype=torch.float64, **z)
            self.nparts = 1024
            self.parts = torch.zeros(self.nparts, dtype=torch.float64, **z)
            gg = Grid(X, Y, Z, 0, X + 2, (X + 2) * (Y + 2))
            self.fwork = torch.empty(lib.cnn_features_workspace_bytes(ctypes.byref(gg)),
                                     dtype=torch.uint8, **z)
            self.wwork = torch.empty(lib.conv3d_bf16_wgrad_workspace_bytes(32),
                                     dtype=torch.uint8, **z)
            self.wf, self.wd, self.gw, self.gb = [], [], [], []
            for (_, cinp, _, _) in LAYERS:
                self.wf.append(torch.empty(TAPS * CO * cinp, dtype=torch.bfloat16, **z))
                self.wd.append(torch.empty(TAPS * CO * cinp, dtype=torch.bfloat16, **z))
                self.gw.append(torch.zeros((TAPS, CO, cinp), dtype=torch.float32, **z))
                self.gb.append(torch.zeros(CO, dtype=torch.float32, **z))
            self._layer_bufs = True
            self._pack()

    def _pack(self):
        for li, (_, cinp, _, _) in enumerate(LAYERS):
            _check(lib.cnn_pack_weights(cinp, _ptr(self.w[li]), _ptr(self.wf[li]),
                                        _ptr(self.wd[li]), _stream()))

    def features(self, u, f):
        self._check_volume(u)
        self._bufs()
        g = grid_of(u)
        _check(lib.cnn_features(ctypes.byref(g), _ptr(u), _ptr(f), _ptr(self.feat),
                                _ptr(self.scale), _ptr(self.fwork), self.fwork.numel(),
                                _stream()))

    def forward(self, u, f):
        """u_hat (FP32, field layout) for the problem (u: Dirichlet halo, f)."""
        X, Y, Z = self.shape
        self.features(u, f)
        ins = [self.feat, self.h[0], self.h[1], self.h[2]]
        for li, (_, cinp, _, relu) in enumerate(LAYERS):
            last = li == len(LAYERS) - 1
            _check(lib.conv3d_bf16_fwd(X, Y, Z, cinp, _ptr(ins[li]), _ptr(self.wf[li]),
                                       _ptr(self.b[li]), None if last else _ptr(self.h[li]),
                                       _ptr(self.out32) if last else None, int(relu), _stream()))
        return self.out32

    def target(self, u_solved, out=None):
        """Training target u / (s * out_scale) (FP32) for a solved field; uses
        the scale of the last features() call."""
        self._bufs()
        if out is None:
            out = torch.zeros_like(self.out32)
        g = grid_of(u_solved)
        _check(lib.cnn_target(ctypes.byref(g), _ptr(u_solved), _ptr(self.scale),
                              self.out_scale, _ptr(out), _stream()))
        return out

    def backward(self, target):
        """Parameter gradients (into gw, gb) for the last forward(); the loss
        partials go to ``parts`` (sum / voxels = the MSE loss)."""
        X, Y, Z = self.shape
        _check(lib.cnn_mse_grad(X, Y, Z, _ptr(self.out32), _ptr(target), _ptr(self.dpre[3]),
                                _ptr(self.parts), self.nparts, _stream()))
        ins = [self.feat, self.h[0], self.h[1], self.h[2]]
        for li in range(len(LAYERS) - 1, -1, -1):
            cinp = LAYERS[li][1]
            _check(lib.conv3d_bf16_wgrad(X, Y, Z, cinp, _ptr(ins[li]), _ptr(self.dpre[li]),
                                         _ptr(self.gw[li]), _ptr(self.gb[li]), _ptr(self.wwork),
                                         self.wwork.numel(), _stream()))
            if li > 0:
                _check(lib.conv3d_bf16_dgrad(X, Y, Z, cinp, _ptr(self.dpre[li]),
                                             _ptr(self.wd[li]), _ptr(ins[li]),
                                             _ptr(self.dpre[li - 1]), _stream()))
        return self.parts

    def act_numpy(self, t, c):
        """A BF16 channels-last activation as a float64 [C, Z, Y, X] interior array."""
        X, Y, Z = self.shape
        a = t.float().view(Z + 2, Y + 2, X + 2, c)[1:-1, 1:-1, 1:-1, :].cpu().numpy()
        return np.transpose(a, (3, 0, 1, 2)).astype(np.float64)
