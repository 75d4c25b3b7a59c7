"""Learned warm start for the Jacobi solve: host-side orchestration of the
BF16 MFMA convolution kernels (argument marshalling and buffers only; every
arithmetic step runs in libmistencil).

Network: 3x3x3 convolutions 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first
three, "same" zero padding; input [f/s, g/s] (right-hand side and boundary
lift, scaled by s = max(max|f|, max|g|)); output u_hat with the guess
u = s * lambda * u_hat, lambda = max(n)^2 / 8. 57,985 parameters. Trained by
MSE against Jacobi solutions, Adam (lr 1e-3, betas 0.9 / 0.999), FP32
master weights with BF16 copies.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import Grid, _check, _ptr, _stream, grid_of, lib, _field_check

# (real input channels, padded input channels, real output channels, ReLU)
LAYERS = [(2, 8, 32, True), (32, 32, 32, True), (32, 32, 32, True), (32, 32, 1, False)]
TAPS = 27
CO = 32


def output_scale(nx, ny, nz):
    n = max(nx, ny, nz)
    return n * n / 8.0


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
    """Buffers and parameters of the warm-start network for one volume size."""

    def __init__(self, nx, ny, nz, seed=0, device="cuda", params=None):
        self.shape = (nx, ny, nz)
        self.dev = torch.device(device)
        self.lam = output_scale(nx, ny, nz)
        vox = (nx + 2) * (ny + 2) * (nz + 2)
        z = dict(device=self.dev)
        self.feat = torch.zeros(vox * 8, dtype=torch.bfloat16, **z)
        self.h = [torch.zeros(vox * CO, dtype=torch.bfloat16, **z) for _ in range(3)]
        self.out32 = torch.zeros((nz + 2, ny + 2, nx + 2), dtype=torch.float32, **z)
        self.dpre = [torch.zeros(vox * CO, dtype=torch.bfloat16, **z) for _ in range(4)]
        self.dfeat = torch.zeros(vox * 8, dtype=torch.bfloat16, **z)
        self.scale = torch.zeros(1, dtype=torch.float64, **z)
        self.nparts = 1024
        self.parts = torch.zeros(self.nparts, dtype=torch.float64, **z)
        self.wwork = torch.empty(lib.conv3d_bf16_wgrad_workspace_bytes(32), dtype=torch.uint8, **z)
        self.step = 0
        self.set_params(params if params is not None else init_params(seed))

    # -------------------------------------------------------------- params
    def set_params(self, params):
        z = dict(device=self.dev)
        self.w, self.b, self.mw, self.vw, self.mb, self.vb = [], [], [], [], [], []
        self.wf, self.wd, self.gw, self.gb = [], [], [], []
        for (w, b), (_, cinp, _, _) in zip(params, LAYERS):
            wt = torch.as_tensor(np.asarray(w, np.float32)).to(self.dev).contiguous()
            self.w.append(wt)
            self.b.append(torch.as_tensor(np.asarray(b, np.float32)).to(self.dev).contiguous())
            for lst in (self.mw, self.vw, self.gw):
                lst.append(torch.zeros_like(wt))
            for lst in (self.mb, self.vb, self.gb):
                lst.append(torch.zeros(CO, dtype=torch.float32, **z))
            self.wf.append(torch.empty(TAPS * CO * cinp, dtype=torch.bfloat16, **z))
            self.wd.append(torch.empty(TAPS * CO * cinp, dtype=torch.bfloat16, **z))
            _check(lib.cnn_pack_weights(cinp, _ptr(wt), _ptr(self.wf[-1]), _ptr(self.wd[-1]),
                                        _stream()))

    def params(self):
        return [(w.detach().cpu().numpy(), b.detach().cpu().numpy()) for w, b in zip(self.w, self.b)]

    def save(self, path):
        d = {}
        for i, (w, b) in enumerate(self.params()):
            d[f"w{i}"], d[f"b{i}"] = w, b
        d["shape"] = np.array(self.shape)
        d["step"] = np.array(self.step)
        np.savez(path, **d)

    @staticmethod
    def load_params(path):
        d = np.load(path)
        return [(d[f"w{i}"], d[f"b{i}"]) for i in range(len(LAYERS))]

    # ------------------------------------------------------------- forward
    def features(self, u, f):
        _field_check(u, "u", torch.float64)
        g = grid_of(u)
        if tuple(u.shape) != (self.shape[2] + 2, self.shape[1] + 2, self.shape[0] + 2):
            raise ValueError("field shape does not match the network's volume")
        _check(lib.cnn_features(ctypes.byref(g), _ptr(u), _ptr(f), _ptr(self.feat),
                                _ptr(self.scale), _ptr(self.parts), self.nparts, _stream()))

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

    def guess(self, u, f, x):
        """Write s * lambda * u_hat into x's interior (x's halo untouched)."""
        self.forward(u, f)
        g = grid_of(x)
        _check(lib.cnn_guess(ctypes.byref(g), _ptr(self.out32), _ptr(self.scale),
                             float(self.lam), _ptr(x), _stream()))
        return x

    def target(self, u_solved, f_dummy=None, out=None):
        """Training target u / (s * lambda) (FP32) for a solved field; uses
        the scale of the last features() call."""
        if out is None:
            out = torch.zeros_like(self.out32)
        g = grid_of(u_solved)
        _check(lib.cnn_target(ctypes.byref(g), _ptr(u_solved), _ptr(self.scale),
                              float(self.lam), _ptr(out), _stream()))
        return out

    # ------------------------------------------------------------ training
    def backward(self, target):
        """Loss (returned as a device tensor) and parameter gradients for the
        last forward()."""
        X, Y, Z = self.shape
        _check(lib.cnn_mse_grad(X, Y, Z, _ptr(self.out32), _ptr(target), _ptr(self.dpre[3]),
                                _ptr(self.parts), self.nparts, _stream()))
        loss = self.parts.sum() / float(X * Y * Z)
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
        return loss

    def adam(self, lr=1e-3):
        self.step += 1
        for li, (_, cinp, _, _) in enumerate(LAYERS):
            _check(lib.cnn_adam(cinp, _ptr(self.w[li]), _ptr(self.b[li]), _ptr(self.mw[li]),
                                _ptr(self.vw[li]), _ptr(self.mb[li]), _ptr(self.vb[li]),
                                _ptr(self.gw[li]), _ptr(self.gb[li]), _ptr(self.wf[li]),
                                _ptr(self.wd[li]), ctypes.c_float(lr), self.step, _stream()))

    def train_step(self, u, f, target, lr=1e-3):
        self.forward(u, f)
        loss = self.backward(target)
        self.adam(lr)
        return loss

    # ----------------------------------------------------------- helpers
    def act_numpy(self, t, c):
        """A BF16 channels-last activation as a float64 [C, Z, Y, X] interior array."""
        X, Y, Z = self.shape
        a = t.float().view(Z + 2, Y + 2, X + 2, c)[1:-1, 1:-1, 1:-1, :].cpu().numpy()
        return np.transpose(a, (3, 0, 1, 2)).astype(np.float64)
