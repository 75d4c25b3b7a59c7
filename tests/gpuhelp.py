"""Device helpers for the GPU parity tests (layout only, no arithmetic)."""

import sys

import numpy as np
import torch


def dev(a: np.ndarray, pad_x: int = 0, pad_y: int = 0) -> torch.Tensor:
    """Copy a halo-padded numpy field to the device, optionally into a buffer
    with extra row/plane pitch (the padding is filled with NaN)."""
    nz2, ny2, nx2 = a.shape
    if pad_x == 0 and pad_y == 0:
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dt = torch.float64 if a.dtype == np.float64 else torch.float32
    buf = torch.full((nz2, ny2 + pad_y, nx2 + pad_x), float("nan"), dtype=dt, device="cuda")
    view = buf[:, :ny2, :nx2]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return view


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def empty_like_layout(t: torch.Tensor, fill=float("nan")) -> torch.Tensor:
    """A tensor with the same logical shape and strides as ``t``."""
    out = torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)
    # empty_strided may allocate more than numel for padded strides
    out.fill_(fill)
    return out


def note(msg: str):
    print(msg, file=sys.stderr, flush=True)


def on_slab(fn, arrays, z0, k, n):
    """``fn`` (a 3x3x3 "same" operator of [C, Z, Y, X] arrays) on output
    planes z0 .. z0+k-1 of an n-plane volume, run on the planes those outputs
    read (z0-1 .. z0+k, clipped to the volume): the zero padding beyond a cut
    plane only reaches that plane's outputs, which are not returned."""
    lo, hi = max(z0 - 1, 0), min(z0 + k + 1, n)
    return fn(*[a[:, lo:hi] for a in arrays])[:, z0 - lo:z0 - lo + k]
