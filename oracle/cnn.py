"""Oracle for the learned warm start -- TEST INFRASTRUCTURE ONLY.

A small 3D CNN maps the right-hand side and the boundary data of a Poisson
problem to an initial guess. The paper has no learned component; this
follows the project's reading (feature definition, scaling, network shape)
recorded with each function. Everything is FP64 numpy; the BF16 rounding the
GPU applies to inputs, weights and stored activations is emulated where the
GPU rounds (round to nearest even).

Layout: an activation is an array [C, Z, Y, X] over the interior (no halo);
"same" convolution pads with zeros. Weights are [Cout, Cin, 3, 3, 3] with
index [.., dz + 1, dy + 1, dx + 1] for the tap at offset (dx, dy, dz); the
layer computes out[co, p] = b[co] + sum_{ci, d} w[co, ci, d] * x[ci, p + d].
"""

from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def round_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first rounded to float32 (the GPU's accumulator type)."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(x)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _shift(xpad, d, shape):
    """View of the zero-padded activation at offset d = (dx, dy, dz)."""
    dx, dy, dz = d
    _, z, y, x = shape
    return xpad[:, 1 + dz:1 + dz + z, 1 + dy:1 + dy + y, 1 + dx:1 + dx + x]


def conv3d(x, w, b=None):
    """'Same' 3x3x3 convolution (cross-correlation) with zero padding."""
    cin, z, y, xx = x.shape
    cout = w.shape[0]
    xpad = np.zeros((cin, z + 2, y + 2, xx + 2))
    xpad[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((cout, z, y, xx))
    for dx, dy, dz in TAPS:
        wt = w[:, :, dz + 1, dy + 1, dx + 1]  # [cout, cin]
        out += np.tensordot(wt, _shift(xpad, (dx, dy, dz), x.shape), axes=(1, 0))
    if b is not None:
        out += b.reshape(cout, 1, 1, 1)
    return out


def conv3d_dgrad(g, w):
    """Gradient w.r.t. the input of conv3d for output gradient g."""
    cout, z, y, xx = g.shape
    cin = w.shape[1]
    gpad = np.zeros((cout, z + 2, y + 2, xx + 2))
    gpad[:, 1:-1, 1:-1, 1:-1] = g
    out = np.zeros((cin, z, y, xx))
    for dx, dy, dz in TAPS:
        wt = w[:, :, dz + 1, dy + 1, dx + 1]  # [cout, cin]
        # x[ci, p + d] feeds out[co, p]: dx[ci, q] += w[co, ci, d] g[co, q - d]
        out += np.tensordot(wt, _shift(gpad, (-dx, -dy, -dz), g.shape), axes=(0, 0))
    return out


def conv3d_wgrad(x, g):
    """Gradients w.r.t. weights and bias of conv3d for input x, output grad g."""
    cin, z, y, xx = x.shape
    cout = g.shape[0]
    xpad = np.zeros((cin, z + 2, y + 2, xx + 2))
    xpad[:, 1:-1, 1:-1, 1:-1] = x
    dw = np.zeros((cout, cin, 3, 3, 3))
    gm = g.reshape(cout, -1)
    for dx, dy, dz in TAPS:
        xs = _shift(xpad, (dx, dy, dz), x.shape).reshape(cin, -1)
        dw[:, :, dz + 1, dy + 1, dx + 1] = gm @ xs.T
    db = g.sum(axis=(1, 2, 3))
    return dw, db


class Net:
    """Layers 2 -> C -> C -> C -> 1, ReLU after the first three, no
    activation after the last. ``bf16`` emulates the GPU's storage rounding:
    inputs and weights rounded to BF16 before each layer, hidden activations
    stored as BF16 after bias + ReLU, the output kept in FP32."""

    def __init__(self, params, bf16=True):
        self.params = params  # list of (w, b)
        self.bf16 = bf16

    def _r(self, a):
        return round_bf16(a) if self.bf16 else np.asarray(a, dtype=np.float64)

    def forward(self, x):
        acts = [self._r(x)]
        pre = []
        n = len(self.params)
        for li, (w, b) in enumerate(self.params):
            z = conv3d(acts[-1], self._r(w), b)
            pre.append(z)
            if li < n - 1:
                acts.append(self._r(np.maximum(z, 0.0)))
            else:
                out = z.astype(np.float32).astype(np.float64) if self.bf16 else z
                acts.append(out)
        self.acts, self.pre = acts, pre
        return acts[-1]

    def backward(self, gout):
        """Gradients of sum(gout * output) w.r.t. every (w, b), after
        forward(). Hidden gradients pass through the ReLU mask (pre > 0)."""
        grads = [None] * len(self.params)
        g = np.asarray(gout, dtype=np.float64)
        for li in range(len(self.params) - 1, -1, -1):
            w, _ = self.params[li]
            if li < len(self.params) - 1:
                g = g * (self.pre[li] > 0)
            dw, db = conv3d_wgrad(self.acts[li], g)
            grads[li] = (dw, db)
            if li > 0:
                g = conv3d_dgrad(g, self._r(w))
                if self.bf16:
                    g = round_bf16(g)
        return grads


def mse_and_grad(pred, target):
    """Mean squared error over all voxels and its gradient w.r.t. pred."""
    d = pred - target
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of parameter p with gradient g; moments
    m, v updated in place; t is the 1-based step count. Returns new p."""
    m *= b1
    m += (1 - b1) * g
    v *= b2
    v += (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps)


def boundary_lift(u):
    """g = for every interior cell, the sum of the Dirichlet halo values among
    its six neighbours (the boundary's contribution to the 7-point sum), with
    the interior of u ignored. Input/Output: halo-padded array (Z+2, Y+2, X+2)
    in, interior array (Z, Y, X) out."""
    z = np.array(u, dtype=np.float64, copy=True)
    z[1:-1, 1:-1, 1:-1] = 0.0
    nz, ny, nx = (s - 2 for s in z.shape)
    g = np.zeros((nz, ny, nx))
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        g += z[1 + dz:nz + 1 + dz, 1 + dy:ny + 1 + dy, 1 + dx:nx + 1 + dx]
    return g


# Half-widths of the cube averages of f/s among the features: windows of
# side 5, 11, 23, 47 and 95 cells.
BOX_HALF = (2, 5, 11, 23, 47)


def box_sum_axis(a, h, axis):
    """b[p] = sum of a[p + d e_axis] for d = -h .. h in increasing d, with
    zero outside the array (a [Z, Y, X] array; axis 0 = z)."""
    n = a.shape[axis]
    out = np.zeros_like(a)
    for d in range(-h, h + 1):
        lo, hi = max(0, -d), min(n, n - d)  # out[lo:hi] += a[lo+d:hi+d]
        if lo >= hi:
            continue
        dst = [slice(None)] * 3
        src = [slice(None)] * 3
        dst[axis] = slice(lo, hi)
        src[axis] = slice(lo + d, hi + d)
        out[tuple(dst)] = out[tuple(dst)] + a[tuple(src)]
    return out


def box_mean(a, h):
    """Mean of a over the (2h+1)^3 cube around each cell, zero outside the
    interior: sums along x, then y, then z (each in increasing offset), then
    one division by the cube's volume."""
    t = box_sum_axis(np.asarray(a, dtype=np.float64), h, 2)
    t = box_sum_axis(t, h, 1)
    t = box_sum_axis(t, h, 0)
    return t / float((2 * h + 1) ** 3)


def features(u, f):
    """Network input, 8 channels over the interior, and the scale s =
    max(max|f|, max|g|) (1 if 0). Channels: f/s, g/s, the cube means of f/s
    of half-widths BOX_HALF[0..3], phi (the product of sin(pi (i+1)/(n+1))
    over the axes, i.e. the slowest Jacobi mode: the cell's place in the
    domain), the cube mean of half-width BOX_HALF[4]. f and u are halo-padded.

    Reading (the paper has no learned part): a 3x3x3 four-layer network sees
    a 9^3 patch, while the solution at a cell depends on the right-hand side
    everywhere; the cube means give that patch the source mass around it at
    several scales, and phi where it sits between the zero boundaries."""
    fi = np.asarray(f, dtype=np.float64)[1:-1, 1:-1, 1:-1] if f is not None else None
    g = boundary_lift(u)
    if fi is None:
        fi = np.zeros_like(g)
    s = max(float(np.max(np.abs(fi))), float(np.max(np.abs(g))))
    if s == 0.0:
        s = 1.0
    fs = fi / s
    nz, ny, nx = fs.shape
    phi, _ = slowest_modes(nx, ny, nz)
    chans = [fs, g / s] + [box_mean(fs, h) for h in BOX_HALF[:4]] + [phi, box_mean(fs, BOX_HALF[4])]
    return np.stack(chans), s


def smooth_guess(x, f, sweeps, omega=2.0 / 3.0):
    """`sweeps` damped Jacobi sweeps on L(x) = f (Dirichlet halo of x):
    x <- x + omega * (J(x) - x) with J(x) = (S(x) - f) * fl(1/6) the plain
    sweep's update, evaluated in that order in FP64.

    Reading: a learned guess carries cell-to-cell errors; in plain Jacobi the
    modes near the checkerboard decay no faster than the smoothest one, so
    such errors cost as many sweeps as a wrong smooth component. A damped
    sweep multiplies every mode by 1 - omega (1 - mu) (mu its plain Jacobi
    factor), which for omega = 2/3 is at most 1/3 in size for mu <= 0, so a
    few of them remove those errors and leave the smooth part of the guess
    nearly untouched."""
    from .stencil import interior, jacobi_sweep
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(sweeps):
        j = interior(jacobi_sweep(x, f))
        xi = interior(x)
        x[1:-1, 1:-1, 1:-1] = xi + omega * (j - xi)
    return x


# ------------------------------------------------------- start selection
#
# Reading (the paper has no learned part): plain Jacobi from the zero
# interior is the guess's fallback. Three rules decide whether a solve starts
# from the network's guess or from u0 (u with its interior zeroed):
#   "residual"   -- the guess iff ||r(guess)|| < ||r(u0)||;
#   "slow_modes" -- the guess iff the projection of r(guess) on the two
#                   slowest-decaying eigenvectors of the Jacobi iteration is
#                   shorter than that of r(u0): these two components decay
#                   by rho per sweep, slower than every other, so they set
#                   the sweep count at a tight tolerance, while the residual
#                   norm of a guess is dominated by fast-decaying,
#                   high-frequency components;
#   "force"      -- always the guess.
# Ties go to u0.

RULES = ("residual", "slow_modes", "force")


def slowest_modes(nx, ny, nz):
    """phi(i, j, k) = sin(pi (i+1)/(nx+1)) sin(pi (j+1)/(ny+1)) sin(pi (k+1)/(nz+1))
    and psi = (-1)^(i+j+k) phi over the interior (arrays [Z, Y, X]): the
    eigenvectors of the 7-point operator with a zero Dirichlet halo whose
    Jacobi iteration factors are +rho and -rho, rho = the mean of the three
    cos(pi/(n+1))."""
    def axis(n):
        return np.sin(np.pi * np.arange(1, n + 1) / (n + 1))
    phi = axis(nz)[:, None, None] * axis(ny)[None, :, None] * axis(nx)[None, None, :]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sign = 1.0 - 2.0 * ((i + j + k) % 2)
    return phi, sign * phi


def slow_mode_norm(r):
    """sqrt(<r, phi>^2 + <r, psi>^2) for an interior array r [Z, Y, X]."""
    r = np.asarray(r, dtype=np.float64)
    phi, psi = slowest_modes(r.shape[2], r.shape[1], r.shape[0])
    p, q = float(np.sum(r * phi)), float(np.sum(r * psi))
    return float(np.sqrt(p * p + q * q))


def start_choice(u, f, guess, rule):
    """Whether a solve of L(x) = f (Dirichlet halo of u) starts from `guess`
    (interior array [Z, Y, X]) under `rule`; also returns the four measures
    (||r(guess)||, ||r(u0)||, slow(r(guess)), slow(r(u0))), all in FP64."""
    from .stencil import residual
    if rule not in RULES:
        raise ValueError(rule)
    u0 = np.array(u, dtype=np.float64, copy=True)
    u0[1:-1, 1:-1, 1:-1] = 0.0
    xg = u0.copy()
    xg[1:-1, 1:-1, 1:-1] = guess
    rg, r0 = residual(xg, f), residual(u0, f)
    meas = (float(np.sqrt(np.sum(rg * rg))), float(np.sqrt(np.sum(r0 * r0))),
            slow_mode_norm(rg), slow_mode_norm(r0))
    if rule == "force":
        use = True
    elif rule == "residual":
        use = meas[0] < meas[1]
    else:
        use = meas[2] < meas[3]
    return use, meas
