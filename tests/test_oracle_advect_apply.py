"""Pins of the oracle's advection source term and general stencil apply."""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from test_oracle_jacobi import Counted, counted_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def _fields(nx, ny, nz, seed):
    u, v, w = synth.velocity_fields(nx, ny, nz, seed)
    t1, t2 = synth.tzc_arrays(nz, seed + 100)
    return u, v, w, t1, t2


# ----------------------------------------------------------------- advection

def test_advection_costs_63_flops_per_cell_like_the_paper():
    facts = json.load(open(GOLDEN))
    nx, ny, nz = 3, 2, 2
    u, v, w, t1, t2 = _fields(nx, ny, nz, 1)
    cu, cv, cw = counted_grid(u), counted_grid(v), counted_grid(w)
    Counted.n = 0
    oracle.advect_source(cu, cv, cw, t1, t2, 0.25, 0.25)
    assert Counted.n == facts["pw_advection_flops_per_cell"]["value"] * nx * ny * nz


def test_constant_fields_give_zero_source():
    shape = (6, 7, 8)
    u, v, w = np.full(shape, 1.5), np.full(shape, -2.25), np.full(shape, 3.0)
    t = synth.rng(3).uniform(0.5, 2.0, 4)
    for s in oracle.advect_source(u, v, w, t, t, 0.25, 0.7):
        assert np.all(s == 0.0)


def test_doubling_the_velocities_scales_the_source_by_four_exactly():
    u, v, w, t1, t2 = _fields(9, 8, 7, 2)
    a = oracle.advect_source(u, v, w, t1, t2, 0.25, 0.25)
    b = oracle.advect_source(2 * u, 2 * v, 2 * w, t1, t2, 0.25, 0.25)
    for x, y in zip(a, b):
        assert np.array_equal(4 * x, y)


def test_each_coefficient_enters_linearly():
    u, v, w, t1, t2 = _fields(6, 5, 4, 3)
    z = np.zeros_like(t1)
    only_x = oracle.advect_source(u, v, w, z, z, 1.0, 0.0)
    only_y = oracle.advect_source(u, v, w, z, z, 0.0, 1.0)
    only_z = oracle.advect_source(u, v, w, t1, t2, 0.0, 0.0)
    full = oracle.advect_source(u, v, w, t1, t2, 0.5, 0.25)
    for a, b, c, d in zip(only_x, only_y, only_z, full):
        assert np.allclose((0.5 * a + 0.25 * b) + c, d, rtol=1e-13, atol=1e-12)


def test_rounding_error_is_within_the_forward_bound():
    """Exact rational evaluation of the same expression: each output is
    within c * eps * M of it, M being the expression with every input and
    operation taken in absolute value."""
    nx, ny, nz = 4, 3, 3
    u, v, w, t1, t2 = _fields(nx, ny, nz, 4)
    got = oracle.advect_source(u, v, w, t1, t2, 0.25, 0.25)

    def frac(a):
        return np.vectorize(Fraction, otypes=[object])(a)

    ex = oracle.advect_source(frac(u), frac(v), frac(w), frac(t1), frac(t2),
                              Fraction(1, 4), Fraction(1, 4))
    # Every path through the expression tree has at most six roundings
    # (add and multiply inside P, the difference, the coefficient product,
    # two sums), so |fl - exact| <= gamma_6 * M with M the sum of
    # |coefficient * P| over the six products of the output.
    mags = _abs_products(np.abs(u), np.abs(v), np.abs(w), np.abs(t1), np.abs(t2), 0.25, 0.25)
    for a, e, m in zip(got, ex, mags):
        err = np.abs(a - np.array(e, dtype=np.float64))
        assert np.all(err <= 7 * 2.0 ** -53 * m)


def _abs_products(u, v, w, t1, t2, tcx, tcy):
    """Sum of |coefficient * P| over the six products of each field, given
    nonnegative inputs: the advection formula with every '-' turned into '+'."""
    sh = oracle.stencil.shifted
    nz = u.shape[0] - 2
    a1 = t1.reshape(nz, 1, 1)
    a2 = t2.reshape(nz, 1, 1)

    def tot(pxm, pxp, pym, pyp, pzm, pzp):
        return tcx * (pxm + pxp) + tcy * (pym + pyp) + a1 * pzm + a2 * pzp

    su = tot(sh(u, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, 0, 0, 0)),
             sh(u, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 1, 0, 0)),
             sh(u, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 1, -1, 0)),
             sh(u, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 1, 0, 0)),
             sh(u, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 1, 0, -1)),
             sh(u, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 1, 0, 0)))
    sv = tot(sh(v, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, -1, 1, 0)),
             sh(v, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 0, 1, 0)),
             sh(v, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 0, 0, 0)),
             sh(v, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 0, 1, 0)),
             sh(v, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 0, 1, -1)),
             sh(v, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 0, 1, 0)))
    sw = tot(sh(w, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, -1, 0, 1)),
             sh(w, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 0, 0, 1)),
             sh(w, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 0, -1, 1)),
             sh(w, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 0, 0, 1)),
             sh(w, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 0, 0, 0)),
             sh(w, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 0, 0, 1)))
    return su, sv, sw


# analytic fields on the unit periodic cube for the convergence pin
_MODES = {
    "u": [(1.3, (1, 2, 1), 0.3), (0.7, (2, 0, 1), 1.1)],
    "v": [(0.9, (0, 1, 2), 2.0), (1.1, (1, 1, 1), 0.2)],
    "w": [(1.2, (2, 1, 0), 0.5), (0.6, (1, 2, 2), 1.7)],
}


def _eval(name, x, y, z, d=None):
    """Field value (d=None) or its derivative along axis d (0, 1, 2)."""
    out = 0.0
    for a, k, th in _MODES[name]:
        ph = 2 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + th
        if d is None:
            out = out + a * np.sin(ph)
        else:
            out = out + a * 2 * math.pi * k[d] * np.cos(ph)
    return out


def _sample(name, n, stag):
    h = 1.0 / n
    ii = (np.arange(-1, n + 1) + stag[0]) * h
    jj = (np.arange(-1, n + 1) + stag[1]) * h
    kk = (np.arange(-1, n + 1) + stag[2]) * h
    z, y, x = np.meshgrid(kk, jj, ii, indexing="ij")
    return _eval(name, x, y, z)


def _continuous_source(phi, n, stag):
    """-1/2 [div(vel phi) + vel . grad phi] at phi's own sample points."""
    h = 1.0 / n
    ii = (np.arange(n) + stag[0]) * h
    jj = (np.arange(n) + stag[1]) * h
    kk = (np.arange(n) + stag[2]) * h
    z, y, x = np.meshgrid(kk, jj, ii, indexing="ij")
    p = _eval(phi, x, y, z)
    vel = [_eval(c, x, y, z) for c in "uvw"]
    dvel = [_eval(c, x, y, z, d) for d, c in enumerate("uvw")]
    dp = [_eval(phi, x, y, z, d) for d in range(3)]
    return -0.5 * sum(dvel[d] * p + 2 * vel[d] * dp[d] for d in range(3))


def test_advection_converges_at_second_order_to_the_continuous_operator():
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        u = _sample("u", n, (0.5, 0, 0))
        v = _sample("v", n, (0, 0.5, 0))
        w = _sample("w", n, (0, 0, 0.5))
        t = np.full(n, 1.0 / (4 * h))
        su, sv, sw = oracle.advect_source(u, v, w, t, t, 1 / (4 * h), 1 / (4 * h))
        e = max(np.max(np.abs(su - _continuous_source("u", n, (0.5, 0, 0)))),
                np.max(np.abs(sv - _continuous_source("v", n, (0, 0.5, 0)))),
                np.max(np.abs(sw - _continuous_source("w", n, (0, 0, 0.5)))))
        errs.append(e)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(o > 1.8 for o in orders), (errs, orders)


# ------------------------------------------------------------- stencil apply

def test_listing1_four_point_average_matches_array_slicing():
    """Listing 1's two-dimensional average on its own 256x256 array (loop
    bounds, offsets and factor from the golden file), against the same
    average written independently with numpy slices: each interior point
    takes a quarter of the sum of its four axis neighbours in the old array
    (stencil.apply is out-of-place)."""
    facts = json.load(open(GOLDEN))["listing1"]
    n = 256
    assert (facts["loop_lo"], facts["loop_hi"]) == (2, n - 1)  # 1-based: interior 1..n-2
    d = synth.rng(7).random((n, n))  # d[y, x]; x is the first (contiguous) index
    want = (d[:-2, 1:-1] + d[2:, 1:-1] + d[1:-1, :-2] + d[1:-1, 2:]) * facts["scale"]
    grid = np.zeros((3, n, n))
    grid[1] = d
    taps = [(dx, dy, 0, 1.0) for dx, dy in facts["offsets_first_second_index"]]
    got = oracle.stencil_apply(taps, grid, scale=facts["scale"])
    assert got.shape == (1, n - 2, n - 2)  # output bounds [0,254) x [0,254)
    np.testing.assert_allclose(got[0], want, rtol=1e-15, atol=0)
    # the offsets name the four axis neighbours, once each
    assert sorted(map(tuple, facts["offsets_first_second_index"])) == [(-1, 0), (0, -1), (0, 1),
                                                                      (1, 0)]


def test_delta_tap_is_an_exact_shift():
    u = synth.rng(9).standard_normal((6, 7, 8))
    for d in [(1, 0, 0), (0, -1, 0), (0, 0, 1), (-1, 1, -1)]:
        got = oracle.stencil_apply([(d[0], d[1], d[2], 1.0)], u)
        assert np.array_equal(got, u[1 + d[2]:5 + d[2], 1 + d[1]:6 + d[1], 1 + d[0]:7 + d[0]])


def test_taps_with_rhs_reproduce_the_jacobi_update_bit_for_bit():
    u = synth.dirichlet_uniform(9, 8, 7, 3)
    u[1:-1, 1:-1, 1:-1] = synth.rng(4).random((7, 8, 9))
    f = synth.gaussian_sources(9, 8, 7, 3, 5)
    taps = [(1, 0, 0, 1.0), (-1, 0, 0, 1.0), (0, 1, 0, 1.0), (0, -1, 0, 1.0),
            (0, 0, 1, 1.0), (0, 0, -1, 1.0)]
    got = oracle.stencil_apply(taps, u, rhs=f, rhs_coef=-1.0, scale=oracle.C6_F64)
    assert np.array_equal(got, oracle.jacobi_sweep(u, f)[1:-1, 1:-1, 1:-1])


def test_tzc1_weights_the_lower_face_and_tzc2_the_upper():
    """With only tzc1 switched on the source at level k depends on the lower
    face (levels k-1, k) alone; with only tzc2 on the upper face (k, k+1)."""
    u, v, w, t1, t2 = _fields(5, 4, 6, 5)
    z = np.zeros_like(t1)
    lo = oracle.advect_source(u, v, w, t1, z, 0.0, 0.0)
    hi = oracle.advect_source(u, v, w, z, t2, 0.0, 0.0)
    k = 3  # interior level; array plane k + 1
    u2, v2, w2 = u.copy(), v.copy(), w.copy()
    for a in (u2, v2, w2):
        a[k + 2:] += 1.0  # change everything above level k
    lo2 = oracle.advect_source(u2, v2, w2, t1, z, 0.0, 0.0)
    for a, b in zip(lo, lo2):
        assert np.array_equal(a[k], b[k])
    u3, v3, w3 = u.copy(), v.copy(), w.copy()
    for a in (u3, v3, w3):
        a[:k + 1] += 1.0  # change every level below k
    hi3 = oracle.advect_source(u3, v3, w3, z, t2, 0.0, 0.0)
    for a, b in zip(hi, hi3):
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(lo[0][k], oracle.advect_source(u3, v3, w3, t1, z, 0.0, 0.0)[0][k])
