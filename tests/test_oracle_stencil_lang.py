"""Pins of the stencil-program interpreter: programs that restate the
oracle's own sweep, advection term and tap stencil give the same bits;
precedence and grouping follow Python's for the same text; offsets, profiles
and lets mean what the language says; malformed programs are rejected."""

import numpy as np
import pytest

import oracle
import synth
from oracle import stencil_lang as sl
from stencil_programs import JACOBI, advection, random_program


def _field(nx, ny, nz, seed, dtype=np.float64):
    a = synth.dirichlet_uniform(nx, ny, nz, seed)
    a[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((nz, ny, nx))
    return a.astype(dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_jacobi_program_equals_the_sweep(dtype):
    u = _field(13, 7, 5, 1, dtype)
    f = synth.gaussian_sources(13, 7, 5, 3, 2).astype(dtype)
    (v,) = sl.run(JACOBI, [u, f], dtype=dtype)
    want = oracle.jacobi_sweep(u, f) if dtype == np.float64 else oracle.sweep_f32(u, f)
    assert v.dtype == dtype
    assert np.array_equal(v, want[1:-1, 1:-1, 1:-1])


def test_advection_program_equals_the_advection_term():
    u, v, w = synth.velocity_fields(12, 9, 7, 3)
    t1, t2 = synth.tzc_arrays(7, 4)
    got = sl.run(advection(), [u, v, w], [0.25, 0.5], [t1, t2])
    want = oracle.advect_source(u, v, w, t1, t2, 0.25, 0.5)
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_, w_)


def test_tap_program_equals_stencil_apply():
    u = _field(9, 8, 6, 5)
    taps = [(1, 0, 0, 0.5), (-1, 1, 0, -0.25), (0, 0, -1, 3.0), (1, -1, 1, 0.125)]
    text = "field u;\nout o = " + " + ".join(
        f"{w!r} * u[{dx},{dy},{dz}]" for dx, dy, dz, w in taps) + ";\n"
    (got,) = sl.run(text, [u])
    assert np.array_equal(got, oracle.stencil_apply(taps, u))


@pytest.mark.parametrize("expr", ["1 - 2 - 3", "2 * 3 + 4 * 5", "8 / 2 / 2", "-3 * -2 - -1",
                                  "1 - (2 - 3)", "0.1 + 0.2 * 3", "1 / 3 * 3 - 1",
                                  "2.5e-3 - 1e2 / 7", "-(4 - 9) / .5", "1e308 * 10 - 1e308"])
def test_precedence_and_grouping_match_python(expr):
    (got,) = sl.run(f"out o = {expr};", [], interior_shape=(1, 1, 1))
    with np.errstate(all="ignore"):
        want = eval(expr)  # Python float arithmetic: same precedence, left grouping
    assert got.shape == (1, 1, 1)
    assert got[0, 0, 0] == want or (np.isinf(want) and got[0, 0, 0] == want)


def test_offsets_profiles_and_lets():
    nx, ny, nz = 6, 5, 4
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    x, y, z = (a.astype(np.float64) for a in (i, j, k))
    t = np.arange(nz, dtype=np.float64) * 10.0
    (dx, dy, dz, pz, lt) = sl.run(
        "field x, y, z; profile t; let d = x[1,0,0] - x[-1,0,0];"
        "out ox = d; out oy = y[0,1,0] - y[0,0,0]; out oz = z[0,0,-1] - z; out ot = t + z;",
        [x, y, z], profiles=[t])[:4] + [None]
    assert np.all(dx == 2) and np.all(dy == 1) and np.all(dz == -1)
    # level k of the interior is z = k + 1 in halo-padded coordinates
    assert np.array_equal(pz, t.reshape(nz, 1, 1) + z[1:-1, 1:-1, 1:-1])


def test_float32_constants_and_params_round_once():
    u = _field(4, 3, 2, 9, np.float32)
    (got,) = sl.run("field u; param c; out o = u * 0.1 + c;", [u], [1.0 / 3.0], dtype=np.float32)
    want = u[1:-1, 1:-1, 1:-1] * np.float32(0.1) + np.float32(1.0 / 3.0)
    assert got.dtype == np.float32 and np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(4))
def test_random_programs_parse_and_evaluate_finite(seed):
    text = random_program(seed)
    a, b, c = (_field(5, 4, 3, 20 + n) for n in range(3))
    outs = sl.run(text, [a, b, c], [0.5, -1.25], [np.linspace(0.5, 2.0, 3)])
    assert len(outs) == 2 and all(np.all(np.isfinite(o)) for o in outs)


@pytest.mark.parametrize("bad", ["field u; out v = u[2,0,0];", "field u; out v = w;",
                                 "field u; out v = u + ;", "field u out v = u;",
                                 "field u; out v = 1e999;", "field u; param u; out v = u;",
                                 "field u; let a = u; out v = a[1,0,0];", "field u;",
                                 "field u; out v = 1x;", "field u; out o = u; out p = o;",
                                 "field let; out o = 1;", "field u; out v = u[1,0];"])
def test_malformed_programs_are_rejected(bad):
    with pytest.raises(ValueError):
        sl.parse(bad)
