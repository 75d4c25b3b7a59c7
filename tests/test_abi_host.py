"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mistencil.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_the_four_named_entry_points():
    names = declared_functions()
    for n in ("stencil_apply", "jacobi_solve", "advect_source", "residual_norm"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2310_01882_amd as ms
    raw = ctypes.CDLL(ms.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing
    # the binding covers the same set
    assert set(declared_functions()) <= set(ms.SIGNATURES)


def test_version_and_error_strings():
    import paper_2310_01882_amd as ms
    assert b"gfx950" in ms.lib.ms_version()
    assert isinstance(ms.last_error(), str)


def _grid(ms, nx=8, ny=6, nz=4, sy=None, sz=None):
    sy = sy if sy is not None else nx + 2
    sz = sz if sz is not None else sy * (ny + 2)
    return ms.Grid(nx, ny, nz, 0, sy, sz)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
FAKE2 = ctypes.c_void_p(0x10000000)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-1), dict(sy=9), dict(sz=50)])
def test_bad_grids_are_rejected(bad):
    import paper_2310_01882_amd as ms
    kw = dict(nx=8, ny=6, nz=4)
    kw.update(bad)
    g = _grid(ms, **kw)
    rc = ms.lib.jacobi_sweeps(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, 1, None, FAKE,
                              1 << 20, None)
    assert rc == ms.MS_EINVAL
    assert ms.last_error()
    assert ms.lib.residual_workspace_bytes(ctypes.byref(g)) == 0


def test_null_and_aliased_buffers_are_rejected():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    assert ms.lib.jacobi_sweeps(ctypes.byref(g), ms.MS_F64, None, FAKE2, None, 1, None, FAKE,
                                1 << 20, None) == ms.MS_EINVAL
    # u and u_tmp overlap
    assert ms.lib.jacobi_sweeps(ctypes.byref(g), ms.MS_F64, FAKE, ctypes.c_void_p(0x1008), None,
                                1, None, FAKE, 1 << 20, None) == ms.MS_EINVAL
    assert "overlap" in ms.last_error()


def test_workspace_too_small_is_reported():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    need = ms.lib.jacobi_sweeps_workspace_bytes(ctypes.byref(g))
    assert need > 0
    rc = ms.lib.jacobi_sweeps(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, 1, None, FAKE,
                              need - 1, None)
    assert rc == ms.MS_EWORKSPACE


def test_bad_dtype_is_unsupported():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    out = ctypes.c_double()
    rc = ms.lib.residual_norm(ctypes.byref(g), 7, FAKE, None, ctypes.byref(out), 0, FAKE,
                              1 << 20, None)
    assert rc == ms.MS_EUNSUPPORTED


def test_stencil_apply_validation():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    taps = (ms.Tap * 2)()
    taps[0].dx, taps[0].w = 1, 1.0
    taps[1].dz, taps[1].w = 2, 1.0  # beyond the one-cell halo
    st = ms.Stencil(2, 0, taps, 0.0, 1.0)
    assert ms.lib.stencil_apply(ctypes.byref(st), ctypes.byref(g), ms.MS_F64, FAKE, None, FAKE2,
                                None) == ms.MS_EINVAL
    st = ms.Stencil(0, 0, taps, 0.0, 1.0)
    assert ms.lib.stencil_apply(ctypes.byref(st), ctypes.byref(g), ms.MS_F64, FAKE, None, FAKE2,
                                None) == ms.MS_EUNSUPPORTED
    taps[1].dz = 1
    st = ms.Stencil(2, 0, taps, 0.0, 1.0)
    # in-place apply is not allowed (stencil.apply is out-of-place)
    assert ms.lib.stencil_apply(ctypes.byref(st), ctypes.byref(g), ms.MS_F64, FAKE, None, FAKE,
                                None) == ms.MS_EINVAL


def test_solve_options_are_validated():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    o = ms.solve_opts(precision=5)
    assert ms.lib.jacobi_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) == 0
    o = ms.solve_opts(precision=ms.MS_SOLVE_F32_REFINED, inner_eta=2.0)
    r = ms.SolveResult()
    rc = ms.lib.jacobi_solve(ctypes.byref(g), ctypes.byref(o), FAKE, None, FAKE2, 1 << 30, None,
                             ctypes.byref(r), None)
    assert rc == ms.MS_EINVAL
    o = ms.solve_opts()
    need = ms.lib.jacobi_workspace_bytes(ctypes.byref(g), ctypes.byref(o))
    assert need > 2 * (10 * 8 * 6 * 8)  # two extra FP64 buffers at least
    rc = ms.lib.jacobi_solve(ctypes.byref(g), ctypes.byref(o), FAKE, None, FAKE2, need - 1,
                             None, ctypes.byref(r), None)
    assert rc == ms.MS_EWORKSPACE


def test_advect_rejects_aliasing_outputs():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    p = [ctypes.c_void_p(0x100000 * (n + 1)) for n in range(8)]
    rc = ms.lib.advect_source(ctypes.byref(g), p[0], p[1], p[2], p[3], p[4], 0.25, 0.25, p[0],
                              p[5], p[6], None)
    assert rc == ms.MS_EINVAL


def test_tuning_table_round_trip_without_a_device():
    import paper_2310_01882_amd as ms
    ms.tuning_clear()
    e = dict(dtype=0, nx=64, ny=32, nz=16, vec_ok=2, vec=2, wx=1, rows=4, target_blocks=512,
             us_per_sweep=12.5)
    ms.tuning_load([e])
    assert ms.tuning_table() == [e]
    bad = dict(e, rows=3)
    with pytest.raises(ms.MsError):
        ms.tuning_load([bad])
    ms.tuning_clear()
    assert ms.tuning_table() == []


def test_batch_tuning_table_round_trip_without_a_device():
    import paper_2310_01882_amd as ms
    ms.batch_tuning_clear()
    e = dict(precision=ms.MS_SOLVE_F32_REFINED, nx=69, ny=240, nz=221, team=37, tx=32, zsplit=4,
             us_per_sweep=3.5)
    ms.batch_tuning_load([e])
    assert ms.batch_tuning_table() == [e]
    for bad in (dict(e, tx=48), dict(e, zsplit=3), dict(e, team=0), dict(e, precision=7)):
        with pytest.raises(ms.MsError):
            ms.batch_tuning_load([bad])
    assert ms.batch_tuning_table() == [e]  # a rejected load inserts nothing
    ms.batch_tuning_clear()
    assert ms.batch_tuning_table() == []


def test_sweep_shape_query_follows_the_tuning_table_and_alignment():
    import paper_2310_01882_amd as ms
    n, sy = 128, 160
    g = ms.Grid(n, n, n, 0, sy, sy * 130)
    base = 0x7F0000000000
    aligned = [base + k * (1 << 24) + 124 for k in range(4)]  # one float before 128 B

    def shape(ptrs):
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        out = ms.Tuning()
        assert ms.lib.ms_sweep_shape(ctypes.byref(g), ms.MS_F32, arr, len(ptrs),
                                     ctypes.byref(out)) == ms.MS_OK
        return out

    ms.tuning_clear()
    d = shape(aligned)
    assert d.vec_ok == 4 and d.us_per_sweep == 0.0  # untuned default
    e = dict(dtype=ms.MS_F32, nx=n, ny=n, nz=n, vec_ok=4, vec=1, wx=2, rows=2,
             target_blocks=1024, us_per_sweep=8.4)
    ms.tuning_load([e])
    t = shape(aligned)
    assert (t.vec, t.wx, t.rows, t.target_blocks, t.us_per_sweep) == (1, 2, 2, 1024, 8.4)
    # one buffer off the 16-byte phase: narrower lanes, a different table key
    m = shape(aligned[:3] + [aligned[3] + 4])
    assert m.vec_ok == 1 and m.us_per_sweep == 0.0
    ms.tuning_clear()


def test_red_black_and_solve_method_validation():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    assert ms.lib.rbgs_sweeps(ctypes.byref(g), 7, FAKE, FAKE2, None, 1, None, FAKE, 1 << 20,
                              None) == ms.MS_EUNSUPPORTED
    assert ms.lib.rbgs_sweeps(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, -1, None, FAKE,
                              1 << 20, None) == ms.MS_EINVAL
    assert ms.lib.rbgs_sweeps(ctypes.byref(g), ms.MS_F64, FAKE, FAKE, None, 1, None, FAKE,
                              1 << 20, None) == ms.MS_EINVAL  # u and u_tmp overlap
    o = ms.solve_opts(method=5)
    assert ms.lib.jacobi_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) == 0
    assert "method" in ms.last_error()
    assert ms.lib.jacobi_workspace_bytes(ctypes.byref(g),
                                         ctypes.byref(ms.solve_opts(method=ms.MS_METHOD_RBGS))) > 0


def test_streamed_sweeps_validation():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    ws = ms.lib.jacobi_sweeps_streamed_workspace_bytes
    assert ws(ctypes.byref(g), ms.MS_F64, 0, 4) == 0  # sweeps_per_pass < 1
    assert ws(ctypes.byref(g), ms.MS_F64, 2, 0) == 0  # slab_planes < 1
    need = ws(ctypes.byref(g), ms.MS_F64, 2, 2)
    # two sets of three slab buffers of S + 2T + 2 planes, plus partial tables
    assert need >= 2 * 3 * (2 + 4 + 2) * g.sz * 8
    assert ws(ctypes.byref(g), ms.MS_F32, 2, 2) < need
    call = ms.lib.jacobi_sweeps_streamed
    assert call(ctypes.byref(g), ms.MS_F64, FAKE, FAKE, None, 3, 2, 2, FAKE, need,
                None) == ms.MS_EINVAL  # u and u_tmp overlap
    assert call(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, 3, 2, 2, FAKE, need - 1,
                None) == ms.MS_EWORKSPACE
    assert call(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, -1, 2, 2, FAKE, need,
                None) == ms.MS_EINVAL


def test_stream_batch_validation():
    import paper_2310_01882_amd as ms
    arr = (ms.Instance * 2)()
    for n in range(2):
        arr[n].grid = _grid(ms)
        arr[n].x = 0x100000 * (n + 1)
    o = ms.solve_opts()
    ws = ms.lib.jacobi_batched_streams_workspace_bytes
    assert ws(2, arr, ctypes.byref(o), 0) == 0  # workers < 1
    one = ms.lib.jacobi_workspace_bytes(ctypes.byref(arr[0].grid), ctypes.byref(o))
    assert ws(2, arr, ctypes.byref(o), 4) >= 4 * one
    res = (ms.SolveResult * 2)()
    assert ms.lib.jacobi_solve_batched_streams(2, arr, ctypes.byref(o), 65, FAKE, 1 << 30, res,
                                               None) == ms.MS_EINVAL
    arr[1].x = arr[0].x  # overlapping instances
    assert ms.lib.jacobi_solve_batched_streams(2, arr, ctypes.byref(o), 2, FAKE, 1 << 30, res,
                                               None) == ms.MS_EINVAL
    assert ms.lib.jacobi_batched_plan_workspace_bytes(2) > 0
    assert ms.lib.jacobi_batched_plan_workspace_bytes(0) == 0


def test_warmstart_entry_points_validate_before_touching_a_device():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    assert ms.lib.warmstart_params_floats() == ms.lib.warmstart_layer_offset(4)
    assert ms.lib.warmstart_params_bytes() == 12 * ms.lib.warmstart_params_floats()
    # 63,169 real parameters, stored padded: 27*32*(8+32+32+32) weights + 4*32 biases
    assert ms.lib.warmstart_params_floats() == 27 * 32 * 104 + 128
    need = ms.lib.warmstart_workspace_bytes(ctypes.byref(g), 0)
    need_t = ms.lib.warmstart_workspace_bytes(ctypes.byref(g), 1)
    assert 0 < need < need_t
    P = [ctypes.c_void_p(0x1000000 * (n + 1)) for n in range(6)]
    fwd = ms.lib.warmstart_forward
    ok = dict(out_scale=4.0, smooth=4, rule=ms.MS_START_SLOW_MODES, work_bytes=need)

    def call(**kw):
        a = dict(ok, **kw)
        return fwd(ctypes.byref(g), P[0], P[1], P[2], a["out_scale"], a["smooth"], a["rule"],
                   P[3], P[4], a["work_bytes"], None, None, None)

    assert call(rule=7) == ms.MS_EINVAL
    assert call(smooth=3) == ms.MS_EINVAL
    assert call(smooth=66) == ms.MS_EINVAL
    assert call(out_scale=0.0) == ms.MS_EINVAL
    assert call(out_scale=float("inf")) == ms.MS_EINVAL
    assert call(work_bytes=need - 1) == ms.MS_EWORKSPACE
    # x overlapping f
    assert fwd(ctypes.byref(g), P[0], P[1], P[2], 4.0, 0, 0, ctypes.c_void_p(P[1].value + 8),
               P[4], need, None, None, None) == ms.MS_EINVAL
    step = ms.lib.warmstart_train_step
    assert step(ctypes.byref(g), P[0], P[1], P[2], P[3], 4.0, ctypes.c_float(0.0), 1, P[4], need_t,
                None, None) == ms.MS_EINVAL
    assert step(ctypes.byref(g), P[0], P[1], P[2], P[3], 4.0, ctypes.c_float(1e-3), 0, P[4],
                need_t, None, None) == ms.MS_EINVAL
    assert step(ctypes.byref(g), P[0], P[1], None, P[3], 4.0, ctypes.c_float(1e-3), 1, P[4],
                need_t, None, None) == ms.MS_EINVAL
    assert step(ctypes.byref(g), P[0], P[1], P[2], P[3], 4.0, ctypes.c_float(1e-3), 1, P[4],
                need, None, None) == ms.MS_EWORKSPACE
    assert ms.last_error()


def test_noalloc_sweeps_validate_and_report_their_scratch():
    import paper_2310_01882_amd as ms
    g = _grid(ms)
    assert ms.lib.jacobi_sweeps_noalloc_scratch_bytes() >= \
        ms.lib.jacobi_sweeps_workspace_bytes(ctypes.byref(g))
    assert ms.lib.jacobi_sweeps_noalloc(ctypes.byref(g), ms.MS_F64, FAKE, FAKE, None, 1, 1, None,
                                        None) == ms.MS_EINVAL
    assert ms.lib.jacobi_sweeps_noalloc(ctypes.byref(g), ms.MS_F64, FAKE, FAKE2, None, 1, 3, None,
                                        None) == ms.MS_EUNSUPPORTED
    assert ms.lib.jacobi_sweeps_noalloc(ctypes.byref(g), 9, FAKE, FAKE2, None, 1, 1, None,
                                        None) == ms.MS_EUNSUPPORTED
