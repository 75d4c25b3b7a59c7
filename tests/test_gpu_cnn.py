"""GPU warm-start kernels against the CNN oracle (BF16 inputs and weights,
FP32 accumulation on the device vs FP64 on the host)."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import dev, note, on_slab
from oracle import cnn

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402
from paper_2310_01882_amd import warmstart as wsm  # noqa: E402

X, Y, Z = 40, 6, 5  # x not a multiple of the 32-voxel wave tile


def _bf16_act(a, cpad):
    """[C, Z, Y, X] float array -> zero-haloed channels-last BF16 device tensor."""
    c, z, y, x = a.shape
    t = torch.zeros((z + 2, y + 2, x + 2, cpad), dtype=torch.float32)
    t[1:-1, 1:-1, 1:-1, :c] = torch.from_numpy(np.transpose(a, (1, 2, 3, 0)).copy())
    return t.to(torch.bfloat16).cuda().reshape(-1)


def _act_np(t, c, cpad, shape=(X, Y, Z)):
    x, y, z = shape
    a = t.float().view(z + 2, y + 2, x + 2, cpad)[1:-1, 1:-1, 1:-1, :c].cpu().numpy()
    return np.transpose(a, (3, 0, 1, 2)).astype(np.float64)


def _weights(cin, cinp, cout, seed, scale=0.2):
    w = np.zeros((27, 32, cinp), np.float32)
    w[:, :cout, :cin] = scale * synth.rng(seed).standard_normal((27, cout, cin))
    wf = torch.empty(27 * 32 * cinp, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty_like(wf)
    wt = torch.from_numpy(w).cuda()
    assert ms.lib.cnn_pack_weights(cinp, ms._ptr(wt), ms._ptr(wf), ms._ptr(wd), None) == 0
    return w, wf, wd


def _close(got, want, tol=1e-2):
    g, w = got.ravel(), want.ravel()
    cos = float(g @ w / (np.linalg.norm(g) * np.linalg.norm(w) + 1e-300))
    rel = float(np.linalg.norm(g - w) / (np.linalg.norm(w) + 1e-300))
    assert cos >= 0.999 and rel <= tol, (cos, rel)


@pytest.fixture(params=["row-blocked", "one-row", "lane-shifted"])
def conv_kernel(request, monkeypatch):
    """The 32-channel layers have the lane-shifted row kernels (default),
    the row-blocked ones (MS_CONV_SHIFT=0) and the one-row kernels
    (MS_CONV_ROWS=0); all are checked."""
    if request.param == "one-row":
        monkeypatch.setenv("MS_CONV_ROWS", "0")
    monkeypatch.setenv("MS_CONV_SHIFT", "1" if request.param == "lane-shifted" else "0")
    return request.param


@pytest.mark.parametrize("shape", [(70, 9, 3), (61, 13, 4), (30, 4, 2), (31, 5, 1),
                                   (64, 64, 40)])
def test_lane_shifted_conv_equals_row_blocked(shape, monkeypatch):
    """The lane-shifted kernels sum the same products in the same order as
    the row-blocked ones: forward (bias, ReLU, BF16 and FP32 outputs) and
    input gradient (ReLU mask) are equal bit for bit, on random BF16
    values and extents around the 30-voxel tile."""
    nx, ny, nz = shape
    note(f"case: lane-shifted conv {shape}")
    r = synth.rng(23)
    x = cnn.round_bf16(np.maximum(r.standard_normal((32, nz, ny, nx)), 0.0))
    g = cnn.round_bf16(r.standard_normal((32, nz, ny, nx)))
    w, wf, wd = _weights(32, 32, 32, 24)
    bt = torch.from_numpy((0.1 * r.standard_normal(32)).astype(np.float32)).cuda()
    xin, gin = _bf16_act(x, 32), _bf16_act(g, 32)
    res = []
    for shift in ("0", "1"):
        monkeypatch.setenv("MS_CONV_SHIFT", shift)
        out = torch.zeros_like(xin)
        out32 = torch.zeros((nz + 2, ny + 2, nx + 2), dtype=torch.float32, device="cuda")
        din = torch.zeros_like(xin)
        assert ms.lib.conv3d_bf16_fwd(nx, ny, nz, 32, ms._ptr(xin), ms._ptr(wf), ms._ptr(bt),
                                      ms._ptr(out), ms._ptr(out32), 1, None) == 0
        assert ms.lib.conv3d_bf16_dgrad(nx, ny, nz, 32, ms._ptr(gin), ms._ptr(wd),
                                        ms._ptr(xin), ms._ptr(din), None) == 0
        torch.cuda.synchronize()
        res.append((out.cpu(), out32.cpu(), din.cpu()))
    for a, b in zip(*res):
        assert torch.equal(a.view(torch.int16) if a.dtype == torch.bfloat16 else a,
                           b.view(torch.int16) if b.dtype == torch.bfloat16 else b)


@pytest.mark.parametrize("cin,cinp,relu", [(2, 8, True), (32, 32, True), (32, 32, False)])
def test_forward_conv_matches_oracle(cin, cinp, relu, conv_kernel):
    x = cnn.round_bf16(synth.rng(1).standard_normal((cin, Z, Y, X)))
    w, wf, wd = _weights(cin, cinp, 32, 2)
    b = (0.1 * synth.rng(3).standard_normal(32)).astype(np.float32)
    bt = torch.from_numpy(b).cuda()
    xin = _bf16_act(x, cinp)
    out = torch.zeros((Z + 2) * (Y + 2) * (X + 2) * 32, dtype=torch.bfloat16, device="cuda")
    out32 = torch.zeros((Z + 2, Y + 2, X + 2), dtype=torch.float32, device="cuda")
    rc = ms.lib.conv3d_bf16_fwd(X, Y, Z, cinp, ms._ptr(xin), ms._ptr(wf), ms._ptr(bt),
                                ms._ptr(out), ms._ptr(out32), int(relu), None)
    assert rc == 0
    torch.cuda.synchronize()
    wo = cnn.round_bf16(wsm.to_oracle_weights(w, cin, 32))
    ref = cnn.conv3d(x, wo, b.astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0.0)
    got = _act_np(out, 32, 32)
    # one BF16 rounding of an FP32 vs an FP64 sum: within 2^-8 relative
    assert np.all(np.abs(got - cnn.round_bf16(ref)) <= 2.0 ** -7 * np.abs(ref) + 1e-6)
    got32 = out32[1:-1, 1:-1, 1:-1].cpu().numpy().astype(np.float64)
    mag = cnn.conv3d(np.abs(x), np.abs(wo), np.abs(b.astype(np.float64)))[0]
    assert np.all(np.abs(got32 - ref[0]) <= 1e-5 * mag + 1e-7)
    # the halo of the output stays zero
    o = out.float().view(Z + 2, Y + 2, X + 2, 32)
    assert torch.all(o[0] == 0) and torch.all(o[:, :, -1] == 0)


@pytest.mark.parametrize("cin,cinp", [(2, 8), (32, 32)])
def test_dgrad_and_wgrad_match_oracle(cin, cinp, conv_kernel):
    r = synth.rng(4)
    x = cnn.round_bf16(np.maximum(r.standard_normal((cin, Z, Y, X)), 0.0))  # a ReLU output
    g = cnn.round_bf16(r.standard_normal((32, Z, Y, X)))
    w, wf, wd = _weights(cin, cinp, 32, 5)
    wo = cnn.round_bf16(wsm.to_oracle_weights(w, cin, 32))
    xin, gin = _bf16_act(x, cinp), _bf16_act(g, 32)
    din = torch.zeros_like(xin)
    assert ms.lib.conv3d_bf16_dgrad(X, Y, Z, cinp, ms._ptr(gin), ms._ptr(wd), ms._ptr(xin),
                                    ms._ptr(din), None) == 0
    dw = torch.zeros(27 * 32 * cinp, dtype=torch.float32, device="cuda")
    db = torch.zeros(32, dtype=torch.float32, device="cuda")
    work = torch.empty(ms.lib.conv3d_bf16_wgrad_workspace_bytes(cinp), dtype=torch.uint8,
                       device="cuda")
    assert ms.lib.conv3d_bf16_wgrad(X, Y, Z, cinp, ms._ptr(xin), ms._ptr(gin), ms._ptr(dw),
                                    ms._ptr(db), ms._ptr(work), work.numel(), None) == 0
    torch.cuda.synchronize()
    ref_dx = cnn.conv3d_dgrad(g, wo) * (x > 0)
    _close(_act_np(din, cin, cinp), ref_dx)
    ref_dw, ref_db = cnn.conv3d_wgrad(x, g)
    got_dw = wsm.to_oracle_weights(dw.cpu().numpy().reshape(27, 32, cinp), cin, 32)
    np.testing.assert_allclose(got_dw, ref_dw, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(db.cpu().numpy(), ref_db, rtol=1e-4, atol=1e-4)


def test_adam_matches_oracle():
    w, wf, wd = _weights(32, 32, 32, 6)
    wt = torch.from_numpy(w).cuda()
    b = torch.zeros(32, dtype=torch.float32, device="cuda")
    mw, vw = torch.zeros_like(wt), torch.zeros_like(wt)
    mb, vb = torch.zeros_like(b), torch.zeros_like(b)
    g1 = synth.rng(7).standard_normal(w.shape).astype(np.float32)
    g2 = synth.rng(8).standard_normal(w.shape).astype(np.float32)
    gb = torch.ones(32, dtype=torch.float32, device="cuda")
    pw, m, v = w.astype(np.float64), np.zeros(w.shape), np.zeros(w.shape)
    for t, g in ((1, g1), (2, g2)):
        gt = torch.from_numpy(g).cuda()
        assert ms.lib.cnn_adam(32, ms._ptr(wt), ms._ptr(b), ms._ptr(mw), ms._ptr(vw), ms._ptr(mb),
                               ms._ptr(vb), ms._ptr(gt), ms._ptr(gb), ms._ptr(wf), ms._ptr(wd),
                               ctypes.c_float(1e-3), t, None) == 0
        pw = cnn.adam_step(pw, g.astype(np.float64), m, v, t)
    np.testing.assert_allclose(wt.cpu().numpy(), pw, rtol=1e-5, atol=1e-7)
    # the BF16 copies are the rounded master weights, in both layouts
    assert np.array_equal(wf.float().cpu().numpy(), cnn.round_bf16(wt.cpu().numpy()).ravel())
    wdn = wd.float().cpu().numpy().reshape(27, 32, 32)
    assert np.array_equal(np.transpose(wdn, (0, 2, 1)), cnn.round_bf16(wt.cpu().numpy()))


@pytest.mark.parametrize("lds", ["1", "0"])
@pytest.mark.parametrize("shape", [(20, 12, 9), (70, 130, 3), (257, 5, 40)])
def test_features_match_oracle(shape, lds, monkeypatch):
    """The eight input channels against the oracle, with the box sums staged
    in LDS (default) and in global-memory form (MS_BOX_LDS=0); extents
    shorter than the largest half-width, rows past 256 (one row per round)
    and lines of other lengths per axis."""
    monkeypatch.setenv("MS_BOX_LDS", lds)
    nx, ny, nz = shape
    note(f"case: features {shape} lds={lds}")
    u = synth.dirichlet_uniform(nx, ny, nz, 3)
    f = synth.gaussian_sources(nx, ny, nz, 3, 4)
    net = wsm.WarmStart(nx, ny, nz, seed=1)
    net.features(dev(u), dev(f))
    want, s = cnn.features(u, f)
    assert net.scale.item() == s
    got = net.act_numpy(net.feat, 8)
    # f/s, g/s and the cube means: same FP64 operations in the same order
    for c in (0, 1, 2, 3, 4, 5, 7):
        assert np.array_equal(got[c], cnn.round_bf16(want[c])), c
    # phi: the device's sine may differ from numpy's in the last FP64 bit,
    # so the BF16 value may round one unit either way
    ulp = np.abs(cnn.round_bf16(want[6])) * 2.0 ** -7
    assert np.all(np.abs(got[6] - cnn.round_bf16(want[6])) <= ulp)


def test_full_network_step_matches_oracle():
    """Forward, loss gradient and every weight gradient of the whole network
    against the oracle's BF16-emulating network (cosine >= 0.999, relative
    L2 <= 1e-2)."""
    note("case: warm-start network step 33x10x8")
    nx, ny, nz = 33, 10, 8
    u = synth.dirichlet_uniform(nx, ny, nz, 5)
    f = synth.gaussian_sources(nx, ny, nz, 4, 6)
    target = synth.rng(7).standard_normal((nz, ny, nx)).astype(np.float32)
    net = wsm.WarmStart(nx, ny, nz, seed=11)
    params0 = net.params()
    du, df = dev(u), dev(f)
    tt = torch.zeros((nz + 2, ny + 2, nx + 2), dtype=torch.float32, device="cuda")
    tt[1:-1, 1:-1, 1:-1] = torch.from_numpy(target)
    out = net.forward(du, df)
    loss = net.backward(tt).sum().item() / (nx * ny * nz)
    torch.cuda.synchronize()
    feats, s = cnn.features(u, f)
    oparams = [(wsm.to_oracle_weights(w, cin, cout), b[:cout].astype(np.float64))
               for (w, b), (cin, _, cout, _) in zip(params0, wsm.LAYERS)]
    onet = cnn.Net(oparams, bf16=True)
    ref = onet.forward(feats)[0]
    _close(out[1:-1, 1:-1, 1:-1].cpu().numpy().astype(np.float64), ref)
    ref_loss, gout = cnn.mse_and_grad(ref, target.astype(np.float64))
    assert loss == pytest.approx(ref_loss, rel=1e-2)
    grads = onet.backward(gout[None])
    for li, ((cin, cinp, cout, _), (gw, gb)) in enumerate(zip(wsm.LAYERS, grads)):
        got_w = wsm.to_oracle_weights(net.gw[li].cpu().numpy(), cin, cout)
        _close(got_w, gw, tol=3e-2)
        _close(net.gb[li].cpu().numpy()[:cout].astype(np.float64), gb, tol=3e-2)


def test_training_reduces_the_loss_on_one_instance():
    nx, ny, nz = 32, 32, 16
    u = synth.zeros(nx, ny, nz)
    f = synth.gaussian_sources(nx, ny, nz, 3, 9)
    du, df = dev(u), dev(f)
    x = dev(u)
    ms.jacobi_solve(x, df, rel_tol=1e-8)
    net = wsm.WarmStart(nx, ny, nz, seed=2)
    losses = [net.train_step(du, df, x, lr=3e-3).item() for _ in range(60)]
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.parametrize("shape", [(70, 9, 3), (61, 13, 4), (31, 5, 1), (30, 4, 2)])
def test_first_layer_lane_shifted_forward_on_ragged_extents(shape, monkeypatch):
    """The 8-channel forward in its lane-shifted form (pairs of z taps per
    MFMA, dx from the neighbouring lanes) on extents around its 30 x 4
    tile, against the oracle; inputs, weights and bias are k/8, so every
    sum is exact in FP32 and the BF16 outputs equal the oracle's rounded
    values bit for bit."""
    nx, ny, nz = shape
    monkeypatch.setenv("MS_CONV_SHIFT", "1")
    note(f"case: first-layer lane-shifted forward {shape}")
    r = synth.rng(29)
    x = r.integers(-7, 8, (8, nz, ny, nx)).astype(np.float32) / 8
    w = r.integers(-7, 8, (27, 32, 8)).astype(np.float32) / 8
    b = r.integers(-7, 8, 32).astype(np.float32) / 8
    wt = torch.from_numpy(w).cuda()
    wf = torch.empty(27 * 32 * 8, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty_like(wf)
    assert ms.lib.cnn_pack_weights(8, ms._ptr(wt), ms._ptr(wf), ms._ptr(wd), None) == 0
    bt = torch.from_numpy(b).cuda()
    xin = _bf16_act(x, 8)
    out = torch.zeros((nz + 2) * (ny + 2) * (nx + 2) * 32, dtype=torch.bfloat16, device="cuda")
    assert ms.lib.conv3d_bf16_fwd(nx, ny, nz, 8, ms._ptr(xin), ms._ptr(wf), ms._ptr(bt),
                                  ms._ptr(out), None, 1, None) == 0
    torch.cuda.synchronize()
    wo = wsm.to_oracle_weights(w, 8, 32)
    ref = np.maximum(cnn.conv3d(x.astype(np.float64), wo, b.astype(np.float64)), 0.0)
    assert np.array_equal(_act_np(out, 32, 32, (nx, ny, nz)), cnn.round_bf16(ref))
    o = out.float().view(nz + 2, ny + 2, nx + 2, 32)
    assert torch.all(o[:, -1] == 0) and torch.all(o[:, :, -1] == 0) and torch.all(o[-1] == 0)


@pytest.mark.parametrize("shift", ["0", "1"])
def test_row_blocked_conv_on_ragged_extents(shift, monkeypatch):
    """x not a multiple of 32 (nor of 30) and y not a multiple of the 4-row
    block, both directions, both row-kernel forms, against the oracle."""
    monkeypatch.setenv("MS_CONV_SHIFT", shift)
    nx, ny, nz = 70, 9, 3
    r = synth.rng(11)
    x = cnn.round_bf16(np.maximum(r.standard_normal((32, nz, ny, nx)), 0.0))
    g = cnn.round_bf16(r.standard_normal((32, nz, ny, nx)))
    w, wf, wd = _weights(32, 32, 32, 12)
    wo = cnn.round_bf16(wsm.to_oracle_weights(w, 32, 32))
    b = torch.zeros(32, dtype=torch.float32, device="cuda")
    xin, gin = _bf16_act(x, 32), _bf16_act(g, 32)
    out = torch.zeros_like(xin)
    din = torch.zeros_like(xin)
    assert ms.lib.conv3d_bf16_fwd(nx, ny, nz, 32, ms._ptr(xin), ms._ptr(wf), ms._ptr(b),
                                  ms._ptr(out), None, 0, None) == 0
    assert ms.lib.conv3d_bf16_dgrad(nx, ny, nz, 32, ms._ptr(gin), ms._ptr(wd), ms._ptr(xin),
                                    ms._ptr(din), None) == 0
    torch.cuda.synchronize()
    shape = (nx, ny, nz)
    ref = cnn.conv3d(x, wo, np.zeros(32))
    mag = cnn.conv3d(np.abs(x), np.abs(wo), np.zeros(32))
    got = _act_np(out, 32, 32, shape)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 2e-5 * mag)
    _close(_act_np(din, 32, 32, shape), cnn.conv3d_dgrad(g, wo) * (x > 0))
    # halos stay zero
    o = out.float().view(nz + 2, ny + 2, nx + 2, 32)
    assert torch.all(o[:, -1] == 0) and torch.all(o[:, :, -1] == 0) and torch.all(o[-1] == 0)


@pytest.mark.parametrize("cin,cinp", [(2, 8), (32, 32)])
@pytest.mark.parametrize("shape", [(70, 9, 3), (64, 64, 40)])
def test_row_blocked_wgrad(shape, cin, cinp, monkeypatch):
    """Weight gradient of the first layer (2 channels padded to 8) and of a
    32-channel layer: x past a 32-voxel task and y past a 4-row task
    (70 x 9 x 3), and a volume with several tasks per block (64 x 64 x 40:
    1280 tasks over 512 blocks), against the oracle. The output-gradient halo
    holds nonzero values, which must not enter the sums. A second call gives
    the same bits (fixed reduction order), also when the 32-channel kernel
    reads its operands element by element instead of through the
    transposing LDS reads (MS_WGRAD_TR=0: the same operand values)."""
    nx, ny, nz = shape
    r = synth.rng(13)
    x = cnn.round_bf16(np.maximum(r.standard_normal((cin, nz, ny, nx)), 0.0))
    g = cnn.round_bf16(r.standard_normal((32, nz, ny, nx)))
    xin = _bf16_act(x, cinp)
    gh = torch.full((nz + 2, ny + 2, nx + 2, 32), 3.0, dtype=torch.float32)
    gh[1:-1, 1:-1, 1:-1] = torch.from_numpy(np.transpose(g, (1, 2, 3, 0)).copy())
    gin = gh.to(torch.bfloat16).cuda().reshape(-1)
    work = torch.empty(ms.lib.conv3d_bf16_wgrad_workspace_bytes(cinp), dtype=torch.uint8,
                       device="cuda")
    res = []
    for tr in ("1", "0"):
        monkeypatch.setenv("MS_WGRAD_TR", tr)
        dw = torch.zeros(27 * 32 * cinp, dtype=torch.float32, device="cuda")
        db = torch.zeros(32, dtype=torch.float32, device="cuda")
        assert ms.lib.conv3d_bf16_wgrad(nx, ny, nz, cinp, ms._ptr(xin), ms._ptr(gin),
                                        ms._ptr(dw), ms._ptr(db), ms._ptr(work), work.numel(),
                                        None) == 0
        torch.cuda.synchronize()
        res.append((dw.cpu().numpy(), db.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    ref_dw, ref_db = cnn.conv3d_wgrad(x, g)
    mag_dw, mag_db = cnn.conv3d_wgrad(np.abs(x), np.abs(g))
    dwp = res[0][0].reshape(27, 32, cinp)
    assert np.all(dwp[:, :, cin:] == 0)  # zero input channels get zero gradients
    got_dw = wsm.to_oracle_weights(dwp, cin, 32)
    # BF16 products are exact in FP32; only the FP32 sums round
    assert np.all(np.abs(got_dw - ref_dw) <= 1e-5 * mag_dw + 1e-6)
    assert np.all(np.abs(res[0][1] - ref_db) <= 1e-5 * mag_db + 1e-6)


@pytest.mark.parametrize("cin,cinp", [(2, 8), (32, 32)])
def test_wgrad_at_full_size_on_sampled_outputs(cin, cinp):
    """Weight gradient at 128^3, the warm start's working size, in the launch
    the benchmarks time (16384 tasks over 512 blocks), against the oracle on
    output channels 0..3 x input channels 0..3 (an entry depends on its two
    channels alone, so the oracle runs on those). Inputs are k/8 with
    |k| <= 7: every product is a multiple of 1/64 and every partial sum stays
    far below 2^17, so FP32 sums in any order are exact and the gradients
    must equal the oracle's bit for bit."""
    n, co = 128, 4
    note(f"case: weight gradient 128^3 cin={cinp}")
    r = synth.rng(17)
    x = np.maximum(r.integers(-7, 8, (cin, n, n, n), dtype=np.int8), 0).astype(np.float32) / 8
    g = r.integers(-7, 8, (32, n, n, n), dtype=np.int8).astype(np.float32) / 8
    xin, gin = _bf16_act(x, cinp), _bf16_act(g, 32)
    dw = torch.zeros(27 * 32 * cinp, dtype=torch.float32, device="cuda")
    db = torch.zeros(32, dtype=torch.float32, device="cuda")
    work = torch.empty(ms.lib.conv3d_bf16_wgrad_workspace_bytes(cinp), dtype=torch.uint8,
                       device="cuda")
    assert ms.lib.conv3d_bf16_wgrad(n, n, n, cinp, ms._ptr(xin), ms._ptr(gin), ms._ptr(dw),
                                    ms._ptr(db), ms._ptr(work), work.numel(), None) == 0
    torch.cuda.synchronize()
    del xin, gin
    ci = min(cin, 4)
    ref_dw, ref_db = cnn.conv3d_wgrad(x[:ci].astype(np.float64), g[:co].astype(np.float64))
    dwp = dw.cpu().numpy().reshape(27, 32, cinp)
    assert np.all(dwp[:, :, cin:] == 0)
    got_dw = wsm.to_oracle_weights(dwp, cin, 32)[:co, :ci]
    assert np.array_equal(got_dw, ref_dw)
    assert np.array_equal(db.cpu().numpy()[:co].astype(np.float64), ref_db)


@pytest.mark.parametrize("cin,cinp,shift", [(2, 8, "0"), (8, 8, "1"), (32, 32, "0"),
                                            (32, 32, "1")])
def test_forward_and_input_gradient_at_full_size(cin, cinp, shift, monkeypatch):
    """Forward (bias, ReLU, BF16 and FP32 outputs) and input gradient (ReLU
    mask) at 128^3 in the launch the benchmarks time, against the oracle on
    every channel of the z planes 0-1, 63-64 and 126-127 (the oracle runs on
    the planes those outputs read). Inputs, weights and biases are k/8
    (|k| <= 7): a sum of 27 x cin such products is exact in FP32, so the
    BF16 outputs must equal the oracle's rounded values bit for bit and the
    FP32 output its exact value."""
    n = 128
    monkeypatch.setenv("MS_CONV_SHIFT", shift)
    note(f"case: forward and input gradient 128^3 cin={cinp} shift={shift}")
    r = synth.rng(19)
    x = np.maximum(r.integers(-7, 8, (cin, n, n, n), dtype=np.int8), 0).astype(np.float32) / 8
    g = r.integers(-7, 8, (32, n, n, n), dtype=np.int8).astype(np.float32) / 8
    w = np.zeros((27, 32, cinp), np.float32)
    w[:, :, :cin] = r.integers(-7, 8, (27, 32, cin)).astype(np.float32) / 8
    b = r.integers(-7, 8, 32).astype(np.float32) / 8
    wt = torch.from_numpy(w).cuda()
    wf = torch.empty(27 * 32 * cinp, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty_like(wf)
    assert ms.lib.cnn_pack_weights(cinp, ms._ptr(wt), ms._ptr(wf), ms._ptr(wd), None) == 0
    bt = torch.from_numpy(b).cuda()
    xin, gin = _bf16_act(x, cinp), _bf16_act(g, 32)
    out = torch.zeros((n + 2) ** 3 * 32, dtype=torch.bfloat16, device="cuda")
    out32 = torch.zeros((n + 2, n + 2, n + 2), dtype=torch.float32, device="cuda")
    din = torch.zeros_like(xin)
    assert ms.lib.conv3d_bf16_fwd(n, n, n, cinp, ms._ptr(xin), ms._ptr(wf), ms._ptr(bt),
                                  ms._ptr(out), ms._ptr(out32), 1, None) == 0
    assert ms.lib.conv3d_bf16_dgrad(n, n, n, cinp, ms._ptr(gin), ms._ptr(wd), ms._ptr(xin),
                                    ms._ptr(din), None) == 0
    torch.cuda.synchronize()
    shape = (n, n, n)
    got = _act_np(out, 32, 32, shape)
    got32 = out32[1:-1, 1:-1, 1:-1].cpu().numpy().astype(np.float64)
    got_din = _act_np(din, cin, cinp, shape)
    del xin, gin, out, out32, din
    wo = wsm.to_oracle_weights(w, cin, 32)
    b64 = b.astype(np.float64)
    for z0 in (0, 63, 126):
        ref = on_slab(lambda a: np.maximum(cnn.conv3d(a, wo, b64), 0.0), [x], z0, 2, n)
        assert np.array_equal(got[:, z0:z0 + 2], cnn.round_bf16(ref)), z0
        assert np.array_equal(got32[z0:z0 + 2], ref[0]), z0
        ref_din = on_slab(lambda gg, xx: cnn.conv3d_dgrad(gg, wo) * (xx > 0), [g, x], z0, 2,
                           n)
        assert np.array_equal(got_din[:, z0:z0 + 2], cnn.round_bf16(ref_din)), z0
