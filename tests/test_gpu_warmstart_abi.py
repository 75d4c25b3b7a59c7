"""The learned warm start through its two C-ABI entry points
(warmstart_forward, warmstart_train_step) against the CNN oracle: the guess
(features, network, scaling), the start selection under each rule with its
four FP64 measures, and one training step (loss, and the direction of every
well-determined Adam update). Also: the training step is bit-identical to
the same kernels driven one by one."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from gpuhelp import host, note
from oracle import cnn

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402
from paper_2310_01882_amd import warmstart as wsm  # noqa: E402

NX, NY, NZ = 33, 10, 8
RULES = ("residual", "slow_modes", "force")


def _problem(seed):
    u = synth.dirichlet_uniform(NX, NY, NZ, seed)
    u[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((NZ, NY, NX))  # never read
    f = synth.gaussian_sources(NX, NY, NZ, 3, seed + 2)
    return u, f


def _oracle_net(params):
    return cnn.Net([(wsm.to_oracle_weights(w, cin, cout), b[:cout].astype(np.float64))
                    for (w, b), (cin, _, cout, _) in zip(params, wsm.LAYERS)], bf16=True)


def _close(got, want, tol=1e-2):
    g, w = got.ravel(), want.ravel()
    cos = float(g @ w / (np.linalg.norm(g) * np.linalg.norm(w) + 1e-300))
    rel = float(np.linalg.norm(g - w) / (np.linalg.norm(w) + 1e-300))
    assert cos >= 0.999 and rel <= tol, (cos, rel)


def test_forward_guess_matches_the_oracle_network():
    note("case: warmstart_forward guess 33x10x8")
    u, f = _problem(3)
    net = wsm.WarmStart(NX, NY, NZ, seed=5, out_scale=2.5)
    du, df = ms.field_from(u), ms.field_from(f)
    x = ms.field_from(u)
    used, meas = net.guess(du, df, x, rule="force", smooth=0)
    torch.cuda.synchronize()
    assert used.item() == 1
    feats, s = cnn.features(u, f)
    want = s * 2.5 * _oracle_net(net.params()).forward(feats)[0]
    got = host(x)
    _close(got[1:-1, 1:-1, 1:-1], want)
    # the halo is the Dirichlet data, untouched
    mask = np.ones(got.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(got[mask], u[mask])


@pytest.mark.parametrize("smooth", [2, 4, 8])
def test_guess_smoothing_bit_exact(smooth):
    """The damped sweeps on the guess equal the oracle's smoother applied to
    the device's unsmoothed guess, bit for bit (FP64, same order)."""
    u, f = _problem(5)
    net = wsm.WarmStart(NX, NY, NZ, seed=6, out_scale=2.0)
    du, df = ms.field_from(u), ms.field_from(f)
    x0, xs = ms.field_from(u), ms.field_from(u)
    net.guess(du, df, x0, rule="force", smooth=0)
    net.guess(du, df, xs, rule="force", smooth=smooth)
    torch.cuda.synchronize()
    want = cnn.smooth_guess(host(x0), f, smooth)
    assert np.array_equal(host(xs), want)


@pytest.mark.parametrize("beta_at", [0.0, 0.5, 3.0, None])
def test_start_selection_matches_the_oracle(beta_at):
    """Zero weights and a last-layer bias beta make the network output beta
    exactly, so the guess is the constant s * out_scale * beta (chosen as
    0, the halo's mean, a large value); None keeps random weights. Every
    rule's decision and the four measures are compared with the oracle's on
    the guess the device produced."""
    u, f = _problem(11)
    net = wsm.WarmStart(NX, NY, NZ, seed=7, out_scale=1.0)
    feats, s = cnn.features(u, f)
    if beta_at is not None:
        params = [(np.zeros_like(w), np.zeros_like(b)) for w, b in net.params()]
        params[3][1][0] = np.float32(beta_at / s)
        net.set_params(params)
    du, df = ms.field_from(u), ms.field_from(f)
    xg = ms.field_from(u)
    smooth = 0 if beta_at is not None else 4  # constant guesses stay constant
    net.guess(du, df, xg, rule="force", smooth=smooth)
    guess = host(xg)[1:-1, 1:-1, 1:-1]
    seen = set()
    for rule in RULES:
        note(f"case: start selection {rule}, beta {beta_at}")
        x = ms.field_from(u)
        used, meas = net.guess(du, df, x, rule=rule, smooth=smooth)
        torch.cuda.synchronize()
        want_use, want_meas = cnn.start_choice(u, f, guess, rule)
        assert bool(used.item()) == want_use, (rule, host(meas), want_meas)
        np.testing.assert_allclose(host(meas), want_meas, rtol=1e-10,
                                   atol=1e-12 * max(want_meas))
        got = host(x)
        if want_use:
            assert np.array_equal(got[1:-1, 1:-1, 1:-1], guess)
        else:
            assert not np.any(got[1:-1, 1:-1, 1:-1])
        assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
        seen.add(want_use)
    if beta_at == 0.0:
        assert seen == {False, True}  # only "force" keeps the zero guess


def test_guess_written_in_place_of_u():
    u, f = _problem(13)
    net = wsm.WarmStart(NX, NY, NZ, seed=9)
    du, df = ms.field_from(u), ms.field_from(f)
    x = ms.field_from(u)
    net.guess(du, df, x, rule="force", smooth=4)
    net.guess(du, df, du, rule="force", smooth=4)  # x = u
    torch.cuda.synchronize()
    assert np.array_equal(host(du), host(x))


def test_train_step_matches_the_oracle():
    note("case: warmstart_train_step 33x10x8")
    u, f = _problem(17)
    solved = synth.zeros(NX, NY, NZ)
    solved[1:-1, 1:-1, 1:-1] = synth.rng(19).standard_normal((NZ, NY, NX))
    net = wsm.WarmStart(NX, NY, NZ, seed=21, out_scale=0.5)
    p0 = net.params()
    du, df, ds = ms.field_from(u), ms.field_from(f), ms.field_from(solved)
    lr = 1e-3
    loss = net.train_step(du, df, ds, lr=lr).item()
    p1 = net.params()
    feats, s = cnn.features(u, f)
    onet = _oracle_net(p0)
    pred = onet.forward(feats)[0]
    target = (solved[1:-1, 1:-1, 1:-1] / (s * 0.5)).astype(np.float32).astype(np.float64)
    want_loss, gout = cnn.mse_and_grad(pred, target)
    assert loss == pytest.approx(want_loss, rel=1e-2)
    grads = onet.backward(gout[None])
    # Adam's first step moves every parameter by lr * g / (|g| + eps): the
    # sign of the oracle's gradient wherever it is well above BF16 noise, and
    # that size (up to the FP32 rounding of the weights, ~1e-7 absolute)
    for li, ((cin, _, cout, _), (gw, gb)) in enumerate(zip(wsm.LAYERS, grads)):
        dw = wsm.to_oracle_weights(p1[li][0] - p0[li][0], cin, cout)
        db = (p1[li][1] - p0[li][1])[:cout].astype(np.float64)
        for d, g in ((dw, gw), (db, gb)):
            big = np.abs(g) > 0.05 * np.abs(g).max()
            assert np.array_equal(np.sign(d[big]), -np.sign(g[big])), li
            want = lr * np.abs(g[big]) / (np.abs(g[big]) + 1e-8)
            np.testing.assert_allclose(np.abs(d[big]), want, rtol=1e-3, atol=3e-7)
        # padded channels stay zero
        w1 = p1[li][0]
        assert not np.any(w1[:, cout:, :]) and not np.any(w1[:, :, cin:])


def test_train_step_equals_the_kernels_one_by_one():
    """The entry point runs the same kernels in the same order as the
    layer-by-layer path (features, forward, target, loss gradient, weight and
    input gradients, Adam): parameters and loss come out bit-identical, over
    three steps."""
    u, f = _problem(23)
    solved = synth.zeros(NX, NY, NZ)
    solved[1:-1, 1:-1, 1:-1] = synth.rng(29).standard_normal((NZ, NY, NX))
    du, df, ds = ms.field_from(u), ms.field_from(f), ms.field_from(solved)
    a = wsm.WarmStart(NX, NY, NZ, seed=31)
    b = wsm.WarmStart(NX, NY, NZ, seed=31)
    for t in range(1, 4):
        la = a.train_step(du, df, ds, lr=2e-3).item()
        b.forward(du, df)
        tgt = b.target(ds)
        parts = b.backward(tgt)
        lb = parts.sum().item() / (NX * NY * NZ)
        for li, (_, cinp, _, _) in enumerate(wsm.LAYERS):
            assert ms.lib.cnn_adam(cinp, ms._ptr(b.w[li]), ms._ptr(b.b[li]), ms._ptr(b.mw[li]),
                                   ms._ptr(b.vw[li]), ms._ptr(b.mb[li]), ms._ptr(b.vb[li]),
                                   ms._ptr(b.gw[li]), ms._ptr(b.gb[li]), ms._ptr(b.wf[li]),
                                   ms._ptr(b.wd[li]), ctypes.c_float(2e-3), t, None) == 0
        torch.cuda.synchronize()
        assert la == pytest.approx(lb, rel=1e-12)
        for (wa, ba), (wb, bb) in zip(a.params(), b.params()):
            assert np.array_equal(wa, wb) and np.array_equal(ba, bb)
