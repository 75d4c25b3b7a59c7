"""Pins of the CNN oracle: library convolution, exact special cases, finite
differences for the backward pass, Adam's closed form on a constant gradient
at every step, the MSE loss and its gradient (closed form, scikit-learn,
finite differences), BF16 rounding of known values, and the boundary lift."""

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from oracle import cnn


def _rand(shape, seed):
    return synth.rng(seed).standard_normal(shape)


def test_conv3d_equals_scipy_correlate():
    x = _rand((3, 5, 6, 7), 1)
    w = _rand((2, 3, 3, 3, 3), 2)
    b = _rand(2, 3)
    got = cnn.conv3d(x, w, b)
    for co in range(2):
        want = sum(ndimage.correlate(x[ci], w[co, ci], mode="constant", cval=0.0)
                   for ci in range(3)) + b[co]
        np.testing.assert_allclose(got[co], want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [(1, 0, 0), (0, -1, 0), (0, 0, 1), (-1, 1, -1), (0, 0, 0)])
def test_delta_kernel_is_an_exact_shift(d):
    x = _rand((1, 4, 5, 6), 4)
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, d[2] + 1, d[1] + 1, d[0] + 1] = 1.0
    got = cnn.conv3d(x, w)[0]
    xp = np.pad(x[0], 1)
    dx, dy, dz = d
    want = xp[1 + dz:5 + dz, 1 + dy:6 + dy, 1 + dx:7 + dx]
    assert np.array_equal(got, want)


def test_zero_kernel_gives_the_bias():
    x = _rand((2, 3, 3, 3), 5)
    out = cnn.conv3d(x, np.zeros((4, 2, 3, 3, 3)), np.arange(4.0))
    for co in range(4):
        assert np.all(out[co] == co)


def _tiny_net(seed):
    r = synth.rng(seed)
    shapes = [(4, 2), (4, 4), (1, 4)]
    return [(0.3 * r.standard_normal((co, ci, 3, 3, 3)), 0.1 * r.standard_normal(co))
            for co, ci in shapes]


def test_backward_matches_central_finite_differences():
    params = _tiny_net(6)
    x = _rand((2, 6, 6, 6), 7)
    gout = _rand((1, 6, 6, 6), 8)

    def loss(ps):
        return float(np.sum(gout * cnn.Net(ps, bf16=False).forward(x)))

    net = cnn.Net(params, bf16=False)
    net.forward(x)
    grads = net.backward(gout)
    r = synth.rng(9)
    eps = 1e-6
    for li in range(3):
        w, b = params[li]
        for _ in range(4):
            idx = tuple(int(r.integers(0, s)) for s in w.shape)
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[li][0][idx] += eps
            wm[li][0][idx] -= eps
            fd = (loss(wp) - loss(wm)) / (2 * eps)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-7)
        j = int(r.integers(0, b.shape[0]))
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[li][1][j] += eps
        bm[li][1][j] -= eps
        fd = (loss(bp) - loss(bm)) / (2 * eps)
        assert grads[li][1][j] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_dgrad_matches_finite_differences_of_the_input():
    x = _rand((3, 4, 5, 4), 10)
    w = _rand((2, 3, 3, 3, 3), 11)
    g = _rand((2, 4, 5, 4), 12)
    dx = cnn.conv3d_dgrad(g, w)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 1), (2, 3, 4, 3), (0, 1, 0, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (np.sum(g * cnn.conv3d(xp, w)) - np.sum(g * cnn.conv3d(xm, w))) / (2 * eps)
        assert dx[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 0.0, 1e-3])
    m, v = np.zeros(4), np.zeros(4)
    lr, eps = 1e-3, 1e-8
    out = cnn.adam_step(p, g, m, v, 1, lr=lr, eps=eps)
    # first step: mhat = g, vhat = g^2, so the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(out, p - lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_bf16_rounding_of_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 1 + 2 ** -7, 3.0e38, 0.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, -2.5, 1 + 2 ** -7, 1.765625 * 2.0 ** 127, 0.0])
    got = cnn.round_bf16(vals)
    assert np.array_equal(got, want)
    assert got[1] == 1.0 and got[2] == 1 + 2 ** -6  # ties to even, exactly


def test_boundary_lift_counts_dirichlet_neighbours():
    u = np.full((6, 5, 4), 2.0)  # interior 4 x 3 x 2, halo value 2
    g = cnn.boundary_lift(u)
    assert g.shape == (4, 3, 2)
    # every interior cell of this thin grid touches the halo on several sides
    assert g[0, 0, 0] == 3 * 2.0  # corner: -x, -y, -z neighbours are halo
    assert g[1, 1, 0] == 2.0  # middle of z and y: only -x is halo
    assert g[3, 2, 1] == 3 * 2.0  # opposite corner: +x, +y, +z are halo
    # consistency with the stencil: S(u with zero interior) = g
    z = oracle.zero_interior(synth.dirichlet_uniform(5, 4, 3, 1))
    assert np.allclose(oracle.neighbour_sum(z), cnn.boundary_lift(z), rtol=0, atol=0)


def test_features_scale_free():
    u = synth.dirichlet_uniform(6, 5, 4, 2)
    f = synth.gaussian_sources(6, 5, 4, 3, 3)
    a, s1 = cnn.features(u, f)
    b, s2 = cnn.features(3 * u, 3 * f)
    assert s2 == pytest.approx(3 * s1)
    np.testing.assert_allclose(a, b, rtol=1e-14)
    assert np.max(np.abs(a)) == pytest.approx(1.0)


def test_slab_evaluation_equals_the_whole_volume():
    """The full-size GPU tests evaluate the convolutions on the planes a few
    output planes read; that equals the whole-volume evaluation there, at
    the bottom, in the middle and at the top."""
    from gpuhelp import on_slab

    r = synth.rng(23)
    x = r.standard_normal((3, 9, 5, 6))
    g = r.standard_normal((4, 9, 5, 6))
    w = r.standard_normal((4, 3, 3, 3, 3))
    b = r.standard_normal(4)
    full = cnn.conv3d(x, w, b)
    fulld = cnn.conv3d_dgrad(g, w)
    for z0 in (0, 3, 7):
        assert np.array_equal(on_slab(lambda a: cnn.conv3d(a, w, b), [x], z0, 2, 9),
                              full[:, z0:z0 + 2])
        assert np.array_equal(on_slab(lambda a: cnn.conv3d_dgrad(a, w), [g], z0, 2, 9),
                              fulld[:, z0:z0 + 2])


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.75)])
def test_adam_constant_gradient_closed_form_every_step(b1, b2):
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so
    each step moves p by lr * g / (|g| + eps): p_t = p_0 - t lr g / (|g| + eps)."""
    p0 = np.array([1.0, -2.0, 0.5, 3.0, -0.25])
    g = np.array([0.3, -4.0, 2.5e-2, 1e-3, -7.0])
    m, v = np.zeros(5), np.zeros(5)
    lr, eps = 1e-2, 1e-8
    p = p0.copy()
    for t in range(1, 7):
        p = cnn.adam_step(p, g, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-13)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_adam_first_moment_decays_after_the_gradient_stops():
    """After one step with gradient g and t - 1 steps with zero gradient,
    m_t = (1 - b1) b1^(t-1) g and v_t = (1 - b2) b2^(t-1) g^2, so the step
    at t is lr * m_t/(1 - b1^t) / (sqrt(v_t/(1 - b2^t)) + eps), written
    here with the powers expanded by hand for t = 3."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 0.0
    g = np.array([2.0, -0.5])
    m, v = np.zeros(2), np.zeros(2)
    p = cnn.adam_step(np.zeros(2), g, m, v, 1, lr=lr, b1=b1, b2=b2, eps=eps)
    p = cnn.adam_step(p, np.zeros(2), m, v, 2, lr=lr, b1=b1, b2=b2, eps=eps)
    before = p.copy()
    p = cnn.adam_step(p, np.zeros(2), m, v, 3, lr=lr, b1=b1, b2=b2, eps=eps)
    mhat = 0.1 * 0.81 * g / (1 - 0.729)
    vhat = 0.001 * 0.998001 * g * g / (1 - 0.997002999)
    np.testing.assert_allclose(before - p, lr * mhat / np.sqrt(vhat), rtol=1e-12)


def test_mse_closed_form_on_a_constant_offset():
    """pred = target + c on N voxels: loss c^2, gradient 2c/N everywhere."""
    r = synth.rng(31)
    target = r.standard_normal((4, 5, 6))
    for c in (0.75, -3.0):
        loss, grad = cnn.mse_and_grad(target + c, target)
        assert loss == pytest.approx(c * c, rel=1e-14)
        np.testing.assert_allclose(grad, np.full(target.shape, 2 * c / target.size), rtol=1e-12)


def test_mse_gradient_matches_central_finite_differences():
    r = synth.rng(32)
    pred = r.standard_normal((3, 4, 5))
    target = r.standard_normal((3, 4, 5))
    loss, grad = cnn.mse_and_grad(pred, target)
    from sklearn.metrics import mean_squared_error
    assert loss == pytest.approx(mean_squared_error(target.ravel(), pred.ravel()), rel=1e-13)
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (2, 3, 4), (0, 3, 1)]:
        pp, pm = pred.copy(), pred.copy()
        pp[idx] += eps
        pm[idx] -= eps
        fd = (cnn.mse_and_grad(pp, target)[0] - cnn.mse_and_grad(pm, target)[0]) / (2 * eps)
        assert grad[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)
