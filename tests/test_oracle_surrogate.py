"""Pins of the surrogate oracle (oracle/surrogate.py) against facts that do
not come from the oracle itself: a library's bfloat16 rounding, finite
differences, closed forms of special networks and of Adam, and the plain
method's own regions."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as S
import synth

torch = pytest.importorskip("torch")


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 65504.0]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(v), ref)
    # halfway cases go to the even mantissa
    assert S.bf16(1 + 2 ** -8) == 1.0
    assert S.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_silu_and_its_derivative():
    z = np.linspace(-12, 12, 97)
    h = 1e-6
    fd = (S.silu(z + h) - S.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - S.dsilu(z))) < 1e-8
    assert S.silu(0.0) == 0.0
    assert abs(S.silu(40.0) - 40.0) < 1e-15 * 40
    assert abs(S.silu(-40.0) + 40.0 * np.exp(-40.0)) < 1e-30
    assert S.dsilu(0.0) == 0.5


def small_batch(n=48, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 50, n)
    y = 10.0 ** rng.uniform(-4, 2, n)
    return x, y


@pytest.mark.parametrize("wscale", [0.0, 1.5])
def test_gradient_matches_finite_differences(wscale):
    theta = synth.mlp_init(11).astype(np.float64)
    x, y = small_batch()
    t = np.random.default_rng(6).normal(size=len(x)) * 3
    _, g = S.loss_and_grad(theta, x, y, t, emulate_bf16=False, wscale=wscale)
    rng = np.random.default_rng(7)
    # parameters from every block, biases and the output included
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.SHAPES])
    idx = np.concatenate([rng.integers(offs[k], offs[k + 1], 6) for k in range(len(S.SHAPES))])
    for i in idx:
        h = 1e-5 * max(1.0, abs(theta[i]))
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fp, _ = S.loss_and_grad(tp, x, y, t, emulate_bf16=False, wscale=wscale)
        fm, _ = S.loss_and_grad(tm, x, y, t, emulate_bf16=False, wscale=wscale)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_gradient_stays_within_the_rounding_bound():
    theta = synth.mlp_init(12).astype(np.float64)
    x, y = small_batch(256, 8)
    t = S.target(np.minimum(x, 12.0), y)
    _, g0 = S.loss_and_grad(theta, x, y, t, emulate_bf16=False)
    _, g1 = S.loss_and_grad(theta, x, y, t, emulate_bf16=True)
    # operands rounded to 8 significant bits (2^-9 relative each), four
    # layers deep: a few percent in norm at most
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)
    assert np.dot(g0, g1) / (np.linalg.norm(g0) * np.linalg.norm(g1)) > 0.999


def test_forward_of_constant_network_is_closed_form():
    p = {name: np.zeros(shape) for name, shape in S.SHAPES}
    p["b1"][:] = 0.3; p["b2"][:] = -0.7; p["b3"][:] = 1.1; p["b4"][:] = 0.25
    p["W2"][:] = 0.0; p["w5"][:] = 0.5; p["b5"][0] = -0.125
    theta = S.pack(p)
    x, y = small_batch(10)
    out, _ = S.forward(theta, x, y, emulate_bf16=False)
    h4 = 0.25 / (1 + np.exp(-0.25))
    assert np.allclose(out, 64 * 0.5 * h4 - 0.125, rtol=1e-15, atol=0)
    # a network passing f1 = x/25 - 1 through one unit of each layer
    p = {name: np.zeros(shape) for name, shape in S.SHAPES}
    p["W1"][0, 0] = 1.0
    for k in (2, 3, 4):
        p["W%d" % k][0, 0] = 1.0
    p["w5"][0] = 1.0
    out, _ = S.forward(S.pack(p), x, y, emulate_bf16=False)
    f1 = x / 25 - 1
    assert np.allclose(out, S.silu(S.silu(S.silu(S.silu(f1)))), rtol=1e-14)


def test_adam_steps_for_a_constant_gradient():
    # with bias correction, m_hat = g and v_hat = g^2 at every step, so each
    # step moves by lr g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5]); g = np.array([0.3, -1e-3, 4.0])
    m = np.zeros(3); v = np.zeros(3)
    lr, eps = 1e-2, 1e-8
    th = theta.copy()
    for step in range(1, 6):
        th, m, v = S.adam_step(th, m, v, g, step, lr, eps=eps)
        assert np.allclose(th, theta - step * lr * g / (np.abs(g) + eps), rtol=1e-13, atol=1e-15)


def test_target_is_zero_where_the_method_uses_the_three_node_rule():
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 50, 4000)
    y = 10.0 ** rng.uniform(-4, 2, 4000)
    z = S.target(x, y)
    outside = x * x + y * y >= 100.0
    assert np.all(z[outside] == 0.0)
    assert np.all(np.isfinite(z))
    # inside, the target reconstructs the plain method's series value
    K = S.reconstruct(z, x, y)
    ref = oracle.voigt_series(y[~outside], x[~outside])
    assert np.max(np.abs(K[~outside] / ref - 1)) < 1e-9
    # at the line centre the 3-node rule overshoots for small y (its node at
    # t = 0 is a narrow Lorentzian): z < 0; a little off centre it misses the
    # Gaussian core: z > 0
    assert S.target(0.0, 1e-4)[0] < 0 and S.target(1.0, 1e-4)[0] > 0


def test_weighted_loss_is_the_weighted_mean():
    # with every weight computed by hand: w = 1/(1 + (z/s)^2)
    theta = synth.mlp_init(13).astype(np.float64)
    x, y = small_batch(6, 14)
    t = np.array([0.0, 1.0, -2.0, 4.0, 8.0, -16.0])
    out, _ = S.forward(theta, x, y, emulate_bf16=False)
    w = np.array([1.0, 1 / 1.25, 1 / 2.0, 1 / 5.0, 1 / 17.0, 1 / 65.0])
    loss, _ = S.loss_and_grad(theta, x, y, t, emulate_bf16=False, wscale=2.0)
    assert abs(loss - np.mean(w * (out - t) ** 2)) <= 1e-14 * loss
