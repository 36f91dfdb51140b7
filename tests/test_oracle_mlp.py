"""Pins for the float64 CDF-network oracle: a hand-computed forward pass,
central finite differences of the loss, the closed form of Adam's first step,
monotonicity and a decreasing loss.  CPU only."""
import numpy as np

from oracle import mlp


def test_forward_hand_computed():
    H = mlp.H
    W1 = np.zeros(H); b1 = np.zeros(H)
    W2 = np.zeros((H, H)); b2 = np.zeros(H)
    W3 = np.zeros(H)
    W1[0], b1[0] = 2.0, -0.5          # h1[0] = ramp(2x - 0.5)
    W1[1], b1[1] = 1.0, 0.25          # h1[1] = ramp(x + 0.25)
    W2[3, 0] = 1.0                    # h2[3] = ramp(h1[0] + 0.5*h1[1]) ; asymmetric W2
    W2[3, 1] = 0.5
    W2[0, 3] = 9.0                    # would matter only if W2 were transposed
    W3[3] = 3.0
    p = mlp.pack(W1, b1, W2, b2, W3, 0.125)
    x = np.array([0.0, 0.3, 0.5, 1.0])
    f, _ = mlp.forward(p, x)
    exp = []
    for xv in x:
        h0 = min(max(2 * xv - 0.5, 0), 1)
        h1 = min(max(xv + 0.25, 0), 1)
        h2 = min(max(h0 + 0.5 * h1, 0), 1)
        exp.append(3.0 * h2 + 0.125)
    # x=0: h0=0, h1=.25 -> h2=.125 -> f=.5 ; x=1: h0=1, h1=1 -> h2=1 -> f=3.125
    assert np.allclose(f, exp, rtol=0, atol=1e-15)
    assert f[0] == 0.5 and f[3] == 3.125


def test_gradient_central_differences():
    rng = np.random.default_rng(0)
    for trial in range(4):
        p = mlp.init_params(rng.random(mlp.N_PARAMS))
        p += rng.normal(0, 0.05, size=p.shape) * (1 - mlp.weight_mask())
        x = rng.random(64)
        y = np.sort(rng.random(64))
        _, g = mlp.loss_grad(p, x, y)
        h = 1e-6
        fd = np.zeros_like(p)
        for i in range(p.size):
            e = np.zeros_like(p); e[i] = h
            lp, _ = mlp.loss_grad(p + e, x, y)
            lm, _ = mlp.loss_grad(p - e, x, y)
            fd[i] = (lp - lm) / (2 * h)
        scale = np.max(np.abs(g))
        assert np.allclose(g, fd, rtol=1e-5, atol=1e-7 * scale), np.max(np.abs(g - fd))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    p = mlp.init_params(rng.random(mlp.N_PARAMS))
    g = rng.normal(size=p.shape)
    lr = 1e-3
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=lr)
    # t=1: mhat = g, vhat = g^2, so the step is lr * g / (|g| + eps) ~ lr*sign(g)
    step = p - lr * g / (np.abs(g) + 1e-8)
    w = mlp.weight_mask() > 0
    exp = np.where(w, np.maximum(step, 0), step)
    assert np.allclose(p1, exp, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_monotone_and_pwl_nondecreasing():
    rng = np.random.default_rng(2)
    p = mlp.init_params(rng.random(mlp.N_PARAMS))
    x = np.linspace(0, 1, 4097)
    f, _ = mlp.forward(p, x)
    assert np.all(np.diff(f) >= -1e-15)
    k = mlp.to_pwl(p)
    assert k.shape == (1025,) and np.all(np.diff(k) >= 0) and k.min() >= 0 and k.max() <= 1


def test_training_lowers_loss_on_skewed_cdf():
    rng = np.random.default_rng(3)
    p = mlp.init_params(rng.random(mlp.N_PARAMS))
    x = np.sort(rng.random(2048) ** 4)            # steep CDF at the low end
    y = np.arange(2048) / 2048
    m = np.zeros_like(p); v = np.zeros_like(p)
    l0, _ = mlp.loss_grad(p, x, y)
    for t in range(1, 301):
        _, g = mlp.loss_grad(p, x, y)
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
    l1, _ = mlp.loss_grad(p, x, y)
    assert l1 < 0.2 * l0
    assert np.all(p[mlp.weight_mask() > 0] >= 0)


def _hand_net(w3, b3):
    """h1 = ramp(4x - 1), ramp(2x); h2[o] = ramp(h1[1-o]); f = w3 . h2 + b3."""
    H = mlp.H
    W1 = np.zeros(H); b1 = np.zeros(H)
    W2 = np.zeros((H, H)); b2 = np.zeros(H)
    W3 = np.zeros(H)
    W1[0], b1[0] = 4.0, -1.0
    W1[1] = 2.0
    W2[0, 1] = 1.0
    W2[1, 0] = 1.0
    W3[0], W3[1] = w3
    return mlp.pack(W1, b1, W2, b2, W3, b3)


def test_to_pwl_knots_hand_computed():
    """Knots on the grid x_j = j/4 of two hand-built networks, worked by hand.

    Net A, f = 0.8*ramp(2x) - 0.6*ramp(4x - 1) - 0.2:
      x = 0: -0.2 -> clamp 0;  x = 1/4: 0.8*0.5 - 0 - 0.2 = 0.2;
      x = 1/2: 0.8 - 0.6 - 0.2 = 0 -> running max 0.2;  x = 3/4, 1: 0 -> 0.2.
    Net B, f = 0.5*ramp(2x) + 0.25*ramp(4x - 1) + 0.125:
      0.125, 0.375, 0.875, 0.875, 0.875 (both ramps saturate at x = 1/2).
    A grid of j/5 (x = 0.2: net B gives 0.325) or a missing running maximum
    (net A would give 0 at x = 1/2) changes a knot.
    """
    ka = mlp.to_pwl(_hand_net((0.8, -0.6), -0.2), n_knots=5)
    assert np.allclose(ka, [0.0, 0.2, 0.2, 0.2, 0.2], rtol=0, atol=1e-15)
    kb = mlp.to_pwl(_hand_net((0.5, 0.25), 0.125), n_knots=5)
    assert np.allclose(kb, [0.125, 0.375, 0.875, 0.875, 0.875], rtol=0, atol=1e-15)
    # clamp at the top: f = 3*ramp(2x) -> 0, 1, 1, 1, 1 after clamping
    kc = mlp.to_pwl(_hand_net((3.0, 0.0), 0.0), n_knots=5)
    assert np.allclose(kc, [0.0, 1.0, 1.0, 1.0, 1.0], rtol=0, atol=1e-15)


def test_to_pwl_default_grid_is_1024_segments():
    """1025 knots at x_j = j/1024: net B's knot at j = 100 is
    0.5*ramp(200/1024) + 0.25*ramp(400/1024 - 1) + 0.125 = 0.5*0.1953125 + 0.125."""
    k = mlp.to_pwl(_hand_net((0.5, 0.25), 0.125))
    assert k.shape == (1025,)
    assert k[100] == 0.5 * (200 / 1024) + 0.125
    assert k[256] == 0.5 * 0.5 + 0.125          # 4x - 1 = 0 exactly at x = 1/4
    assert k[1024] == 0.875


def test_gradient_bound_covers_float32_kernel_order():
    """The derived per-element bound on the float32 gradient (tests/mlp_bound.py)
    holds for a numpy float32 emulation of the kernel's order of operations,
    and it is not vacuous: the bound stays a small multiple of the observed
    error and far below the gradient's scale."""
    from mlp_bound import float32_grad, grad_bound
    rng = np.random.default_rng(11)
    for m in (1, 255, 1000, 4096):
        p = mlp.init_params(rng.random(mlp.N_PARAMS)).astype(np.float32).astype(np.float64)
        x = np.sort(rng.random(m) ** 3).astype(np.float32).astype(np.float64)
        y = (np.arange(m) / m).astype(np.float32).astype(np.float64)
        _, g64 = mlp.loss_grad(p, x, y)
        g32 = float32_grad(p, x, y)
        b, amb = grad_bound(p, x, y)
        err = np.abs(g32 - g64)
        assert np.all(err <= b), (m, np.max(err / np.maximum(b, 1e-300)))
        scale = np.max(np.abs(g64))
        assert np.max(b) < 1e-3 * scale, (m, np.max(b) / scale)
