"""The float64 network reference against central finite differences (CPU)."""
import numpy as np

import mlp_reference as R


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(R.NPARAM) * 0.3
    x = rng.standard_normal((40, 8))
    t = rng.standard_normal(40)
    g = R.gradient(w, x, t)
    h = 1e-6
    for i in rng.choice(R.NPARAM, 300, replace=False).tolist() + [0, 511, 4799, 4800]:
        e = np.zeros(R.NPARAM)
        e[i] = h
        fd = (R.loss(w + e, x, t) - R.loss(w - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_layers_by_hand():
    w = np.zeros(R.NPARAM)
    p = {"b3": 0.5}
    # one hidden path: x0 -> h1[0] (weight 2) -> h2[0] (weight 3) -> y (weight 4)
    w[0] = 2.0                  # W1[0][0]
    w[576] = 3.0                # W2[0][0]
    w[4736] = 4.0               # w3[0]
    w[4800] = p["b3"]
    x = np.array([[1.5, 0, 0, 0, 0, 0, 0, 0], [-1.0, 0, 0, 0, 0, 0, 0, 0]])
    y, _ = R.forward(w, x)
    np.testing.assert_allclose(y, [0.5 + 4 * 3 * 2 * 1.5, 0.5])


def test_adam_first_steps_closed_forms():
    """Adam with bias correction (Kingma & Ba 2015), pinned by closed forms
    derived from its definition rather than by restating the recursion:
    * step 1: m_hat = g and v_hat = g^2 exactly, so w1 = w0 - lr g / (|g| + eps);
    * step 2: m_hat = (b1 g1 + g2) / (1 + b1), v_hat = (b2 g1^2 + g2^2) / (1 + b2);
    * a constant gradient keeps m_hat = g and v_hat = g^2 at every step, so
      each step moves every weight by lr g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    w0 = rng.standard_normal(R.NPARAM)
    g1 = rng.standard_normal(R.NPARAM)
    g2 = rng.standard_normal(R.NPARAM)
    z = np.zeros(R.NPARAM)
    w1, m1, v1 = R.adam(w0, g1, z, z, 1, lr, b1, b2, eps)
    np.testing.assert_allclose(w1, w0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    w2, _, _ = R.adam(w1, g2, m1, v1, 2, lr, b1, b2, eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 * g1 + g2 * g2) / (1 + b2)
    np.testing.assert_allclose(w2, w1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-14)
    # a wrong bias correction (none, or the first-moment factor used twice) fails the second step
    assert np.abs(w2 - (w1 - lr * (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (np.sqrt(vh) + eps))).max() > 1e-4
    w, m, v = w0.copy(), z, z
    for t in range(1, 7):
        w_prev = w
        w, m, v = R.adam(w, g1, m, v, t, lr, b1, b2, eps)
        np.testing.assert_allclose(w_prev - w, lr * g1 / (np.abs(g1) + eps), rtol=1e-12, atol=1e-15)
