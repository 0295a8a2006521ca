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
