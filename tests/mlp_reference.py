"""Float64 reference of the work-estimator network (8 -> 64 -> 64 -> 1, ReLU)
and of its mean-squared-error gradient, written from the layer equations:
h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3."""
import numpy as np

SHAPES = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", (1,))]
NPARAM = 4801


def unpack(w):
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(w[o:o + size], np.float64).reshape(shape)
        o += size
    assert o == NPARAM
    return out


def forward(w, x):
    p = unpack(w)
    x = np.asarray(x, np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    return h2 @ p["w3"] + p["b3"][0], (x, z1, h1, z2, h2)


def loss(w, x, t):
    y, _ = forward(w, x)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradient(w, x, t):
    """Analytic gradient of mean((y - t)^2) by back-propagation."""
    p = unpack(w)
    y, (x, z1, h1, z2, h2) = forward(w, x)
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    d2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])


def adam(w, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return w, m, v
