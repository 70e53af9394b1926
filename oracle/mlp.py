"""FP64 reference of the blow-up surrogate MLP -- TEST INFRASTRUCTURE.

Network: 4 standardised inputs (A, sx, sy, sz) -> H (GELU) -> H (GELU) -> 2
outputs (blow-up logit, standardised log blow-up time).  Loss for a batch of
B samples with labels y (1 = blow-up) and targets t (used where y = 1):
    L = (1/B) sum_b BCE(z1_b, y_b) + (1/max(1, sum_b y_b)) sum_b y_b (z2_b - t_b)^2,
    BCE(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)),
GELU(x) = x/2 (1 + erf(x/sqrt 2)).  Adam with bias correction.
Parameters use the flat layout of the GPU library: W1 (H x 4), b1 (H), W2 (H x H),
b2 (H), W3 (2 x H), b3 (2), weights row-major [out][in].

Only tests and the surrogate's checks use this module; it shares no code with
the GPU kernels.
"""
import numpy as np
from scipy.special import erf

N_IN = 4
N_OUT = 2


def sizes(H):
    return [("W1", (H, N_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (N_OUT, H)),
            ("b3", (N_OUT,))]


def num_params(H):
    return sum(int(np.prod(s)) for _, s in sizes(H))


def unflatten(flat, H):
    out, k = {}, 0
    for name, shp in sizes(H):
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def flatten(p, H):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in sizes(H)])


def init(H, seed):
    """He-style uniform initialisation from a seeded generator (the GPU side
    receives these values; it draws no random numbers itself)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in sizes(H):
        if name.startswith("W"):
            fan_in = shp[1]
            bound = np.sqrt(6.0 / fan_in) / np.sqrt(2.0)
            p[name] = rng.uniform(-bound, bound, size=shp)
        else:
            p[name] = np.zeros(shp)
    return p


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def bce(z, y):
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(p, x):
    """x: standardised inputs [B, 4].  Returns (outputs [B, 2], cache)."""
    z1 = x @ p["W1"].T + p["b1"]
    a1 = gelu(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(z2)
    out = a2 @ p["W3"].T + p["b3"]
    return out, (x, z1, a1, z2, a2)


def loss(p, x, y, t):
    out, _ = forward(p, x)
    nb = x.shape[0]
    m = y.astype(np.float64)
    cnt = max(1.0, m.sum())
    return bce(out[:, 0], m).sum() / nb + (m * (out[:, 1] - t) ** 2).sum() / cnt


def gradients(p, x, y, t):
    """Analytic gradients of loss() by the chain rule, layer by layer."""
    out, (x, z1, a1, z2, a2) = forward(p, x)
    nb = x.shape[0]
    m = y.astype(np.float64)
    cnt = max(1.0, m.sum())
    dout = np.zeros_like(out)
    dout[:, 0] = (sigmoid(out[:, 0]) - m) / nb
    dout[:, 1] = 2.0 * m * (out[:, 1] - t) / cnt
    g = {"W3": dout.T @ a2, "b3": dout.sum(0)}
    dz2 = (dout @ p["W3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    pn, mn, vn = {}, {}, {}
    for k in p:
        mn[k] = b1 * m[k] + (1 - b1) * g[k]
        vn[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = mn[k] / (1 - b1 ** step)
        vh = vn[k] / (1 - b2 ** step)
        pn[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return pn, mn, vn
