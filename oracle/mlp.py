"""FP64 oracle of the learned relaxation warm start -- TEST INFRASTRUCTURE.

Plain numpy, FP64 arithmetic, with the BF16 rounding points of the GPU
kernels written out explicitly (round-to-nearest-even to 8 significant bits):

  features  x = bf16([32 nearest offsets (r_j - r_i)/h, phi_i/h, grad phi_i])
  forward   Z1 = bf16(x) bf16(W1)^T + b1,  H1 = GELU(Z1)
            Z2 = bf16(H1) bf16(W2)^T + b2, H2 = GELU(Z2)
            Y  = bf16(H2) bf16(W3)^T + b3
  loss      MSE over the batch and the 3 outputs
  backward  dY = 2 (Y - T) / (3 B)
            dW3 = dY^T bf16(H2),  db3 = sum dY
            dZ2 = (dY bf16(W3)) * GELU'(Z2)
            dW2 = bf16(dZ2)^T bf16(H1),  db2 = sum dZ2
            dZ1 = (bf16(dZ2) bf16(W2)) * GELU'(Z1)
            dW1 = bf16(dZ1)^T bf16(x),   db1 = sum dZ1
  AdamW     decoupled weight decay on every parameter (PyTorch's default),
            bias-corrected moments, FP32 master weights.
GELU is the exact erf form.  The network and its training come from the
workload description (the paper has no learned component).

Only tests/, the smoke check and the benchmark's CPU leg may import this.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_HID, N_OUT, K_NB = 100, 128, 3, 32
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 29827


def bf16(x, exact=False):
    """Round to the nearest BF16 value (8 significant bits, ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    if exact:
        return x
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def unpack(theta):
    out, k = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + sz], dtype=np.float64).reshape(shp)
        k += sz
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases (the
    default initialisation of a PyTorch linear layer), seeded."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        fan_in = shp[1] if len(shp) == 2 else {"b1": N_IN, "b2": N_HID, "b3": N_HID}[name]
        bound = 1.0 / math.sqrt(fan_in)
        d[name] = rng.uniform(-bound, bound, size=shp)
    return pack(d).astype(np.float32)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, exact=False):
    p = unpack(theta)
    x = bf16(X, exact)
    Z1 = x @ bf16(p["W1"], exact).T + p["b1"]
    H1 = gelu(Z1)
    Z2 = bf16(H1, exact) @ bf16(p["W2"], exact).T + p["b2"]
    H2 = gelu(Z2)
    Y = bf16(H2, exact) @ bf16(p["W3"], exact).T + p["b3"]
    return Y, {"x": x, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2}


def loss_and_grad(theta, X, T, exact=False):
    """MSE loss and its gradient with respect to the packed parameters."""
    p = unpack(theta)
    Y, c = forward(theta, X, exact)
    B = X.shape[0]
    diff = Y - T
    loss = float(np.mean(diff ** 2))
    dY = 2.0 * diff / (3.0 * B)
    H2b = bf16(c["H2"], exact)
    H1b = bf16(c["H1"], exact)
    g = {}
    g["W3"] = dY.T @ H2b
    g["b3"] = dY.sum(0)
    dZ2 = (dY @ bf16(p["W3"], exact)) * gelu_grad(c["Z2"])
    dZ2b = bf16(dZ2, exact)
    g["W2"] = dZ2b.T @ H1b
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2b @ bf16(p["W2"], exact)) * gelu_grad(c["Z1"])
    dZ1b = bf16(dZ1, exact)
    g["W1"] = dZ1b.T @ c["x"]
    g["b1"] = dZ1.sum(0)
    return loss, pack(g)


def adamw(theta, grad, m, v, step, lr=1e-3, wd=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update (step counts from 1); returns new (theta, m, v)."""
    theta = np.asarray(theta, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta * (1.0 - lr * wd) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def features(pos, h, center, radius, rows=None, periodic_len=None):
    """Per row i: the 32 nearest j != i with |r_ij| <= 2h, ordered by
    (|r_ij|^2 in FP64, j), offsets (r_j - r_i)/h (zero-padded), then
    phi_i/h and grad phi_i = (r_i - c)/|r_i - c|.  Brute force over all j;
    returns FP64 features before the BF16 rounding."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    c = np.asarray(center, dtype=np.float64)
    rc2 = (2.0 * h) * (2.0 * h)
    out = np.zeros((len(rows), N_IN))
    for k, i in enumerate(rows):
        d = pos - pos[:, i:i + 1]                       # r_j - r_i
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        d2[i] = np.inf
        cand = np.nonzero(d2 <= rc2)[0]
        order = np.lexsort((cand, d2[cand]))[:K_NB]
        sel = cand[order]
        out[k, :3 * len(sel)] = (d[:, sel] / h).T.reshape(-1)
        e = pos[:, i] - c
        rr = math.sqrt(float(e @ e))
        out[k, 96] = (rr - radius) / h
        out[k, 97:100] = e / rr if rr > 0 else 0.0
    return out


def targets(pos_from, pos_to, h):
    """Training targets of the warm start: (r_to - r_from) / h per particle,
    [n][3] from positions [3][n] (FP64)."""
    d = np.asarray(pos_to, dtype=np.float64) - np.asarray(pos_from, dtype=np.float64)
    return (d / h).T.copy()
