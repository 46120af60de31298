"""Oracle of the learned cardinality estimator -- TEST INFRASTRUCTURE ONLY.

A plain numpy fp64 reference of the small network that maps a host's
per-array ("per-layer") column popcounts to a corrected cardinality
estimate, its mean-squared-error gradient and one Adam step. The paper's own
estimator is Thm. 2's corrected linear count; this network is an addition
that is compared against it.

Network (F inputs, two hidden layers of 64, one output):
    z1 = W1 x + b1,  h1 = relu(z1)
    z2 = W2 h1 + b2, h2 = relu(z2)
    y  = w3 . h2 + b3            (predicts t = ln(1 + n))
    loss = mean over the batch of (y - t)^2 / 2
Weights W1, W2, w3 are used in bfloat16 (round to nearest even from the fp32
master copy); biases in fp32. The second layer also takes its inputs in
bfloat16 (its 64 x 64 product is a bf16 contraction on the device's matrix
cores): z1 is computed in fp32 as the device does (bias first, then each
input's product added in input order), and h1 = bf16(relu(z1)) enters z2 and
the gradient of W2. Everything after that is fp64 here. With act_bf16=False
the network is the plain fp64 one (used to pin the gradient by finite
differences). Flat parameter order:
    W1 [64, F] row-major, b1 [64], W2 [64, 64] row-major, b2 [64], w3 [64], b3 [1]
Features (see ``features``): each array's own linear count of the host's
column in log form, ln(1 + g u_a) with u_a = -ln(max(z_a, 1)/g), optionally
followed by the union column's Thm. 2 count in the same form and g * eps,
and optionally by the union column's count against the row-aware shared-bit
mass (sum over rows of the product of row fills, see row_shared in the CBAA
oracle) in the same form and that mass.

Parity unpinned for the training outcome itself (it depends on data); the
gradient is pinned by central finite differences.
"""

from __future__ import annotations

import numpy as np

H = 64


def features(layer_zeros: np.ndarray, union_zeros: np.ndarray, eps: np.ndarray, g: int,
             extended: bool = True, shared: np.ndarray | None = None) -> np.ndarray:
    """Features from per-array zero counts [n, A], union-column zeros [n],
    the hosts' sketch eps [n] and, for the row-aware pair, the hosts' sketch
    shared-bit mass [n] (fp64 arithmetic, fp32 result)."""
    g = float(g)

    def logcount(z, denom):
        with np.errstate(divide="ignore"):
            u = -np.log(np.maximum(z.astype(np.float64), 1.0) / denom)
        return np.log1p(g * np.maximum(u, 0.0))

    cols = [logcount(layer_zeros[:, a], g) for a in range(layer_zeros.shape[1])]
    if extended:
        cols.append(logcount(union_zeros, g - g * eps))
        cols.append(g * eps)
    if shared is not None:
        cols.append(logcount(union_zeros, g - shared))
        cols.append(shared)
    return np.stack(cols, axis=1).astype(np.float32)


def n_params(F: int) -> int:
    return H * F + H + H * H + H + H + 1


def split(theta: np.ndarray, F: int):
    o = 0
    W1 = theta[o:o + H * F].reshape(H, F); o += H * F
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o:o + 1]; o += 1
    return W1, b1, W2, b2, w3, b3


def weight_mask(F: int) -> np.ndarray:
    """True where the parameter is a weight (stored as bf16), False for biases."""
    m = np.zeros(n_params(F), bool)
    o = 0
    m[o:o + H * F] = True; o += H * F + H
    m[o:o + H * H] = True; o += H * H + H
    m[o:o + H] = True
    return m


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round fp32 values to bfloat16 (nearest, ties to even); returned as fp32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(x)
    out = (rounded << 16).astype(np.uint32).view(np.float32)
    out = np.where(nan, np.float32(np.nan), out)
    return out.astype(np.float32)


def compute_params(master: np.ndarray, F: int) -> np.ndarray:
    """Parameters as the forward pass uses them: weights in bf16, biases fp32."""
    m = weight_mask(F)
    p = np.asarray(master, np.float32).copy()
    p[m] = to_bf16(p[m])
    return p


def layer1_fp32(theta: np.ndarray, F: int, x: np.ndarray) -> np.ndarray:
    """z1 in fp32 in the device's order: b1, then + W1[:, f] * x[:, f] for
    f = 0, 1, ..., each product and each sum rounded to fp32."""
    W1, b1 = split(theta, F)[:2]
    W1 = W1.astype(np.float32)
    x = np.asarray(x, np.float32)
    z = np.repeat(b1.astype(np.float32)[None, :], x.shape[0], axis=0)
    for f in range(F):
        z = (z + (x[:, f:f + 1] * W1[None, :, f]).astype(np.float32)).astype(np.float32)
    return z


def forward(theta: np.ndarray, F: int, x: np.ndarray, act_bf16: bool = True):
    W1, b1, W2, b2, w3, b3 = (a.astype(np.float64) for a in split(theta, F))
    if act_bf16:
        z1f = layer1_fp32(theta, F, x)
        z1 = z1f.astype(np.float64)
        h1 = to_bf16(np.maximum(z1f, np.float32(0.0))).astype(np.float64)
        x = np.asarray(x, np.float32).astype(np.float64)
    else:
        x = x.astype(np.float64)
        z1 = x @ W1.T + b1
        h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3[0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(theta: np.ndarray, F: int, x: np.ndarray, t: np.ndarray,
                  act_bf16: bool = True):
    """Mean (y - t)^2 / 2 and its gradient with respect to every parameter
    (with act_bf16, the bf16 rounding of h1 passes gradients unchanged)."""
    W1, b1, W2, b2, w3, b3 = (a.astype(np.float64) for a in split(theta, F))
    y, (x, z1, h1, z2, h2) = forward(theta, F, x, act_bf16)
    B = x.shape[0]
    r = y - t.astype(np.float64)
    loss = 0.5 * float(np.mean(r * r))
    dy = r / B
    dw3 = h2.T @ dy
    db3 = np.array([dy.sum()])
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, db3])
    return loss, g


def adam_step(master, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; returns new state."""
    master = master.astype(np.float64)
    g = grad.astype(np.float64)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


def finite_difference_grad(theta, F, x, t, idx, h=1e-6):
    """Central differences of the fp64 network's loss for the parameters
    listed in idx."""
    out = []
    for i in idx:
        tp = theta.astype(np.float64).copy()
        tm = tp.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = loss_and_grad(tp, F, x, t, act_bf16=False)
        lm, _ = loss_and_grad(tm, F, x, t, act_bf16=False)
        out.append((lp - lm) / (2 * h))
    return np.array(out)
