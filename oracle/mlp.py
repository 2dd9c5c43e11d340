"""FP64 oracle of the node-wise learned predictor (test infrastructure only).

Not part of the paper's method: the paper names learned surrogates only as
related work (Sec. 1).  The extension built on top of the predictor of
Sec. 3.2 is a small per-node network that estimates the error of the
Adams-Bashforth increment (the quantity the snapshot map predicts from past
errors) from the node's displacement history and the force of the new step;
CG refinement (Algorithm 1) still decides the answer, so the network changes
the iteration count only.

Definitions followed here (plain NumPy, float64, no blocking or fusion):
  * network: y = W3 g(W2 g(W1 x + b1) + b2) + b3 with x in R^15, hidden
    widths 64 and 64, y in R^3, g the tanh form of GELU,
        g(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)));
  * parameter vector (5379 values): W1[64][15], b1[64], W2[64][64], b2[64],
    W3[3][64], b3[3], row-major;
  * loss over a batch of B samples: L = 1/(3B) sum_b sum_o (y_bo - t_bo)^2;
  * Adam (Kingma & Ba, Algorithm 1) with bias-corrected moments;
  * features of node n for step it, from its displacements u^{it-1..it-4}
    and force f^{it}: u^{it-1} / s_u, the increments (u^{it-1} - u^{it-2},
    u^{it-2} - u^{it-3}, u^{it-3} - u^{it-4}) / s_d, f^{it} / s_f (3 values
    each); the target is the error of the Adams-Bashforth increment,
    (du^{it} - du_AB^{it}) / s_t.
Weights are used in BF16 by the method; bf16_round gives those values
(round to nearest even of the float32 value).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 15, 64, 3
N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT   # 5379
_C = np.sqrt(2.0 / np.pi)


def unpack(params):
    """Views of the parameter vector: W1, b1, W2, b2, W3, b3."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    out = []
    for shape in ((N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    return out


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float64)


def gelu(z):
    """tanh form of GELU."""
    return 0.5 * z * (1.0 + np.tanh(_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    """d gelu / dz of the tanh form."""
    u = _C * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    du = _C * (1.0 + 3 * 0.044715 * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def forward(params, X):
    """Outputs Y [B][3] and the intermediate values (Z1, H1, Z2, H2)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (Z1, H1, Z2, H2)


def loss_and_grad(params, X, T):
    """Mean squared error and its gradient with respect to the parameter vector."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(params)
    Y, (Z1, H1, Z2, H2) = forward(params, X)
    B = X.shape[0]
    R = Y - T
    L = float(np.sum(R * R) / (3 * B))
    dY = 2.0 * R / (3 * B)
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * gelu_grad(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float32 values to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(u_hist, f, s_u, s_d, s_f):
    """Per-node inputs [N][15] from the displacements u^{it-1..it-4} (list of
    four [3N] vectors, newest first) and the force f^{it} ([3N])."""
    u = [np.asarray(x, dtype=np.float64).reshape(-1, 3) for x in u_hist]
    cols = [u[0] / s_u] + [(u[q] - u[q + 1]) / s_d for q in range(3)]
    cols.append(np.asarray(f, dtype=np.float64).reshape(-1, 3) / s_f)
    return np.concatenate(cols, axis=1)


def correction(params, X, s_t):
    """Estimate of the Adams-Bashforth error, [N][3] (s_t times the outputs)."""
    Y, _ = forward(params, X)
    return s_t * Y
