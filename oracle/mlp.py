"""Per-node MLP smoother, FP64 reference (oracle; test infrastructure only).

The learned part of the workload replaces one damped-Jacobi sweep of the AMG
cycles on the mesh-motion and solid levels by a small network applied node by
node: the input of node i is the Jacobi-scaled residual D^{-1} b at the 3^d
lattice nodes around i (d components each, zero where the neighbour is not an
unknown of the operator), the output is the correction at node i.  The
network has three bias-free layers with ReLU between them,

    delta = W3^T relu(W2^T relu(W1^T z)),

so it is positively homogeneous (delta(a z) = a delta(z), a > 0) and needs
no input normalisation.  Training minimises the diagonal-weighted squared
error L = (1/n) sum_i w_i ||delta_i - e_i||^2 against exact corrections e,
with Adam (beta = 0.9, 0.999, eps = 1e-8).  If the network's correction
would increase the residual norm the damped-Jacobi sweep is used instead.

Every function is plain FP64 numpy.  ``round_bf16`` reproduces the storage
precision of the GPU path (round to nearest even to 8 significant bits) so
that both sides can be fed the same values.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32-representable values to bfloat16 (nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def stencil_inputs(v: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """z[i, s*d + c] = v[nbr[i, s], c] (0 where nbr[i, s] < 0).

    v: (n, d) node values; nbr: (n, S) neighbour indices in lattice-offset
    order (S = 3^d).
    """
    n, S = nbr.shape
    d = v.shape[1]
    z = np.zeros((n, S * d))
    for s in range(S):
        ok = nbr[:, s] >= 0
        z[ok, s * d:(s + 1) * d] = v[nbr[ok, s]]
    return z


def forward(W, z, act_round=None):
    """Returns (y, cache).  act_round optionally rounds the hidden
    activations (the GPU stores them in bfloat16 between layers)."""
    W1, W2, W3 = W
    a1 = z @ W1
    h1 = np.maximum(a1, 0.0)
    if act_round is not None:
        h1 = act_round(h1)
    a2 = h1 @ W2
    h2 = np.maximum(a2, 0.0)
    if act_round is not None:
        h2 = act_round(h2)
    y = h2 @ W3
    return y, (z, a1, h1, a2, h2)


def loss(y, e, w):
    """(1/n) sum_i w_i ||y_i - e_i||^2."""
    return float(np.sum(w[:, None] * (y - e) ** 2) / y.shape[0])


def backward(W, cache, dy, grad_round=None):
    """Gradients of sum(dy * y) with respect to W1, W2, W3 (chain rule by hand).
    grad_round optionally rounds the back-propagated dy, da2, da1 (the GPU
    stores them in bfloat16 before the weight-gradient products)."""
    W1, W2, W3 = W
    z, a1, h1, a2, h2 = cache
    rnd = grad_round if grad_round is not None else (lambda t: t)
    dy = rnd(dy)
    dW3 = h2.T @ dy
    dh2 = dy @ W3.T
    da2 = rnd(dh2 * (a2 > 0.0))
    dW2 = h1.T @ da2
    dh1 = da2 @ W2.T
    da1 = rnd(dh1 * (a1 > 0.0))
    dW1 = z.T @ da1
    return dW1, dW2, dW3


def loss_and_grad(W, z, e, w, act_round=None, grad_round=None):
    y, cache = forward(W, z, act_round)
    dy = (2.0 / y.shape[0]) * w[:, None] * (y - e)
    return loss(y, e, w), backward(W, cache, dy, grad_round)


def adam_step(W, G, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), step counter t starting at 1."""
    out_W, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(W, G, m, v):
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        mh = mm / (1.0 - b1 ** t)
        vh = vv / (1.0 - b2 ** t)
        out_W.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_W, out_m, out_v


def init_weights(k_in: int, hidden: int, d: int, seed: int):
    """He-style seeded initial weights (the random draws are inputs)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((k_in, hidden)) * np.sqrt(2.0 / k_in)
    W2 = rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)
    W3 = rng.standard_normal((hidden, d)) * np.sqrt(1.0 / hidden)
    return [W1, W2, W3]


def learned_vcycle(H, B: np.ndarray, X0: np.ndarray) -> np.ndarray:
    """V(1,1) cycle of an AMG hierarchy on the columns of B (n x c) whose
    first pre-smoothing sweep on the finest level is the network's correction
    X0 instead of damped Jacobi.  If X0 does not reduce the residual,
    ||B - A X0||_F > ||B||_F (or is not finite), the plain cycle is used.
    With X0 = omega D^{-1} B this is exactly the plain V(1,1) cycle."""
    from . import amg
    L = H.levels[0]
    B = np.asarray(B, dtype=np.float64).reshape(L.A.shape[0], -1)
    R0 = B - L.A @ X0 if np.all(np.isfinite(X0)) else None
    if R0 is None or not np.linalg.norm(R0) <= np.linalg.norm(B):
        return np.column_stack([amg.vcycle(H, B[:, c]) for c in range(B.shape[1])])
    if H.nlevels == 1:
        raise ValueError("a learned pre-smoother needs at least two levels")
    Bc = L.R @ R0
    E = np.column_stack([amg.vcycle(H, Bc[:, c], 1) for c in range(B.shape[1])])
    X = X0 + L.P @ E
    return X + L.omega * (L.dinv[:, None] * (B - L.A @ X))


def two_grid_energy(delta: np.ndarray, b: np.ndarray, A, P, Ac) -> tuple:
    """Energy training loss of a pre-smoother correction delta for the
    residual b (both n x c, one column per right-hand side):

        L = ||(I - P Ac^{-1} P^T A)(e - delta)||_A^2 - e.b,   e = A^{-1} b,

    the A-norm error left after delta and an exact coarse-grid correction
    (Ac = P^T A P), shifted by the constant e.b.  Returns (L, dL/d delta);
    A is taken as symmetric, so the projection is A-orthogonal and the
    gradient is -2 A (I - P Ac^{-1} P^T A)(e - delta).  Dense solves."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    Pd = P.toarray() if hasattr(P, "toarray") else np.asarray(P)
    Acd = Ac.toarray() if hasattr(Ac, "toarray") else np.asarray(Ac)
    b = np.asarray(b, dtype=np.float64).reshape(Ad.shape[0], -1)
    delta = np.asarray(delta, dtype=np.float64).reshape(b.shape)
    e = np.linalg.solve(Ad, b)
    u = e - delta
    w = u - Pd @ np.linalg.solve(Acd, Pd.T @ (Ad @ u))
    L = float(np.sum(w * (Ad @ w)) - np.sum(e * b))
    return L, -2.0 * (Ad @ w)


def energy_loss_and_grad(W, z, b, A, P, Ac, act_round=None, grad_round=None):
    """Network-level energy loss: delta = forward(W, z) (one row per node, d
    components, node-major like b), then two_grid_energy and the chain rule."""
    y, cache = forward(W, z, act_round)
    L, g = two_grid_energy(y.reshape(-1), b, A, P, Ac)
    return L, backward(W, cache, g.reshape(y.shape), grad_round)
