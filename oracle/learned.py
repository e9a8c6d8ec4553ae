"""FP64 oracle of the learned factorised preconditioner (TEST INFRASTRUCTURE ONLY).

The preconditioner is M^{-1} = G G^T with G lower triangular on the pattern of the lower
triangle of a 5-point operator: the diagonal, the west neighbour (i-1) and the south
neighbour (i-nx).  In the split-preconditioned recurrences (Section 4.5, eq. (zsre2)) this
is L^{-1} = G^T and L^{-T} = G.

A small network maps the local stencil of each row to its three entries of G:

* features f_i = (log a_ii, a_iW/a_ii, a_iE/a_ii, a_iS/a_ii, a_iN/a_ii,
  log(a_WW/a_ii), log(a_SS/a_ii)) where a_WW, a_SS are the diagonal entries of the west
  and south neighbours (missing neighbours give 0);
* h1 = tanh(W1 f + b1) (32), h2 = tanh(W2 h1 + b2) (32), o = W3 h2 + b3 (3);
* G_ii = a_ii^{-1/2} exp(o_0), G_i,i-1 = a_ii^{-1/2} o_1, G_i,i-nx = a_ii^{-1/2} o_2.

G_ii > 0, so G is non-singular and G G^T is SPD for any parameters; o = 0 gives the Jacobi
factor a_ii^{-1/2}.

Loss of one operator with right-hand side b and solution x (x from the ECG solver):
the A-norm error of one preconditioned Richardson step from zero, relative to ||x||_A:
    L = ||G G^T b - x||_A^2 / ||x||_A^2.
With u = G^T b, e = G u - x, w = G^T A e and c = x^T A x its gradient with respect to an
entry G_ij is (2/c) ((A e)_i u_j + b_i w_j).  A batch loss is the mean over operators.
Adam (Kingma and Ba) updates the parameters.

Parameters are one flat vector, in the order W1 (32x7, row-major), b1, W2 (32x32), b2,
W3 (3x32), b3: 1411 values.
"""

from __future__ import annotations

import numpy as np

from workloads.nn_inputs import init_params  # noqa: F401  (seeded input, shared)

NF, NH, NO = 7, 32, 3
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta):
    out = {}
    off = 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    return out


def flatten(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def stencil5(A, nx: int) -> np.ndarray:
    """Five stencil coefficients per row of a 5-point operator in natural order:
    rows (diag, west, east, south, north), shape (5, n); absent neighbours are 0."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    n = A.shape[0]
    i = np.arange(n)
    out = np.zeros((5, n))
    out[0] = A.diagonal()
    w = i % nx > 0
    e = i % nx < nx - 1
    s = i >= nx
    nn = i < n - nx
    out[1, w] = np.asarray(A[i[w], i[w] - 1]).ravel()
    out[2, e] = np.asarray(A[i[e], i[e] + 1]).ravel()
    out[3, s] = np.asarray(A[i[s], i[s] - nx]).ravel()
    out[4, nn] = np.asarray(A[i[nn], i[nn] + nx]).ravel()
    return out


def features(a5: np.ndarray, nx: int) -> np.ndarray:
    d = a5[0]
    n = d.shape[0]
    i = np.arange(n)
    fw = np.zeros(n)
    fs = np.zeros(n)
    w = i % nx > 0
    s = i >= nx
    fw[w] = np.log(d[i[w] - 1] / d[w])
    fs[s] = np.log(d[i[s] - nx] / d[s])
    return np.stack([np.log(d), a5[1] / d, a5[2] / d, a5[3] / d, a5[4] / d, fw, fs], axis=1)


def mlp_forward(theta, F):
    p = unflatten(theta)
    z1 = F @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(z2)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (F, h1, h2)


def mlp_backward(theta, cache, do):
    """Gradient of sum(do * o) with respect to the flat parameters (backpropagation)."""
    p = unflatten(theta)
    F, h1, h2 = cache
    g = {"W3": do.T @ h2, "b3": do.sum(axis=0)}
    d2 = (do @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"] = d1.T @ F
    g["b1"] = d1.sum(axis=0)
    return flatten(g)


def g_diagonals(o, a5, nx):
    """(gd, gw, gs): G_ii, G_i,i-1, G_i,i-nx from the network output."""
    n = a5.shape[1]
    i = np.arange(n)
    s = 1.0 / np.sqrt(a5[0])
    gd = s * np.exp(o[:, 0])
    gw = np.where(i % nx > 0, s * o[:, 1], 0.0)
    gs = np.where(i >= nx, s * o[:, 2], 0.0)
    return gd, gw, gs


def g_matrix(gd, gw, gs, nx):
    import scipy.sparse as sp

    n = gd.shape[0]
    i = np.arange(n)
    w = i % nx > 0
    s = i >= nx
    rows = np.r_[i, i[w], i[s]]
    cols = np.r_[i, i[w] - 1, i[s] - nx]
    vals = np.r_[gd, gw[w], gs[s]]
    G = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    G.sort_indices()
    return G


def loss_and_grad_g(A, G, b, x, nx):
    """Loss of one operator and its gradient with respect to (gd, gw, gs)."""
    n = b.shape[0]
    i = np.arange(n)
    u = G.T @ b
    e = G @ u - x
    Ae = A @ e
    w = G.T @ Ae
    c = float(x @ (A @ x))
    L = float(e @ Ae) / c
    k = 2.0 / c
    dgd = k * (Ae * u + b * w)
    dgw = np.zeros(n)
    dgs = np.zeros(n)
    mw = i % nx > 0
    ms = i >= nx
    dgw[mw] = k * (Ae[mw] * u[i[mw] - 1] + b[mw] * w[i[mw] - 1])
    dgs[ms] = k * (Ae[ms] * u[i[ms] - nx] + b[ms] * w[i[ms] - nx])
    return L, (dgd, dgw, dgs)


def batch_loss_and_grad(theta, ops, nx):
    """Mean loss over operators [(A, a5, b, x), ...] and its gradient (flat)."""
    total = 0.0
    grad = np.zeros(NPARAM)
    for A, a5, b, x in ops:
        o, cache = mlp_forward(theta, features(a5, nx))
        gd, gw, gs = g_diagonals(o, a5, nx)
        L, (dgd, dgw, dgs) = loss_and_grad_g(A, g_matrix(gd, gw, gs, nx), b, x, nx)
        s = 1.0 / np.sqrt(a5[0])
        do = np.stack([dgd * gd, dgw * s, dgs * s], axis=1)
        total += L
        grad += mlp_backward(theta, cache, do)
    return total / len(ops), grad / len(ops)


def adam_step(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
