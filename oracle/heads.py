"""Loss heads of the end-to-end learning pipelines, plain numpy FP64.

TEST INFRASTRUCTURE ONLY: the reference the GPU loss heads are checked
against; only the tests, the package smoke test and the benchmark's CPU
baseline may use it.

Each function is the definition written out (Section 4: the shortest-path
experiment trains a linear cost model through the solver with a regret loss;
the QP part differentiates the solution of a convex QP).
"""

import numpy as np


def linear_costs(f, W):
    """c_hat[b, a] = sum_k W[k] f[b, a, k]."""
    f = np.asarray(f, float)
    W = np.asarray(W, float)
    out = np.zeros(f.shape[:2])
    for k in range(f.shape[2]):
        out += W[k] * f[:, :, k]
    return out


def regret(c_true, x, v_star):
    """loss[b] = c_true[b]' x[b] - v_star[b]: excess true cost of the decision."""
    c_true, x = np.asarray(c_true, float), np.asarray(x, float)
    return np.array([np.dot(c_true[b], x[b]) for b in range(c_true.shape[0])]) - np.asarray(v_star, float)


def linear_costs_backward(f, gc):
    """gW[k] = sum_{b, a} gc[b, a] f[b, a, k] (chain rule through linear_costs)."""
    f, gc = np.asarray(f, float), np.asarray(gc, float)
    return np.array([np.sum(gc * f[:, :, k]) for k in range(f.shape[2])])


def qp_value(F, d, c, x):
    """value[b] = 1/2 x_b'(F F' + diag d_b) x_b + c_b' x_b and its gradient
    (F F' + diag d_b) x_b + c_b."""
    F, d, c, x = (np.asarray(a, float) for a in (F, d, c, x))
    val = np.zeros(c.shape[0])
    grad = np.zeros_like(c)
    for b in range(c.shape[0]):
        qx = F @ (F.T @ x[b]) + d[b] * x[b]
        val[b] = 0.5 * np.dot(x[b], qx) + np.dot(c[b], x[b])
        grad[b] = qx + c[b]
    return val, grad
