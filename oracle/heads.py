"""Loss heads of the end-to-end learning pipelines, plain numpy FP64.

TEST INFRASTRUCTURE ONLY: the reference the GPU loss heads are checked
against; only the tests, the package smoke test and the benchmark's CPU
baseline may use it.

Each function is the definition written out (Section 4: the shortest-path
experiment trains a linear cost model through the solver with a regret loss;
the QP part differentiates the solution of a convex QP; Section 3.4 names the
SPO+ loss of Elmachtoub and Grigas and the perturbed Fenchel-Young loss of
Berthet et al. as the surrogate losses for LP, restated here from their
definitions for a minimisation problem min_{w in S} c'w).
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


def spo_plus_costs(c_hat, c_true):
    """Cost vector of the SPO+ inner problem: 2 c_hat - c_true."""
    return 2.0 * np.asarray(c_hat, float) - np.asarray(c_true, float)


def spo_plus(c_hat, c_true, w_star, z_star, w_tilde):
    """SPO+ loss and subgradient per instance.

    w_star[b] is optimal under c_true[b] with value z_star[b]; w_tilde[b] is
    optimal under 2 c_hat[b] - c_true[b]. Then
      loss[b] = max_{w in S} (c - 2 c_hat)'w + 2 c_hat'w* - z*
              = -(2 c_hat - c)'w_tilde + 2 c_hat'w* - z*,
      grad[b] = 2 (w* - w_tilde), a subgradient of the (convex) loss in c_hat."""
    c_hat, c_true, w_star, w_tilde = (np.asarray(a, float) for a in (c_hat, c_true, w_star, w_tilde))
    z_star = np.asarray(z_star, float)
    B = c_hat.shape[0]
    loss = np.zeros(B)
    for b in range(B):
        inner = 2.0 * c_hat[b] - c_true[b]
        loss[b] = -np.dot(inner, w_tilde[b]) + 2.0 * np.dot(c_hat[b], w_star[b]) - z_star[b]
    return loss, 2.0 * (w_star - w_tilde)


def pfy_costs(c_hat, Z, eps):
    """Perturbed costs of the Fenchel-Young estimator: [B, M, n] with entry
    (b, m) = c_hat[b] + eps Z[b, m] (Z: the caller's standard normal draws)."""
    c_hat, Z = np.asarray(c_hat, float), np.asarray(Z, float)
    return c_hat[:, None, :] + eps * Z


def pfy(c_hat, w_star, Z, eps, w_samples):
    """Perturbed Fenchel-Young loss (up to the constant Omega(w*), which does
    not depend on c_hat) and its gradient, by M samples per instance.

    With maximisation over S of <w, theta + eps Z> and theta = -c_hat (so the
    perturbation is c_hat + eps Z' with Z' = -Z, the same law), the loss is
    F(theta) - <theta, w*> + Omega(w*) and its gradient in theta is
    E[argmax] - w*. In c_hat, with w_samples[b, m] optimal under the
    perturbed costs pfy_costs(c_hat, Z, eps)[b, m]:
      loss[b] = c_hat'w* - (1/M) sum_m (c_hat + eps Z_m)'w_m,
      grad[b] = w* - (1/M) sum_m w_m."""
    c_hat, w_star, Z, ws = (np.asarray(a, float) for a in (c_hat, w_star, Z, w_samples))
    B, M = Z.shape[0], Z.shape[1]
    loss = np.zeros(B)
    grad = np.zeros_like(c_hat)
    for b in range(B):
        acc = 0.0
        wsum = np.zeros(c_hat.shape[1])
        for m in range(M):
            acc += np.dot(c_hat[b] + eps * Z[b, m], ws[b, m])
            wsum += ws[b, m]
        loss[b] = np.dot(c_hat[b], w_star[b]) - acc / M
        grad[b] = w_star[b] - wsum / M
    return loss, grad
