"""O1: direct evaluation of the Laplace potential (Eq. 1, section "The Fast
Multipole Method"), and of its gradient at the targets.

    phi_j = sum_{i, x_i != x_j} q_i / (4 pi |x_i - x_j|)
    grad phi_j = sum_{i, x_i != x_j} -q_i (x_j - x_i) / (4 pi |x_j - x_i|^3)

(The gradient is the derivative of Eq. (1) in the target position; the paper
evaluates potentials only, so it is an extension with a plain definition.)

Self-interaction is excluded.  For general (distinct) source and target
arrays the excluded pairs are exactly those at distance zero: a target that
coincides bitwise with a source does not see that source.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

INV_4PI = 1.0 / (4.0 * np.pi)


def kernel_matrix(x: np.ndarray, y: np.ndarray, kappa: float = 0.0) -> np.ndarray:
    """K[i, j] = 1 / (4 pi |x_i - y_j|), and 0 where x_i == y_j (Eq. 1).

    With kappa > 0 the screened (Yukawa) kernel exp(-kappa r) / (4 pi r): a
    second kernel for the kernel-independent method (the paper's experiments
    use the Laplace kernel only).
    x: (m, 3) evaluation points, y: (n, 3) source points, both float64.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x[:, None, 0] - y[None, :, 0]
    dy = x[:, None, 1] - y[None, :, 1]
    dz = x[:, None, 2] - y[None, :, 2]
    r2 = dx * dx + dy * dy + dz * dz
    with np.errstate(divide="ignore"):
        r = np.sqrt(r2)
        k = INV_4PI / r
        if kappa != 0.0:
            k = k * np.exp(-kappa * r)
    k[r2 == 0.0] = 0.0
    return k


def direct(src: np.ndarray, charges: np.ndarray, tgt: np.ndarray,
           chunk: int = 2048, kappa: float = 0.0) -> np.ndarray:
    """Potentials at tgt due to charges at src, by the O(N^2) sum of Eq. (1).

    src (n_src, 3), tgt (n_tgt, 3) float64; charges (n_src,) or (n_rhs, n_src).
    Returns (n_tgt,) or (n_rhs, n_tgt) float64, matching the charges' rank.
    """
    q = np.asarray(charges, dtype=np.float64)
    one = q.ndim == 1
    q2 = q[None, :] if one else q
    out = np.zeros((q2.shape[0], len(tgt)))
    for s in range(0, len(tgt), chunk):
        k = kernel_matrix(tgt[s:s + chunk], src, kappa)
        out[:, s:s + chunk] = (k @ q2.T).T
    return out[0] if one else out


def gradient_matrices(x: np.ndarray, y: np.ndarray, kappa: float = 0.0) -> np.ndarray:
    """G[c, i, j] = d/dx_c of 1 / (4 pi |x_i - y_j|) = -(x_i - y_j)_c / (4 pi |x_i - y_j|^3),
    and 0 where x_i == y_j.  With kappa > 0, of the screened kernel
    exp(-kappa r) / (4 pi r): -(1 + kappa r) exp(-kappa r) (x_i - y_j)_c / (4 pi r^3).
    Returns (3, m, n) float64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = x[None, :, :].transpose(2, 1, 0) - y[None, :, :].transpose(2, 0, 1)  # (3, m, n)
    r2 = (d * d).sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(r2)
        w = -INV_4PI / (r2 * r)
        if kappa != 0.0:
            w = w * (1.0 + kappa * r) * np.exp(-kappa * r)
    w[r2 == 0.0] = 0.0
    return d * w[None]


def direct_gradient(src: np.ndarray, charges: np.ndarray, tgt: np.ndarray,
                    chunk: int = 1024, kappa: float = 0.0) -> np.ndarray:
    """Gradients of the potential at tgt, by the O(N^2) sum (derivative of Eq. 1).

    charges (n_src,) or (n_rhs, n_src).  Returns (3, n_tgt) or
    (n_rhs, 3, n_tgt), matching the charges' rank.
    """
    q = np.asarray(charges, dtype=np.float64)
    one = q.ndim == 1
    q2 = q[None, :] if one else q
    out = np.zeros((q2.shape[0], 3, len(tgt)))
    for s in range(0, len(tgt), chunk):
        g = gradient_matrices(tgt[s:s + chunk], src, kappa)
        for c in range(3):
            out[:, c, s:s + chunk] = (g[c] @ q2.T).T
    return out[0] if one else out
