"""Oracle residual-reduction loss and its gradient w.r.t. the smoother coefficients.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product.

Loss (Sec. 3.3, Eq. 11; Alg. 1, steps 9-12):
    L = sum_{n=1}^{Nvc} log10(||r_n|| / ||r_{n-1}||),   r_n = f - A u_n,
with u_n the n-th V-cycle iterate from u_0 (Reading: u_0 = 0 unless given).
Validation metric (Sec. 3.3, Eq. 13): log10(||r_{n+1}|| / ||r^{omega-J}_{n+1}||).

The gradient with respect to each level's coefficients is computed by the complex
step, Im L(c + i h e_k) / h with h = 1e-30, which is exact to rounding because
every operation of the cycle (Horner, divisions, sparse products, the LU solve)
is analytic in c; norms are written sqrt(sum r_i^2) without conjugation. Central
finite differences serve as a second, independent check.
"""
from __future__ import annotations

import numpy as np

from . import amg


def _norm(r):
    return np.sqrt(np.sum(r * r))


def vcycle_loss(h: amg.Hierarchy, coeffs, degree: int, f, u0=None, nvc: int = 1,
                nu1: int = 1, nu2: int = 1):
    """Residual-reduction loss of ``nvc`` V-cycles; coeffs has one row per level (the coarsest row is unused)."""
    A = h.levels[0].A
    coeffs = np.asarray(coeffs)
    Qs = [amg.assemble_smoother(h.levels[l].A, coeffs[l], degree) for l in range(h.nlevels - 1)] + [None]
    u = np.zeros(A.shape[0], dtype=coeffs.dtype if np.iscomplexobj(coeffs) else np.float64) if u0 is None else u0
    f = np.asarray(f, dtype=np.float64)
    r_prev = f - A @ u
    loss = 0.0
    for _ in range(nvc):
        u = amg.vcycle(h, Qs, u, f, nu1, nu2)
        r = f - A @ u
        loss = loss + np.log10(_norm(r) / _norm(r_prev))
        r_prev = r
    return loss


def grad_complex_step(h: amg.Hierarchy, coeffs, degree: int, f, u0=None, nvc: int = 1,
                      nu1: int = 1, nu2: int = 1, step: float = 1e-30) -> np.ndarray:
    """dL/dc for every level and coefficient by the complex step."""
    coeffs = np.asarray(coeffs, dtype=np.float64)
    g = np.zeros_like(coeffs)
    for l in range(h.nlevels - 1):
        for k in range(coeffs.shape[1]):
            c = coeffs.astype(np.complex128)
            c[l, k] += 1j * step
            g[l, k] = np.imag(vcycle_loss(h, c, degree, f, u0, nvc, nu1, nu2)) / step
    return g


def grad_central_fd(h: amg.Hierarchy, coeffs, degree: int, f, u0=None, nvc: int = 1,
                    nu1: int = 1, nu2: int = 1, rel: float = 1e-6) -> np.ndarray:
    """dL/dc by central differences with step 1e-6 max(|c_k|, 1e-2)."""
    coeffs = np.asarray(coeffs, dtype=np.float64)
    g = np.zeros_like(coeffs)
    for l in range(h.nlevels - 1):
        for k in range(coeffs.shape[1]):
            hk = rel * max(abs(coeffs[l, k]), 1e-2)
            cp = coeffs.copy()
            cm = coeffs.copy()
            cp[l, k] += hk
            cm[l, k] -= hk
            g[l, k] = (vcycle_loss(h, cp, degree, f, u0, nvc, nu1, nu2)
                       - vcycle_loss(h, cm, degree, f, u0, nvc, nu1, nu2)) / (2 * hk)
    return g


def validation_metric(h: amg.Hierarchy, coeffs, degree: int, f, u0=None, nu1: int = 1, nu2: int = 1,
                      omega: float = 2.0 / 3.0, ncycles: int = 1) -> float:
    """log10(||r_n|| / ||r_n^{omega-J}||) after n = ncycles cycles from the same u0 (Sec. 3.3, Eq. 13,
    whose r_{n+1} is the residual after the cycles of the loss); negative means better than Jacobi."""
    A = h.levels[0].A
    f = np.asarray(f, dtype=np.float64)
    u0 = np.zeros_like(f) if u0 is None else u0
    coeffs = np.asarray(coeffs, dtype=np.float64)
    Qs = [amg.assemble_smoother(h.levels[l].A, coeffs[l], degree) for l in range(h.nlevels - 1)] + [None]
    Qj = amg.smoothers(h, amg.jacobi_coeffs(omega, degree), degree)
    u, uj = u0, u0
    for _ in range(ncycles):
        u = amg.vcycle(h, Qs, u, f, nu1, nu2)
        uj = amg.vcycle(h, Qj, uj, f, nu1, nu2)
    r = f - A @ u
    rj = f - A @ uj
    return float(np.log10(np.linalg.norm(r) / np.linalg.norm(rj)))
