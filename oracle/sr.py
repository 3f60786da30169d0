"""Stochastic reconfiguration (Method section, Eqs. (5)-(7) and (10)).

With N_s samples i (drawn from |rho|^2, so uniform weights) and the full
log-derivative matrix O (N_s x N_p, real arithmetic so conjugation is the
identity):
    Ebar = (1/N_s) sum_i E_i
    obar = (1/N_s) sum_i O_i
    g    = (1/N_s) sum_i O_i (E_i - Ebar)                 (gradient, Eq. 7)
    S x  = (1/N_s) sum_i O_i (O_i . x - obar . x)         (metric, Eq. 10)
The update theta' = theta - tau G^{-1} g (Eq. 5) is taken with an identity
shift eps (reading: the paper states no regulariser):
    (S + eps I) dtheta = -tau g,   theta <- theta + dtheta,
solved by conjugate gradient applying S only through O x and O^T y, never
forming S (Method section, separable matvec).

Optional weights w_i (the reweighted estimator of Appendix A, Eq. (A1)):
averages become sum_i w_i f_i / sum_i w_i.
"""
from __future__ import annotations

import math

import numpy as np

from .measure import expand_O


def dense_O(lat, configs, O_rows):
    return np.stack([expand_O(lat, S, o) for S, o in zip(configs, O_rows)])


def _weights(n, weights):
    if weights is None:
        return np.full(n, 1.0 / n)
    w = np.asarray(weights, dtype=np.float64)
    return w / w.sum()


def sr_reductions(Ofull, e_loc, weights=None):
    """(Ebar, obar, g) from the dense O."""
    p = _weights(Ofull.shape[0], weights)
    e = np.asarray(e_loc, dtype=np.float64)
    ebar = float(p @ e)
    obar = p @ Ofull
    g = Ofull.T @ (p * (e - ebar))
    return ebar, obar, g


def sr_matvec(Ofull, x, eps, weights=None):
    """(S + eps I) x with S applied as O^T (O x - mean(O x))."""
    p = _weights(Ofull.shape[0], weights)
    y = Ofull @ x
    ybar = float(p @ y)
    return Ofull.T @ (p * (y - ybar)) + eps * x


def sr_matrix(Ofull, weights=None):
    """Dense S (only for small N_p checks)."""
    p = _weights(Ofull.shape[0], weights)
    obar = p @ Ofull
    return (Ofull.T * p) @ Ofull - np.outer(obar, obar)


def cg(apply_A, b, max_iter, rtol):
    """Conjugate gradient (Hestenes-Stiefel), x0 = 0.  The residual test
    ||r|| <= rtol ||b|| is taken before each iteration.  Returns
    (x, iterations, ||r||, breakdown)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    bnorm = math.sqrt(float(b @ b))
    it = 0
    while it < max_iter:
        if math.sqrt(rr) <= rtol * bnorm:
            break
        Ap = apply_A(p)
        pAp = float(p @ Ap)
        if not pAp > 0.0:
            return x, it, math.sqrt(rr), True
        a = rr / pAp
        x = x + a * p
        r = r - a * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, math.sqrt(rr), False


def sr_solve(lat, configs, O_rows, e_loc, tau, eps, max_iter, rtol, weights=None):
    """dtheta with (S + eps I) dtheta = -tau g; also returns g and stats."""
    Ofull = dense_O(lat, configs, O_rows)
    ebar, _, g = sr_reductions(Ofull, e_loc, weights)
    b = -tau * g
    x, it, rn, broke = cg(lambda v: sr_matvec(Ofull, v, eps, weights), b, max_iter, rtol)
    return {"dtheta": x, "g": g, "ebar": ebar, "iters": it, "rnorm": rn, "breakdown": broke}


def sr_solve_dense(lat, configs, O_rows, e_loc, tau, eps, weights=None):
    """The same system solved directly (second oracle for small N_p)."""
    Ofull = dense_O(lat, configs, O_rows)
    ebar, _, g = sr_reductions(Ofull, e_loc, weights)
    A = sr_matrix(Ofull, weights) + eps * np.eye(Ofull.shape[1])
    return np.linalg.solve(A, -tau * g)
