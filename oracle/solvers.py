"""Krylov solvers (paper Sec. 4).

The rational functions of eq. (ratapprx) need x_k = (A + d_k)^{-1} b for every
pole d_k.  The paper does this with one shifted ("multi-shift") conjugate
gradient [Jegerlehner, hep-lat/9612014] that uses a single Krylov space for
all shifts.  The recurrences are written out below from the CG three-term
recurrence: with the base system (A + s0) solved by CG, the residual of the
system shifted by s = d_k - s0 stays collinear with the base residual,
r_s = zeta_s r, and

    zeta_s' = zeta_s zeta_s_old a_old / ( zeta_s_old a_old (1 + a s)
                                          + a b_old (zeta_s_old - zeta_s) )
    a_s = a zeta_s' / zeta_s,      b_s = b (zeta_s' / zeta_s)^2
    x_s += a_s p_s,                p_s = zeta_s' r + b_s p_s

Reading (the paper is silent): the base shift is the smallest pole; shift s is
frozen once |zeta_s| |r| <= tol |b|; the solve stops when every shift is frozen.
"""
from __future__ import annotations

import numpy as np


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    return np.vdot(a.reshape(-1), b.reshape(-1))


def cg(apply_op, b: np.ndarray, tol: float, maxiter: int = 100000):
    """Plain CG for a Hermitian positive-definite operator; returns (x, iters)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = b.copy()
    rr = vdot(r, r).real
    stop = tol * tol * rr
    for k in range(maxiter):
        if rr <= stop:
            return x, k
        w = apply_op(p)
        a = rr / vdot(p, w).real
        x = x + a * p
        r = r - a * w
        rr_new = vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxiter


def multishift_cg(apply_A, b: np.ndarray, sigmas, tol: float, maxiter: int = 100000):
    """Solve (A + sigma_i) x_i = b for all sigma_i >= 0 with one Krylov space.

    Returns a dict: ``x`` (list of solutions), ``iters`` (iterations run),
    ``iters_per_pole``, ``zeta`` and ``r`` (final collinearity factors and base
    residual; the recursive residual of shift i is zeta_i * r).
    """
    sig = np.asarray(sigmas, dtype=np.float64)
    n = len(sig)
    if np.all(b == 0):
        return {"x": [np.zeros_like(b) for _ in range(n)], "iters": 0,
                "iters_per_pole": [0] * n, "zeta": np.ones(n), "r": b.copy()}
    s0 = sig.min()
    shift = sig - s0
    x = [np.zeros_like(b) for _ in range(n)]
    ps = [b.copy() for _ in range(n)]
    r = b.copy()
    p = b.copy()
    zeta = np.ones(n)
    zeta_old = np.ones(n)
    a_old, b_old = 1.0, 0.0
    rr = vdot(r, r).real
    bnorm = np.sqrt(rr)
    active = np.ones(n, dtype=bool)
    iters_per_pole = [0] * n
    k = 0
    while k < maxiter and active.any():
        w = apply_A(p) + s0 * p
        a = rr / vdot(p, w).real
        zeta_new = zeta.copy()
        zeta_new[active] = (zeta[active] * zeta_old[active] * a_old
                            / (zeta_old[active] * a_old * (1 + a * shift[active])
                               + a * b_old * (zeta_old[active] - zeta[active])))
        a_s = a * zeta_new / zeta
        for i in np.nonzero(active)[0]:
            x[i] = x[i] + a_s[i] * ps[i]
        r = r - a * w
        rr_new = vdot(r, r).real
        bet = rr_new / rr
        b_s = bet * (zeta_new / zeta) ** 2
        p = r + bet * p
        for i in np.nonzero(active)[0]:
            ps[i] = zeta_new[i] * r + b_s[i] * ps[i]
        zeta_old[active] = zeta[active]
        zeta[active] = zeta_new[active]
        a_old, b_old, rr = a, bet, rr_new
        k += 1
        for i in np.nonzero(active)[0]:
            iters_per_pole[i] = k
            if abs(zeta[i]) * np.sqrt(rr) <= tol * bnorm:
                active[i] = False
    return {"x": x, "iters": k, "iters_per_pole": iters_per_pole, "zeta": zeta, "r": r}


def true_residuals(apply_A, b: np.ndarray, sigmas, xs) -> np.ndarray:
    """|b - (A + sigma_i) x_i| / |b| for each pole."""
    bn = np.sqrt(vdot(b, b).real)
    out = []
    for s, x in zip(sigmas, xs):
        res = b - (apply_A(x) + s * x)
        out.append(np.sqrt(vdot(res, res).real) / bn)
    return np.array(out)
