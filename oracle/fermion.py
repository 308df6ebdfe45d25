"""Pseudofermion action and force (paper eq. pfact, first term; Sec. 3.2, Sec. 4).

With alpha = 1/2 on the even sub-lattice (two flavours, Sec. 3.2) the action is
S_f = phi^dag A^{-1/2} phi, A = (M^dag M)_ee, evaluated through the rational
form of eq. (ratapprx):

    S_f = c0 |phi|^2 + sum_k c_k Re <phi, X_k>,   X_k = (A + d_k)^{-1} phi.

Force (the paper never writes it; derived here).  With Y_k = D_oe X_k and
D^dag = -D,  dS_f = sum_k c_k ( <X_k, dD_eo Y_k> - <Y_k, dD_oe X_k> ).  For a
link U_mu(x) with staggered sign s and the variation U -> exp(i w_a T_a) U:

    dS_f/dw_a = -2 Im tr(T_a s U_mu(x) W),
    W = sum_k c_k Y_k(x+mu) X_k(x)^dag      (x even)
    W = -sum_k c_k X_k(x+mu) Y_k(x)^dag     (x odd),

and the molecular-dynamics force is F = -dS_f/dw.  The sign and factor are
checked against finite differences of S_f in the tests.
"""
from __future__ import annotations

import numpy as np

from . import dirac
from . import lattice as L
from .solvers import multishift_cg, vdot
from .su3 import T


def rational_solve(U, dims, mass, b, rat, tol, maxiter=100000):
    """x_k = (A + pole_k)^{-1} b for every pole of ``rat`` (dict or Rational)."""
    poles = rat["pole"] if isinstance(rat, dict) else rat.pole
    return multishift_cg(lambda v: dirac.apply_A(U, v, dims, mass), b, poles, tol, maxiter)


def rational_apply(U, dims, mass, b, rat, tol, maxiter=100000):
    """r(A) b = c0 b + sum_k c_k (A + d_k)^{-1} b."""
    c0 = rat["c0"] if isinstance(rat, dict) else rat.c0
    res = rat["residue"] if isinstance(rat, dict) else rat.residue
    sol = rational_solve(U, dims, mass, b, rat, tol, maxiter)
    out = c0 * b
    for c, x in zip(res, sol["x"]):
        out = out + c * x
    return out


def chiral_condensate(U, dims, mass, etas, tol) -> tuple[float, float]:
    """Stochastic estimate of (1/V) Tr M^{-1}, M = 2m + D (one staggered field).

    M^{-1} = (2m - D)(4m^2 - D^2)^{-1}; D changes parity while (4m^2 - D^2)^{-1}
    keeps it, so only 2m (4m^2 - D^2)^{-1} contributes to the trace, and its
    even and odd blocks (4m^2 - D_eo D_oe and 4m^2 - D_oe D_eo) have the same
    spectrum: Tr M^{-1} = 4m Tr_e A^{-1}.  With noise eta on the even sites,
    E[eta eta^dag] = 1, Tr_e A^{-1} = E[Re eta^dag A^{-1} eta].  Returns the
    mean over the given noise vectors and its standard error."""
    V = L.volume(dims)
    vals = []
    for eta in etas:
        x = multishift_cg(lambda v: dirac.apply_A(U, v, dims, mass), eta, [0.0], tol)["x"][0]
        vals.append(4.0 * mass * float(vdot(eta, x).real) / V)
    vals = np.array(vals)
    err = float(vals.std(ddof=1) / np.sqrt(len(vals))) if len(vals) > 1 else 0.0
    return float(vals.mean()), err


def fermion_action(U, dims, mass, phi, rat, tol) -> float:
    return float(vdot(phi, rational_apply(U, dims, mass, phi, rat, tol)).real)


def fermion_force(U, dims, mass, phi, rat, tol) -> np.ndarray:
    """F_a(x, mu) = 2 Im tr(T_a s U_mu(x) W(x, mu)), shape (Nt,Nz,Ny,Nx,4,8)."""
    res = rat["residue"] if isinstance(rat, dict) else rat.residue
    sol = rational_solve(U, dims, mass, phi, rat, tol)
    return force_from_solutions(U, dims, sol["x"], res)


def force_from_solutions(U, dims, xs, res) -> np.ndarray:
    """The force above from given X_k (even half vectors) and residues c_k."""
    par = L.parity(dims)
    eps = np.where(par == 0, 1.0, -1.0)
    # chi_k: X_k on even sites, Y_k = D_oe X_k on odd sites
    chis = []
    for x in xs:
        y = dirac.dslash_half(U, x, dims, 1)
        chis.append(L.half_to_full(x, dims, 0) + L.half_to_full(y, dims, 1))
    ut = dirac.dressed_links(U, dims)
    nx, ny, nz, nt = dims
    F = np.zeros((nt, nz, ny, nx, 4, 8))
    for mu in range(4):
        W = np.zeros((nt, nz, ny, nx, 3, 3), dtype=np.complex128)
        for c, chi in zip(res, chis):
            W += c * np.einsum("...a,...b->...ab", L.fwd(chi, mu), chi.conj())
        W *= eps[..., None, None]
        M = np.einsum("...ij,...jk->...ik", ut[..., mu, :, :], W)
        F[..., mu, :] = 2 * np.einsum("aij,...ji->...a", T, M).imag
    return F
