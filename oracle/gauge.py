"""Plaquette (Wilson) gauge action and its force (paper eq. pfact, second term).

Reading of eq. (pfact): the paper writes (1/(6g^2)) sum_{mu,nu} (3 - tr box),
and quotes the coupling "1/(6g^2) = 5.6", a value that only makes sense as the
usual beta = 6/g^2.  The standard form is used:

    S_g = beta * sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3),
    P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,

on plain links (the staggered phases and the fermion boundary sign belong to
the Dirac operator, not to the gauge action).

Force: for U_mu(x) -> exp(i w_a T_a) U_mu(x),
    dS_g/dw_a = (beta/3) Im tr(T_a U_mu(x) A_mu(x)),
with A_mu(x) the sum of the six staples that close the plaquettes through the
link; the molecular-dynamics force is F = -dS/dw.
"""
from __future__ import annotations

import numpy as np

from . import lattice as L
from .su3 import T, dagger


def _mm(a, b):
    return np.einsum("...ij,...jk->...ik", a, b)


def plaquette(U, mu, nu):
    u_mu = U[..., mu, :, :]
    u_nu = U[..., nu, :, :]
    return _mm(_mm(u_mu, L.fwd(u_nu, mu)), _mm(dagger(L.fwd(u_mu, nu)), dagger(u_nu)))


def mean_plaquette(U, dims) -> float:
    """< Re tr P / 3 > over all sites and the 6 planes."""
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            acc += np.trace(plaquette(U, mu, nu), axis1=-2, axis2=-1).real.sum() / 3
    return acc / (6 * L.volume(dims))


def polyakov_loop(U, dims) -> complex:
    """Spatial average of (1/3) tr of the ordered product of the time links
    U_t(x,0) U_t(x,1) ... U_t(x,N_t-1) at every spatial site x: the Wilson line
    that closes around the periodic time direction, a gauge-invariant
    observable of the sampled configurations (expectation values of Sec. 2)."""
    nt = dims[3]
    ut = U[..., 3, :, :]  # (t, z, y, x, 3, 3)
    P = ut[0]
    for t in range(1, nt):
        P = _mm(P, ut[t])
    return complex(np.trace(P, axis1=-2, axis2=-1).mean() / 3)


def gauge_action(U, dims, beta: float) -> float:
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            acc += (1 - np.trace(plaquette(U, mu, nu), axis1=-2, axis2=-1).real / 3).sum()
    return beta * acc


def staples(U, mu):
    """A_mu(x) = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                                 + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) ]."""
    u_mu = U[..., mu, :, :]
    A = np.zeros_like(u_mu)
    for nu in range(4):
        if nu == mu:
            continue
        u_nu = U[..., nu, :, :]
        A += _mm(_mm(L.fwd(u_nu, mu), dagger(L.fwd(u_mu, nu))), dagger(u_nu))
        # lower staple: all factors live at x - nu (and x + mu - nu)
        low = _mm(_mm(dagger(L.fwd(u_nu, mu)), dagger(u_mu)), u_nu)
        A += L.bwd(low, nu)
    return A


def gauge_force(U, dims, beta: float) -> np.ndarray:
    """F_a(x, mu) = -(beta/3) Im tr(T_a U_mu(x) A_mu(x)), shape (Nt,Nz,Ny,Nx,4,8)."""
    nx, ny, nz, nt = dims
    F = np.zeros((nt, nz, ny, nx, 4, 8))
    for mu in range(4):
        M = _mm(U[..., mu, :, :], staples(U, mu))
        F[..., mu, :] = -(beta / 3) * np.einsum("aij,...ji->...a", T, M).imag
    return F
