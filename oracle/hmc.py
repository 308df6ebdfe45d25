"""RHMC trajectory (paper Sec. 3.1, with the rational functions of Sec. 4).

Step 1: Gaussian momenta p (H = p^2/2 + S) and the pseudofermion heat bath
        phi = (M^dag M)^{alpha/2} xi with alpha = 1/2 on the even sub-lattice,
        i.e. phi = r_{+1/4}(A) xi, xi drawn with density exp(-xi^dag xi).
Step 2: molecular dynamics dU/dt = i p U, dp/dt = F = -dS/dw, integrated with
        leapfrog (reading: the paper does not name the integrator):
            p += dt/2 F(U); [U = exp(i dt p) U; p += dt F(U)] x (N-1);
            U = exp(i dt p) U; p += dt/2 F(U).
Step 3: Metropolis with P_acc = min(1, exp(-dH)); U is restored on rejection.

The fermion action at both ends uses the action's rational function
r_{-1/2}(A) explicitly (S_f = phi^dag r_{-1/2}(A) phi), so the accept/reject
step is exact for the rational action.  Kinetic term: K = (1/2) sum_a p_a^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fermion, gauge, naik
from .su3 import expi, reunitarise, to_matrix


def kinetic(P: np.ndarray) -> float:
    return 0.5 * float(np.sum(P * P))


def link_update(U: np.ndarray, P: np.ndarray, dt: float) -> np.ndarray:
    """U <- reunitarise(exp(i dt p) U)."""
    E = expi(dt * to_matrix(P))
    return reunitarise(np.einsum("...ij,...jk->...ik", E, U))


@dataclass
class HMCParams:
    beta: float
    mass: float
    tau: float
    n_steps: int
    r_md: dict          # force rational function (x^-1/2)
    r_action: dict      # action rational function (x^-1/2)
    r_heatbath: dict    # heat-bath rational function (x^+1/4)
    tol_md: float = 1e-10
    tol_action: float = 1e-12
    naik: tuple | None = None   # (c1, c3): the improved operator (Sec. 8 Summary) instead of the one-hop one


def _fermion_force(U, dims, prm, phi, rat, tol):
    if prm.naik:
        return naik.fermion_force(U, dims, prm.mass, phi, rat, tol, *prm.naik)
    return fermion.fermion_force(U, dims, prm.mass, phi, rat, tol)


def _fermion_action(U, dims, prm, phi, rat, tol):
    if prm.naik:
        return naik.fermion_action(U, dims, prm.mass, phi, rat, tol, *prm.naik)
    return fermion.fermion_action(U, dims, prm.mass, phi, rat, tol)


def total_force(U, dims, prm: HMCParams, phi):
    F = gauge.gauge_force(U, dims, prm.beta)
    if phi is not None:
        F = F + _fermion_force(U, dims, prm, phi, prm.r_md, prm.tol_md)
    return F


def hamiltonian(U, P, dims, prm: HMCParams, phi):
    K = kinetic(P)
    Sg = gauge.gauge_action(U, dims, prm.beta)
    Sf = 0.0 if phi is None else _fermion_action(U, dims, prm, phi, prm.r_action, prm.tol_action)
    return K, Sg, Sf


def leapfrog(U, P, dims, prm: HMCParams, phi, force=None):
    """Integrate tau with n_steps leapfrog steps; returns (U, P)."""
    force = force or (lambda u: total_force(u, dims, prm, phi))
    dt = prm.tau / prm.n_steps
    P = P + 0.5 * dt * force(U)
    for step in range(prm.n_steps):
        U = link_update(U, P, dt)
        P = P + (dt if step < prm.n_steps - 1 else 0.5 * dt) * force(U)
    return U, P


def heatbath(U, dims, mass, xi, r_hb, tol, naik_weights=None):
    if naik_weights:
        sol = naik.rational_solve(U, dims, mass, xi, r_hb, tol, *naik_weights)
        out = r_hb["c0"] * xi
        for c, x in zip(r_hb["residue"], sol["x"]):
            out = out + c * x
        return out
    return fermion.rational_apply(U, dims, mass, xi, r_hb, tol)


def trajectory(U0, dims, prm: HMCParams, P0, xi, u, with_fermions=True):
    """One trajectory with given momenta P0, noise xi and Metropolis uniform u."""
    phi = heatbath(U0, dims, prm.mass, xi, prm.r_heatbath, prm.tol_action, prm.naik) if with_fermions else None
    K0, Sg0, Sf0 = hamiltonian(U0, P0, dims, prm, phi)
    U1, P1 = leapfrog(U0, P0, dims, prm, phi)
    K1, Sg1, Sf1 = hamiltonian(U1, P1, dims, prm, phi)
    dH = (K1 + Sg1 + Sf1) - (K0 + Sg0 + Sf0)
    accepted = bool(u < np.exp(-dH))
    return {"dH": dH, "accepted": accepted, "U": U1 if accepted else U0, "U_proposed": U1,
            "P": P1, "phi": phi, "H0": (K0, Sg0, Sf0), "H1": (K1, Sg1, Sf1),
            "plaquette": gauge.mean_plaquette(U1 if accepted else U0, dims)}
