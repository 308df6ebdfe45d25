"""Naik-improved staggered hopping operator -- TEST INFRASTRUCTURE ONLY.

The paper's Summary (Sec. 8) names "improved" staggered quarks, whose
operator reaches deeper than one site, as the next workload after the naive
operator of Sec. 3.2; it gives no formula.  Reading used here (the standard
tree-level Naik improvement): the one-hop term of Sec. 3.2 is weighted by c1
and a three-hop term, parallel-transported along the three links of the
straight path, is added with weight c3:

  (D psi)(x) = sum_mu { c1 [ Ut_mu(x) psi(x+mu) - Ut_mu(x-mu)^dag psi(x-mu) ]
                      + c3 [ Ut_mu(x) Ut_mu(x+mu) Ut_mu(x+2mu) psi(x+3mu)
                             - Ut_mu(x-mu)^dag Ut_mu(x-2mu)^dag Ut_mu(x-3mu)^dag psi(x-3mu) ] }

with Ut the links dressed with the staggered phase and the antiperiodic time
sign (exactly as in the naive operator), c1 = 9/8 and c3 = -1/24.  These two
numbers are the unique pair for which the free dispersion
c1 sin p + c3 sin 3p equals p up to O(p^5) (tree-level removal of the O(a^2)
error).  Because eta_mu(x) does not depend on x_mu, the product of the three
dressed links carries the phase eta_mu(x) once and one time-boundary sign per
crossing of the boundary.  A three-hop changes the parity, so the even-odd
block form of Sec. 3.2, D^dag = -D, and A = 4m^2 - D_eo D_oe carry over.

The operator here is written as that path definition with no precomputed long
links; the dense builder walks the path link by link.
"""
from __future__ import annotations

import numpy as np

from . import dirac
from . import lattice as L
from .solvers import multishift_cg, vdot
from .su3 import T

C1 = 9.0 / 8.0
C3 = -1.0 / 24.0


def _mv(u, v):
    return np.einsum("...ab,...b->...a", u, v)


def _mhv(u, v):
    """u^dag v per site."""
    return np.einsum("...ba,...b->...a", u.conj(), v)


def dslash(U: np.ndarray, psi: np.ndarray, dims, c1: float = C1, c3: float = C3) -> np.ndarray:
    """The improved hopping operator on a full-lattice field (path definition)."""
    ut = dirac.dressed_links(U, dims)
    out = np.zeros_like(psi)
    for mu in range(4):
        u = ut[..., mu, :, :]
        # one hop
        out += c1 * _mv(u, L.fwd(psi, mu))
        out -= c1 * L.bwd(_mhv(u, psi), mu)
        # three hops forward: Ut(x) [Ut(x+mu) [Ut(x+2mu) psi(x+3mu)]]
        v = L.fwd(L.fwd(L.fwd(psi, mu), mu), mu)          # psi(x+3mu)
        v = _mv(L.fwd(L.fwd(u, mu), mu), v)               # Ut(x+2mu) psi(x+3mu)
        v = _mv(L.fwd(u, mu), v)                          # Ut(x+mu) ...
        v = _mv(u, v)                                     # Ut(x) ...
        out += c3 * v
        # three hops backward: Ut(x-mu)^dag Ut(x-2mu)^dag Ut(x-3mu)^dag psi(x-3mu)
        w = _mhv(L.bwd(L.bwd(L.bwd(u, mu), mu), mu), L.bwd(L.bwd(L.bwd(psi, mu), mu), mu))
        w = _mhv(L.bwd(L.bwd(u, mu), mu), w)
        w = _mhv(L.bwd(u, mu), w)
        out -= c3 * w
    return out


def dslash_half(U: np.ndarray, vin: np.ndarray, dims, out_parity: int, c1: float = C1,
                c3: float = C3) -> np.ndarray:
    """D_oe (out_parity=1, even input) or D_eo (out_parity=0, odd input) on half vectors."""
    full = L.half_to_full(vin, dims, 1 - out_parity)
    return L.full_to_half(dslash(U, full, dims, c1, c3), dims, out_parity)


def apply_A(U: np.ndarray, chi: np.ndarray, dims, mass: float, c1: float = C1, c3: float = C3) -> np.ndarray:
    """A = 4 m^2 - D_eo D_oe with the improved D, on an even half vector."""
    y = dslash_half(U, chi, dims, 1, c1, c3)
    return 4 * mass * mass * chi - dslash_half(U, y, dims, 0, c1, c3)


def dense_dslash(U: np.ndarray, dims, c1: float = C1, c3: float = C3) -> np.ndarray:
    """The full 3V x 3V improved hopping matrix, entry by entry with plain
    loops: every term walks its path one link at a time, multiplying the
    staggered phase and, per link that leaves the last time slice, -1
    (tiny lattices only).  Rows/cols: 3*l + colour."""
    nx, ny, nz, nt = dims
    n = [nx, ny, nz, nt]
    V = nx * ny * nz * nt
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)

    def addr(c):
        return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))

    def link(c, mu):
        """dressed link on (c, mu)"""
        eta = (-1) ** sum(c[:mu])
        bc = -1 if (mu == 3 and c[3] == nt - 1) else 1
        return eta * bc * U[c[3], c[2], c[1], c[0], mu]

    def step(c, mu, d):
        cc = list(c)
        cc[mu] = (c[mu] + d) % n[mu]
        return cc

    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    c = [x, y, z, t]
                    i = addr(c)
                    for mu in range(4):
                        for hops, w in ((1, c1), (3, c3)):
                            # forward path x -> x+hops*mu: product of the links it walks
                            P = np.eye(3, dtype=np.complex128)
                            cur = c
                            for _ in range(hops):
                                P = P @ link(cur, mu)
                                cur = step(cur, mu, 1)
                            k = addr(cur)
                            D[3 * i:3 * i + 3, 3 * k:3 * k + 3] += w * P
                            # backward path x -> x-hops*mu: adjoints of the links it walks back over
                            P = np.eye(3, dtype=np.complex128)
                            cur = c
                            for _ in range(hops):
                                cur = step(cur, mu, -1)
                                P = P @ link(cur, mu).conj().T
                            k = addr(cur)
                            D[3 * i:3 * i + 3, 3 * k:3 * k + 3] -= w * P
    return D


def free_eigenvalue(p, mass: float, c1: float = C1, c3: float = C3) -> float:
    """A's eigenvalue on a plane wave of momentum p at U = 1:
    4 m^2 + 4 sum_mu (c1 sin p_mu + c3 sin 3 p_mu)^2."""
    return 4 * mass * mass + 4 * sum((c1 * np.sin(q) + c3 * np.sin(3 * q)) ** 2 for q in p)


# ---- pseudofermion action and force of the improved operator ------------
#
# S_f = c0 |phi|^2 + sum_k c_k Re <phi, X_k>, X_k = (A + d_k)^{-1} phi with the
# improved A.  With chi_k = X_k on even and Y_k = D_oe X_k on odd sites
# (improved D_oe), eps = +1 / -1 on even / odd sites and
#   W1(x, mu) = eps(x) sum_k c_k chi_k(x+mu)  chi_k(x)^dag,
#   W3(x, mu) = eps(x) sum_k c_k chi_k(x+3mu) chi_k(x)^dag,
# the variation U_mu(z) -> exp(i w_a T_a) U_mu(z) of every dressed link
# (phase and boundary sign included) that D contains gives F = -dS/dw:
#   F_a(z, mu) = 2 c1 Im tr(T_a Ut(z) W1(z))
#              + 2 c3 Im tr(T_a Ut(z) [ Ut(z+mu) Ut(z+2mu) W3(z)
#                                        + Ut(z+mu) W3(z-mu) Ut(z-mu)
#                                        + W3(z-2mu) Ut(z-2mu) Ut(z-mu) ]),
# the three terms being the link's positions 0, 1, 2 in the three-link paths
# that start at z, z-mu and z-2mu.  (The one-hop term is the derivation of the
# plain operator's force, weighted by c1.)  Sign and factor are pinned by
# finite differences of S_f in the tests, not trusted.


def rational_solve(U, dims, mass, b, rat, tol, c1=C1, c3=C3, maxiter=100000):
    return multishift_cg(lambda v: apply_A(U, v, dims, mass, c1, c3), b, rat["pole"], tol, maxiter)


def fermion_action(U, dims, mass, phi, rat, tol, c1=C1, c3=C3) -> float:
    sol = rational_solve(U, dims, mass, phi, rat, tol, c1, c3)
    out = rat["c0"] * phi
    for c, x in zip(rat["residue"], sol["x"]):
        out = out + c * x
    return float(vdot(phi, out).real)


def fermion_force(U, dims, mass, phi, rat, tol, c1=C1, c3=C3) -> np.ndarray:
    """F_a(x, mu) of the improved operator's rational action, shape (Nt,Nz,Ny,Nx,4,8)."""
    sol = rational_solve(U, dims, mass, phi, rat, tol, c1, c3)
    return force_from_solutions(U, dims, sol["x"], rat["residue"], c1, c3)


def force_from_solutions(U, dims, xs, res, c1=C1, c3=C3) -> np.ndarray:
    par = L.parity(dims)
    eps = np.where(par == 0, 1.0, -1.0)[..., None, None]
    chis = []
    for x in xs:
        y = dslash_half(U, x, dims, 1, c1, c3)
        chis.append(L.half_to_full(x, dims, 0) + L.half_to_full(y, dims, 1))
    ut = dirac.dressed_links(U, dims)
    nx, ny, nz, nt = dims
    F = np.zeros((nt, nz, ny, nx, 4, 8))
    mm = lambda a, b: np.einsum("...ij,...jk->...ik", a, b)  # noqa: E731
    for mu in range(4):
        u = ut[..., mu, :, :]
        W1 = np.zeros((nt, nz, ny, nx, 3, 3), dtype=np.complex128)
        W3 = np.zeros_like(W1)
        for c, chi in zip(res, chis):
            W1 += c * np.einsum("...a,...b->...ab", L.fwd(chi, mu), chi.conj())
            W3 += c * np.einsum("...a,...b->...ab", L.fwd(L.fwd(L.fwd(chi, mu), mu), mu), chi.conj())
        W1 *= eps
        W3 *= eps
        u_p1 = L.fwd(u, mu)                 # Ut(z+mu)
        u_p2 = L.fwd(u_p1, mu)              # Ut(z+2mu)
        u_m1 = L.bwd(u, mu)                 # Ut(z-mu)
        u_m2 = L.bwd(u_m1, mu)              # Ut(z-2mu)
        w3_m1 = L.bwd(W3, mu)               # W3(z-mu)
        w3_m2 = L.bwd(w3_m1, mu)            # W3(z-2mu)
        M3 = mm(mm(u_p1, u_p2), W3) + mm(mm(u_p1, w3_m1), u_m1) + mm(mm(w3_m2, u_m2), u_m1)
        M = c1 * mm(u, W1) + c3 * mm(u, M3)
        F[..., mu, :] = 2 * np.einsum("aij,...ji->...a", T, M).imag
    return F
