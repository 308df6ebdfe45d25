"""Staggered Dirac operator and the half-lattice operator (paper Sec. 3.2).

M_ik = 2m delta_ik + sum_mu ( U_{i,mu} delta_{i,k-mu} - U^dag_{i-mu,mu} delta_{i,k+mu} ),
with the staggered phases and the antiperiodic time factor absorbed into U.
Writing D for the hopping part, M = 2m + D with D^dag = -D, and D only connects
sites of opposite parity, so M = [[2m, D_eo], [D_oe, 2m]] in the even/odd split
and (M^dag M)_ee = 4m^2 - D_eo D_oe.  (The paper's block notation uses m for
the diagonal 2m; the mass of a configuration enters as 2m.)

The functions below act on full-lattice arrays (zero on the parity that is not
in use) so that no checkerboard index arithmetic is needed; ``*_half`` variants
take and return canonical half vectors (V/2, 3).
"""
from __future__ import annotations

import numpy as np

from . import lattice as L


def dressed_links(U: np.ndarray, dims) -> np.ndarray:
    """s_mu(x) U_mu(x): links with the staggered phase and boundary sign."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = L.staggered_sign(dims, mu)[..., None, None] * U[..., mu, :, :]
    return out


def dslash(U: np.ndarray, psi: np.ndarray, dims) -> np.ndarray:
    """(D psi)(x) = sum_mu [ Ut_mu(x) psi(x+mu) - Ut_mu(x-mu)^dag psi(x-mu) ]."""
    ut = dressed_links(U, dims)
    out = np.zeros_like(psi)
    for mu in range(4):
        u = ut[..., mu, :, :]
        out += np.einsum("...ab,...b->...a", u, L.fwd(psi, mu))
        out -= L.bwd(np.einsum("...ba,...b->...a", u.conj(), psi), mu)
    return out


def dslash_half(U: np.ndarray, vin: np.ndarray, dims, out_parity: int) -> np.ndarray:
    """D_oe (out_parity=1, even input) or D_eo (out_parity=0, odd input) on half vectors."""
    full = L.half_to_full(vin, dims, 1 - out_parity)
    return L.full_to_half(dslash(U, full, dims), dims, out_parity)


def apply_A(U: np.ndarray, chi: np.ndarray, dims, mass: float) -> np.ndarray:
    """Half-lattice operator A = (M^dag M)_ee = 4 m^2 - D_eo D_oe on an even half vector."""
    return 4 * mass * mass * chi - dslash_half(U, dslash_half(U, chi, dims, 1), dims, 0)


def dense_dslash(U: np.ndarray, dims) -> np.ndarray:
    """The full 3V x 3V hopping matrix D, built entry by entry from the defining
    formula with plain loops (tiny lattices only).  Rows/cols: 3*l + colour."""
    nx, ny, nz, nt = dims
    n = [nx, ny, nz, nt]
    V = nx * ny * nz * nt
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)

    def addr(c):
        return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))

    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    c = [x, y, z, t]
                    i = addr(c)
                    for mu in range(4):
                        eta = (-1) ** sum(c[:mu])
                        # forward hop: link (x, mu), sign flips if it crosses the t boundary
                        cp = list(c)
                        cp[mu] = (c[mu] + 1) % n[mu]
                        sf = eta * (-1 if (mu == 3 and c[3] == nt - 1) else 1)
                        k = addr(cp)
                        D[3 * i:3 * i + 3, 3 * k:3 * k + 3] += sf * U[t, z, y, x, mu]
                        # backward hop: link (x - mu, mu)
                        cm = list(c)
                        cm[mu] = (c[mu] - 1) % n[mu]
                        sb = eta * (-1 if (mu == 3 and cm[3] == nt - 1) else 1)
                        k = addr(cm)
                        ul = U[cm[3], cm[2], cm[1], cm[0], mu]
                        D[3 * i:3 * i + 3, 3 * k:3 * k + 3] -= sb * ul.conj().T
    return D
