"""Seeded field factories in the canonical boundary layouts.

Canonical layouts (all complex128 / float64, C order):

* gauge field  ``U[t, z, y, x, mu, a, b]``  -- SU(3) link from site x in
  direction mu (mu = 0,1,2,3 for x,y,z,t); a,b are colour row/column.  The site
  address in C order is ``l = x + Nx*(y + Ny*(z + Nz*t))``, the 0-based form of
  the lexicographic address of Sec. 2 of the paper.
* half vector  ``psi[k, a]`` -- colour vector on the k-th site of one
  checkerboard parity ((x+y+z+t) mod 2), counted in lexicographic order.
* momentum     ``P[t, z, y, x, mu, c]`` -- the 8 real coordinates of a
  traceless Hermitian matrix in the basis T_c = lambda_c / 2.

Seeds: ``SeedSequence([0x171009178, config, kind])``.  The generators draw
random numbers and do the minimal linear algebra needed to turn them into group
elements (an eigen-decomposition to exponentiate a random Hermitian matrix, a
QR for Haar elements, an SVD to clean the result onto SU(3)).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0x171009178


def make_rng(config: int, kind: int) -> np.random.Generator:
    """numpy Generator seeded by SeedSequence([SEED_BASE, config, kind])."""
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, int(config), int(kind)]))


def lattice_volume(dims) -> int:
    nx, ny, nz, nt = dims
    return int(nx) * int(ny) * int(nz) * int(nt)


def _gell_mann() -> np.ndarray:
    """The 8 Gell-Mann matrices lambda_1..lambda_8, shape (8,3,3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1] = -1j
    lam[1, 1, 0] = 1j
    lam[2, 0, 0] = 1
    lam[2, 1, 1] = -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2] = -1j
    lam[4, 2, 0] = 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2] = -1j
    lam[6, 2, 1] = 1j
    lam[7, 0, 0] = lam[7, 1, 1] = 1 / np.sqrt(3)
    lam[7, 2, 2] = -2 / np.sqrt(3)
    return lam


def _clean_su3(m: np.ndarray) -> np.ndarray:
    """Nearest unitary (polar factor W V^dagger of the SVD), then det -> 1."""
    w, _, vh = np.linalg.svd(m)
    u = w @ vh
    det = np.linalg.det(u)
    return u / (det ** (1.0 / 3.0))[..., None, None]


def random_su3_near_identity(dims, eps: float, rng: np.random.Generator) -> np.ndarray:
    """U = exp(i*eps*H) per link, H = sum_a h_a lambda_a/2 with h_a ~ N(0,1).

    Returns the canonical gauge array of shape (Nt,Nz,Ny,Nx,4,3,3).
    """
    nx, ny, nz, nt = dims
    shape = (nt, nz, ny, nx, 4)
    h = rng.standard_normal(shape + (8,))
    herm = np.einsum("...a,aij->...ij", h, _gell_mann() / 2)
    lam, vec = np.linalg.eigh(herm)
    u = np.einsum("...ia,...a,...ja->...ij", vec, np.exp(1j * eps * lam), vec.conj())
    return _clean_su3(u)


def haar_su3(dims, rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(3) links (QR of a complex Ginibre matrix with the
    diagonal phase fix of Mezzadri, Notices AMS 54 (2007) 592), det -> 1."""
    nx, ny, nz, nt = dims
    shape = (nt, nz, ny, nx, 4, 3, 3)
    z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


def gaussian_half_vector(dims, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Half-lattice colour vector (V/2, 3) complex; each real component ~ N(0, scale^2)."""
    vh = lattice_volume(dims) // 2
    return scale * (rng.standard_normal((vh, 3)) + 1j * rng.standard_normal((vh, 3)))


def gaussian_momentum(dims, rng: np.random.Generator) -> np.ndarray:
    """Momentum coordinates (Nt,Nz,Ny,Nx,4,8), each ~ N(0,1)."""
    nx, ny, nz, nt = dims
    return rng.standard_normal((nt, nz, ny, nx, 4, 8))


def load_rational(name: str) -> dict:
    """Read a stored rational-approximation table (c0, residue[], pole[], ...)
    from ``synth/rational/<name>.json``."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rational", name + ".json")
    with open(path) as f:
        return json.load(f)
