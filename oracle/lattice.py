"""Lattice geometry (paper Sec. 2 site address; Sec. 3.2 even/odd split).

Arrays over the lattice are indexed ``[t, z, y, x, ...]`` so that the C-order
flat index is the 0-based lexicographic address l = x + Nx(y + Ny(z + Nz t)).

Reading of Sec. 3.2: a site is even or odd by the parity of x+y+z+t (the
checkerboard of the paper's even-odd figure).  The text says "parity of the
address l", which for even Nx would be the parity of x alone and would not give
the block structure the section derives, so the checkerboard is used.

Staggered phases (absorbed into the links in Sec. 3.2) are the Kogut-Susskind
eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z); the
time boundary is antiperiodic, i.e. an extra -1 on the t-links leaving the last
time slice.
"""
from __future__ import annotations

import numpy as np

# lattice array axis of direction mu (0=x, 1=y, 2=z, 3=t) in [t,z,y,x,...] arrays
AXIS = (3, 2, 1, 0)


def volume(dims) -> int:
    nx, ny, nz, nt = dims
    return nx * ny * nz * nt


def coords(dims):
    """Integer coordinate arrays x, y, z, t of shape (Nt,Nz,Ny,Nx)."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z, t


def parity(dims) -> np.ndarray:
    x, y, z, t = coords(dims)
    return (x + y + z + t) % 2


def fwd(f: np.ndarray, mu: int) -> np.ndarray:
    """g(x) = f(x + mu-hat), periodic wrap."""
    return np.roll(f, -1, axis=AXIS[mu])


def bwd(f: np.ndarray, mu: int) -> np.ndarray:
    """g(x) = f(x - mu-hat), periodic wrap."""
    return np.roll(f, 1, axis=AXIS[mu])


def staggered_sign(dims, mu: int) -> np.ndarray:
    """eta_mu(x) times the antiperiodic-time factor of link (x, mu)."""
    x, y, z, t = coords(dims)
    nt = dims[3]
    if mu == 0:
        s = np.ones_like(x)
    elif mu == 1:
        s = (-1) ** x
    elif mu == 2:
        s = (-1) ** (x + y)
    else:
        s = (-1) ** (x + y + z) * np.where(t == nt - 1, -1, 1)
    return s.astype(np.float64)


def full_to_half(full: np.ndarray, dims, par: int) -> np.ndarray:
    """Sites of parity ``par`` in lexicographic order: (V/2, ...)."""
    mask = parity(dims).reshape(-1) == par
    return full.reshape((volume(dims),) + full.shape[4:])[mask]


def half_to_full(half: np.ndarray, dims, par: int) -> np.ndarray:
    """Embed a half-lattice field into a full one, zero on the other parity."""
    nx, ny, nz, nt = dims
    out = np.zeros((volume(dims),) + half.shape[1:], dtype=half.dtype)
    out[parity(dims).reshape(-1) == par] = half
    return out.reshape((nt, nz, ny, nx) + half.shape[1:])
