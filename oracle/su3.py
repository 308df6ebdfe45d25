"""SU(3) helpers: algebra coordinates, exp(iX), reunitarisation.

Momenta and forces are traceless Hermitian matrices X = sum_a X_a T_a with
T_a = lambda_a / 2 (Gell-Mann), stored as their 8 real coordinates
X_a = 2 tr(T_a X).  The molecular-dynamics equation for the links, dU/dt = i p U
(Sec. 3.1), makes exp(i dt p) U the link update.
"""
from __future__ import annotations

import numpy as np


def generators() -> np.ndarray:
    """T_a = lambda_a/2, shape (8,3,3); tr(T_a T_b) = delta_ab / 2."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


T = generators()


def to_matrix(coef: np.ndarray) -> np.ndarray:
    """sum_a coef_a T_a for coef of shape (..., 8)."""
    return np.einsum("...a,aij->...ij", coef, T)


def to_coords(mat: np.ndarray) -> np.ndarray:
    """X_a = 2 Re tr(T_a X) for Hermitian X (..., 3, 3)."""
    return 2 * np.einsum("aij,...ji->...a", T, mat).real


def dagger(m: np.ndarray) -> np.ndarray:
    return np.swapaxes(m, -1, -2).conj()


def expi(herm: np.ndarray) -> np.ndarray:
    """exp(i H) for Hermitian H, via the eigen-decomposition H = V diag(l) V^dag."""
    lam, vec = np.linalg.eigh(herm)
    return np.einsum("...ia,...a,...ja->...ij", vec, np.exp(1j * lam), vec.conj())


def reunitarise(u: np.ndarray) -> np.ndarray:
    """Project a near-SU(3) matrix back onto SU(3): normalise row 0, make row 1
    orthogonal to it and normalise (Gram-Schmidt), row 2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.sqrt(np.sum(np.abs(r0) ** 2, axis=-1, keepdims=True))
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1, keepdims=True))
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=-2)
