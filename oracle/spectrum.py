"""Spectral range of the half-lattice operator and the check of a rational
table's interval against it (test infrastructure; paper Appendix, where the
approximation interval must reach below the smallest eigenvalue (2ma)^2 and
above the largest one).

A = 4m^2 - D_eo D_oe = 4m^2 + D_oe^dag D_oe (Sec. 3.2), so
* 4m^2 is a lower bound of the spectrum, reached exactly when D_oe has a
  kernel and approached closely on rough fields;
* |D_oe| <= 8 (eight hops, each a unitary link times a sign), so 4m^2 + 64
  is a certain upper bound;
* the Rayleigh quotient <v, A v> / <v, v> of any v is at most lambda_max, and
  for v = A^k v0 it rises to lambda_max as k grows (power iteration).

The check: the interval [xmin, xmax] of a table covers the spectrum when
xmin <= 4m^2 and either xmax >= 4m^2 + 64 (certain) or (1 + margin) times the
power-iteration estimate is <= xmax (the estimate is approached from below,
hence the margin).
"""
from __future__ import annotations

import numpy as np

from . import dirac

CERTAIN_GAP = 64.0   # |D_oe|^2 <= 64


def power_rayleigh(U, dims, mass, v0, iters: int) -> float:
    """Rayleigh quotient of A after `iters` power iterations from v0 (the
    vector is normalised after every application; the quotient does not
    depend on the scale)."""
    v = np.array(v0, dtype=np.complex128)
    v /= np.linalg.norm(v)
    for _ in range(iters):
        v = dirac.apply_A(U, v, dims, mass)
        v /= np.linalg.norm(v)
    Av = dirac.apply_A(U, v, dims, mass)
    return float(np.vdot(v, Av).real / np.vdot(v, v).real)


def interval_covers(mass, xmin, xmax, lam_est, margin) -> bool:
    """The rule above, for a power-iteration estimate lam_est."""
    lo = 4.0 * mass * mass
    if xmin > lo:
        return False
    if xmax >= lo + CERTAIN_GAP:
        return True
    return (1.0 + margin) * lam_est <= xmax
