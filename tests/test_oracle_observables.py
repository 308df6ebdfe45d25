"""Pins for the oracle's Polyakov loop: unit links, a closed form for
constant diagonal time links, gauge invariance (which fails for the reversed
product) and the centre transformation (which tells tr P from its conjugate)."""
import numpy as np

import synth
from oracle import gauge, lattice as L

DIMS = (4, 2, 4, 6)


def _U(seed, eps=0.7):
    return synth.random_su3_near_identity(DIMS, eps, synth.make_rng(700, seed))


def test_unit_links_give_one():
    U = np.broadcast_to(np.eye(3, dtype=complex), (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3, 3)).copy()
    assert abs(gauge.polyakov_loop(U, DIMS) - 1.0) < 1e-15


def test_constant_diagonal_time_links_closed_form():
    U = _U(1)
    t1, t2 = 0.37, -1.1
    d = np.diag(np.exp(1j * np.array([t1, t2, -(t1 + t2)])))
    U[..., 3, :, :] = d
    nt = DIMS[3]
    exp = (np.exp(1j * nt * t1) + np.exp(1j * nt * t2) + np.exp(-1j * nt * (t1 + t2))) / 3
    assert abs(gauge.polyakov_loop(U, DIMS) - exp) < 1e-14


def test_gauge_invariance():
    U = _U(2)
    Om = synth.haar_su3(DIMS, synth.make_rng(700, 3))[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    p0 = gauge.polyakov_loop(U, DIMS)
    assert abs(gauge.polyakov_loop(Ug, DIMS) - p0) < 1e-13
    # the product taken in the opposite order is not invariant: the pin bites
    rev = U.copy()
    rev[..., 3, :, :] = U[::-1, ..., 3, :, :]
    revg = Ug.copy()
    revg[..., 3, :, :] = Ug[::-1, ..., 3, :, :]
    assert abs(gauge.polyakov_loop(revg, DIMS) - gauge.polyakov_loop(rev, DIMS)) > 1e-3


def test_centre_transformation_multiplies_by_z():
    U = _U(4)
    z = np.exp(2j * np.pi / 3)
    Uz = U.copy()
    Uz[0, ..., 3, :, :] *= z  # every time link leaving the t = 0 slice
    assert abs(gauge.polyakov_loop(Uz, DIMS) - z * gauge.polyakov_loop(U, DIMS)) < 1e-14
    assert abs(gauge.polyakov_loop(U, DIMS)) > 1e-3
