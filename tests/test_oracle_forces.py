"""Pins for the oracle's gauge and fermion forces and the link update: finite
differences of the actions, gauge covariance, exp(iX) against scipy."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import fermion, gauge, hmc
from oracle import lattice as L
from oracle.su3 import expi, reunitarise, to_matrix

DIMS = (4, 4, 2, 4)


def _links(kind, eps=0.5):
    rng = synth.make_rng(902, kind)
    return synth.random_su3_near_identity(DIMS, eps, rng), rng


def _move(U, omega, h):
    return np.einsum("...ij,...jk->...ik", expi(h * to_matrix(omega)), U)


def _fd(action, U, omega, h=1e-4):
    return (action(_move(U, omega, h)) - action(_move(U, omega, -h))) / (2 * h)


def test_gauge_action_unit_and_strong_coupling_free():
    nx, ny, nz, nt = DIMS
    U = np.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    assert gauge.gauge_action(U, DIMS, 5.4) == 0.0
    assert gauge.mean_plaquette(U, DIMS) == pytest.approx(1.0)
    # Haar links: <Re tr P / 3> = 0 in expectation (strong-coupling limit beta -> 0)
    Uh = synth.haar_su3((8, 8, 8, 8), synth.make_rng(902, 9))
    assert abs(gauge.mean_plaquette(Uh, (8, 8, 8, 8))) < 0.02


def test_gauge_force_finite_difference():
    U, rng = _links(1)
    beta = 5.4
    F = gauge.gauge_force(U, DIMS, beta)
    for trial in range(2):
        omega = rng.standard_normal(F.shape)
        fd = _fd(lambda u: gauge.gauge_action(u, DIMS, beta), U, omega)
        an = -np.sum(omega * F)
        assert abs(fd - an) <= 1e-7 * abs(an)


def test_fermion_force_finite_difference():
    U, rng = _links(2)
    rat = synth.load_rational("xm050_n8_m0.1")
    m = 0.1
    phi = synth.gaussian_half_vector(DIMS, rng)
    F = fermion.fermion_force(U, DIMS, m, phi, rat, 1e-13)
    for trial in range(2):
        omega = rng.standard_normal(F.shape)
        fd = _fd(lambda u: fermion.fermion_action(u, DIMS, m, phi, rat, 1e-13), U, omega)
        an = -np.sum(omega * F)
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_forces_gauge_covariant():
    """Under U -> Om U Om(x+mu)^dag, phi -> Om phi the force matrices rotate
    as F -> Om F Om^dag (the 8 coordinates are those of the rotated matrix)."""
    U, rng = _links(3)
    Om = synth.haar_su3(DIMS, rng)[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(DIMS, rng)
    phig = np.einsum("kij,kj->ki", L.full_to_half(Om, DIMS, 0), phi)
    from oracle.su3 import to_coords
    for f, fg in [(gauge.gauge_force(U, DIMS, 5.4), gauge.gauge_force(Ug, DIMS, 5.4)),
                  (fermion.fermion_force(U, DIMS, 0.1, phi, rat, 1e-13),
                   fermion.fermion_force(Ug, DIMS, 0.1, phig, rat, 1e-13))]:
        rot = to_coords(np.einsum("...ij,...mjk,...lk->...mil", Om, to_matrix(f), Om.conj()))
        assert np.abs(rot - fg).max() < 1e-9 * np.abs(f).max()


def test_expi_matches_scipy_and_reunitarise():
    rng = synth.make_rng(902, 4)
    X = to_matrix(rng.standard_normal((20, 8)))
    E = expi(X)
    for k in range(20):
        assert np.abs(E[k] - scipy.linalg.expm(1j * X[k])).max() < 1e-14
    assert np.abs(np.einsum("kij,kjl->kil", E, expi(-X)) - np.eye(3)).max() < 1e-14
    # reunitarise: identity on SU(3), and maps a perturbed matrix to SU(3)
    U = synth.haar_su3((2, 2, 2, 2), rng)
    assert np.abs(reunitarise(U) - U).max() < 1e-14
    Up = reunitarise(U + 1e-3 * rng.standard_normal(U.shape))
    assert np.abs(np.einsum("...ji,...jk->...ik", Up.conj(), Up) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(Up) - 1).max() < 1e-14


def test_link_update_is_md_flow():
    """d/dt U = i p U: one tiny step agrees with the first-order flow."""
    U, rng = _links(5)
    P = rng.standard_normal(U.shape[:-2] + (8,))
    dt = 1e-6
    U1 = hmc.link_update(U, P, dt)
    dU = (U1 - U) / dt
    expect = 1j * np.einsum("...ij,...jk->...ik", to_matrix(P), U)
    assert np.abs(dU - expect).max() < 1e-5
