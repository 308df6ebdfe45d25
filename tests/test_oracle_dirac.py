"""Pins for the oracle's Dirac operator and half-lattice operator (paper Sec. 3.2)."""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice as L
from oracle.solvers import vdot


def _fields(dims, eps=0.3, kind=0):
    rng = synth.make_rng(900, kind)
    return synth.random_su3_near_identity(dims, eps, rng), rng


def _unit_links(dims):
    nx, ny, nz, nt = dims
    U = np.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_free_field_plane_wave(dims):
    """At U = 1 a plane wave e^{ip.x} with periodic spatial and antiperiodic
    temporal momenta gives (D_oe psi_e)(x) = sum_mu eta_mu(x) 2i sin(p_mu) psi(x)."""
    nx, ny, nz, nt = dims
    U = _unit_links(dims)
    x, y, z, t = L.coords(dims)
    p = (2 * np.pi * 1 / nx, 2 * np.pi * 1 / ny, 2 * np.pi * (nz // 2) / nz, (2 * 1 + 1) * np.pi / nt)
    c = np.array([0.3 + 0.1j, -0.7j, 0.5])
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None] * c
    eta = [np.ones_like(x), (-1.0) ** x, (-1.0) ** (x + y), (-1.0) ** (x + y + z)]
    factor = sum(eta[mu] * 2j * np.sin(p[mu]) for mu in range(4))
    expect = L.full_to_half(factor[..., None] * psi, dims, 1)
    got = dirac.dslash_half(U, L.full_to_half(psi, dims, 0), dims, 1)
    assert np.abs(got - expect).max() < 1e-13


def test_free_spectrum_4444():
    """A = 4m^2 + 4 sum_mu sin^2 p_mu at U = 1: on 4^4 with m = 0.1 the spectrum
    is {2.04, 6.04, 10.04, 14.04}."""
    dims = (4, 4, 4, 4)
    U = _unit_links(dims)
    m = 0.1
    vh = L.volume(dims) // 2
    cols = []
    for k in range(3 * vh):
        e = np.zeros((vh, 3), dtype=np.complex128)
        e.reshape(-1)[k] = 1
        cols.append(dirac.apply_A(U, e, dims, m).reshape(-1))
    A = np.array(cols).T
    ev = np.linalg.eigvalsh(A)
    assert np.allclose(sorted(set(np.round(ev, 10))), [2.04, 6.04, 10.04, 14.04])


def test_dense_bruteforce_2222_and_4444():
    """The roll-based operator equals the entry-by-entry dense matrix."""
    for dims in [(2, 2, 2, 2), (4, 2, 2, 4)]:
        U, rng = _fields(dims, kind=1)
        D = dirac.dense_dslash(U, dims)
        V = L.volume(dims)
        psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
        nx, ny, nz, nt = dims
        got = dirac.dslash(U, psi.reshape(nt, nz, ny, nx, 3), dims).reshape(-1)
        assert np.abs(got - D @ psi.reshape(-1)).max() < 1e-13
        # D is anti-Hermitian and only couples opposite parities
        assert np.abs(D + D.conj().T).max() < 1e-14
        par = np.repeat(L.parity(dims).reshape(-1), 3)
        assert np.abs(D[np.ix_(par == 0, par == 0)]).max() == 0
        assert np.abs(D[np.ix_(par == 1, par == 1)]).max() == 0


def test_anti_hermitian_blocks():
    """<a_o, D_oe b_e> = -<D_eo a_o, b_e>."""
    dims = (4, 4, 4, 4)
    U, rng = _fields(dims, kind=2)
    a = synth.gaussian_half_vector(dims, rng)
    b = synth.gaussian_half_vector(dims, rng)
    lhs = vdot(a, dirac.dslash_half(U, b, dims, 1))
    rhs = -vdot(dirac.dslash_half(U, a, dims, 0), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gauge_covariance_and_invariance():
    """D[U^Om](Om psi) = Om D[U] psi, hence <chi, A chi> is gauge invariant."""
    dims = (4, 4, 4, 4)
    U, rng = _fields(dims, kind=3)
    Om = synth.haar_su3(dims, rng)[..., 0, :, :]  # one SU(3) matrix per site
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    nx, ny, nz, nt = dims
    psi = rng.standard_normal((nt, nz, ny, nx, 3)) + 1j * rng.standard_normal((nt, nz, ny, nx, 3))
    lhs = dirac.dslash(Ug, np.einsum("...ij,...j->...i", Om, psi), dims)
    rhs = np.einsum("...ij,...j->...i", Om, dirac.dslash(U, psi, dims))
    assert np.abs(lhs - rhs).max() < 1e-13
    chi = synth.gaussian_half_vector(dims, rng)
    Om_e = L.full_to_half(Om, dims, 0)
    chig = np.einsum("kij,kj->ki", Om_e, chi)
    e0 = vdot(chi, dirac.apply_A(U, chi, dims, 0.1)).real
    e1 = vdot(chig, dirac.apply_A(Ug, chig, dims, 0.1)).real
    assert abs(e0 - e1) < 1e-13 * abs(e0)


def test_A_hermitian_positive_bounded():
    dims = (4, 4, 4, 4)
    U, rng = _fields(dims, eps=1.0, kind=4)
    m = 0.1
    a = synth.gaussian_half_vector(dims, rng)
    b = synth.gaussian_half_vector(dims, rng)
    ab = vdot(a, dirac.apply_A(U, b, dims, m))
    ba = vdot(b, dirac.apply_A(U, a, dims, m))
    assert abs(ab - ba.conjugate()) < 1e-12 * abs(ab)
    aa = vdot(a, dirac.apply_A(U, a, dims, m)).real
    nn = vdot(a, a).real
    assert 4 * m * m * nn <= aa <= (4 * m * m + 64) * nn
