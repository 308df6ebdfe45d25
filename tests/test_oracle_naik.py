"""Pins for the oracle's Naik-improved operator (Sec. 8 Summary: "improved"
quarks with a deeper stencil; reading: tree-level Naik term, c1 = 9/8,
c3 = -1/24, three-hop paths of dressed links)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import dirac, naik, lattice as L
from oracle.solvers import vdot


def _unit_links(dims):
    nx, ny, nz, nt = dims
    U = np.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def _fields(dims, eps=0.4, kind=0):
    rng = synth.make_rng(910, kind)
    return synth.random_su3_near_identity(dims, eps, rng), rng


def test_coefficients_remove_the_p3_error():
    """c1 sin p + c3 sin 3p = p - (3/40) p^5 + O(p^7): unit slope (c1 + 3 c3 = 1),
    no p^3 term (c1 + 27 c3 = 0) -- the pair is fixed by these two equations."""
    assert naik.C1 + 3 * naik.C3 == pytest.approx(1.0, abs=1e-15)
    assert naik.C1 + 27 * naik.C3 == pytest.approx(0.0, abs=1e-15)
    for p in (1e-2, 2e-2, 4e-2):
        f = naik.C1 * np.sin(p) + naik.C3 * np.sin(3 * p)
        assert (f - p) / p ** 5 == pytest.approx(-3.0 / 40.0, rel=2e-2)


@pytest.mark.parametrize("dims", [(8, 4, 6, 8), (6, 6, 4, 4)])
def test_free_field_plane_wave(dims):
    """At U = 1: (D psi)(x) = sum_mu eta_mu(x) 2i (c1 sin p_mu + c3 sin 3p_mu) psi(x)
    for psi = c e^{ip.x}, periodic spatial and antiperiodic temporal momenta
    (the three-hop across the time boundary picks up the boundary sign)."""
    nx, ny, nz, nt = dims
    U = _unit_links(dims)
    x, y, z, t = L.coords(dims)
    p = (2 * np.pi * 1 / nx, 2 * np.pi * 2 / ny, 2 * np.pi * 1 / nz, (2 * 1 + 1) * np.pi / nt)
    c = np.array([0.2 - 0.4j, 1.0, -0.3j])
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None] * c
    eta = [np.ones_like(x), (-1.0) ** x, (-1.0) ** (x + y), (-1.0) ** (x + y + z)]
    factor = sum(eta[mu] * 2j * (9 / 8 * np.sin(p[mu]) - 1 / 24 * np.sin(3 * p[mu])) for mu in range(4))
    got = naik.dslash(U, psi, dims)
    assert np.abs(got - factor[..., None] * psi).max() < 1e-13


def test_free_spectrum_matches_the_momentum_sum():
    """At U = 1 the full-lattice M^dag M = 4m^2 - D^2 has the eigenvalue
    4m^2 + 4 sum_mu (c1 sin p_mu + c3 sin 3p_mu)^2 on every plane wave (the
    eta phases make the directions anticommute, and a three-hop is an odd
    shift), 3 colours each.  The even block A holds half of each eigenvalue's
    multiplicity (D_oe maps its eigenspaces one-to-one onto the odd block's),
    and every multiplicity is even (p -> p + pi), so the sorted spectrum of A
    (dense, from the operator on 4^4) is every second value of the sorted
    momentum sum."""
    dims = (4, 4, 4, 4)
    m = 0.1
    U = _unit_links(dims)
    vh = L.volume(dims) // 2
    cols = []
    for k in range(3 * vh):
        e = np.zeros((vh, 3), dtype=np.complex128)
        e.reshape(-1)[k] = 1
        cols.append(naik.apply_A(U, e, dims, m).reshape(-1))
    ev = np.sort(np.linalg.eigvalsh(np.array(cols).T))
    ps = [2 * np.pi * np.arange(4) / 4] * 3 + [(2 * np.arange(4) + 1) * np.pi / 4]
    lam = []
    for q in itertools.product(*ps):
        lam.append(4 * m * m + 4 * sum((9 / 8 * np.sin(a) - 1 / 24 * np.sin(3 * a)) ** 2 for a in q))
    lam = np.sort(np.repeat(lam, 3))  # 3 colours: 3V values for the full lattice
    assert np.allclose(ev, lam[::2], atol=1e-12)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 4, 2, 4), (4, 2, 6, 2)])
def test_dense_bruteforce(dims):
    """The roll-based path operator equals the matrix built link by link;
    D is anti-Hermitian and only couples opposite parities."""
    U, rng = _fields(dims, kind=sum(dims))
    D = naik.dense_dslash(U, dims)
    V = L.volume(dims)
    psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    nx, ny, nz, nt = dims
    got = naik.dslash(U, psi.reshape(nt, nz, ny, nx, 3), dims).reshape(-1)
    assert np.abs(got - D @ psi.reshape(-1)).max() < 1e-13
    assert np.abs(D + D.conj().T).max() < 1e-14
    par = np.repeat(L.parity(dims).reshape(-1), 3)
    assert np.abs(D[np.ix_(par == 0, par == 0)]).max() == 0
    assert np.abs(D[np.ix_(par == 1, par == 1)]).max() == 0


def test_three_hop_term_alone_on_a_long_axis():
    """Only the three-hop term (c1 = 0, c3 = 1) on an 8-site x axis: a source
    at x = 0 reaches exactly x = 3, through the backward term
    -U(2)^dag U(1)^dag U(0)^dag, and x = 5, through the forward term
    U(5) U(6) U(7) (the path wraps to x = 8 = 0)."""
    dims = (8, 2, 2, 2)
    U, rng = _fields(dims, kind=5)
    nx, ny, nz, nt = dims
    psi = np.zeros((nt, nz, ny, nx, 3), dtype=np.complex128)
    v = np.array([1.0, 0.5j, -0.25])
    psi[0, 0, 0, 0] = v
    out = naik.dslash(U, psi, dims, c1=0.0, c3=1.0)
    u = U[0, 0, 0, :, 0]  # x-links along the axis through the origin (eta_0 = 1)
    # the output at x holds the path from x to the source
    exp3 = u[2].conj().T @ u[1].conj().T @ u[0].conj().T @ v  # from x=3: backward path to 0
    exp5 = u[5] @ u[6] @ u[7] @ v                             # from x=5: forward path to 8 = 0
    assert np.abs(out[0, 0, 0, 3] + exp3).max() < 1e-14
    assert np.abs(out[0, 0, 0, 5] - exp5).max() < 1e-14
    mask = np.ones(nx, bool)
    mask[[3, 5]] = False
    assert np.abs(out[0, 0, 0, mask]).max() == 0


def test_reduces_to_the_naive_operator():
    dims = (4, 4, 2, 6)
    U, rng = _fields(dims, kind=6)
    nx, ny, nz, nt = dims
    psi = rng.standard_normal((nt, nz, ny, nx, 3)) + 1j * rng.standard_normal((nt, nz, ny, nx, 3))
    assert np.abs(naik.dslash(U, psi, dims, c1=1.0, c3=0.0) - dirac.dslash(U, psi, dims)).max() < 1e-14


def test_gauge_covariance_and_invariance():
    """D[U^Om](Om psi) = Om D[U] psi; <chi, A chi> is gauge invariant."""
    dims = (4, 4, 6, 4)
    U, rng = _fields(dims, kind=7)
    Om = synth.haar_su3(dims, rng)[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    nx, ny, nz, nt = dims
    psi = rng.standard_normal((nt, nz, ny, nx, 3)) + 1j * rng.standard_normal((nt, nz, ny, nx, 3))
    lhs = naik.dslash(Ug, np.einsum("...ij,...j->...i", Om, psi), dims)
    rhs = np.einsum("...ij,...j->...i", Om, naik.dslash(U, psi, dims))
    assert np.abs(lhs - rhs).max() < 1e-13
    chi = synth.gaussian_half_vector(dims, rng)
    chig = np.einsum("kij,kj->ki", L.full_to_half(Om, dims, 0), chi)
    e0 = vdot(chi, naik.apply_A(U, chi, dims, 0.1)).real
    e1 = vdot(chig, naik.apply_A(Ug, chig, dims, 0.1)).real
    assert abs(e0 - e1) < 1e-13 * abs(e0)


def test_A_hermitian_positive_bounded():
    """<a,Ab> = conj<b,Aa>; 4m^2 |a|^2 <= <a,Aa> <= (4m^2 + (8(c1+|c3|))^2) |a|^2."""
    dims = (4, 4, 4, 4)
    U, rng = _fields(dims, eps=1.0, kind=8)
    m = 0.05
    a = synth.gaussian_half_vector(dims, rng)
    b = synth.gaussian_half_vector(dims, rng)
    ab = vdot(a, naik.apply_A(U, b, dims, m))
    ba = vdot(b, naik.apply_A(U, a, dims, m))
    assert abs(ab - ba.conjugate()) < 1e-12 * abs(ab)
    aa = vdot(a, naik.apply_A(U, a, dims, m)).real
    nn = vdot(a, a).real
    bound = 4 * m * m + (8 * (naik.C1 + abs(naik.C3))) ** 2
    assert 4 * m * m * nn <= aa <= bound * nn


# ---- the improved operator's pseudofermion force --------------------------

def _move(U, omega, h):
    from oracle.su3 import expi, to_matrix
    return np.einsum("...ij,...jk->...ik", expi(h * to_matrix(omega)), U)


@pytest.mark.parametrize("dims", [(4, 4, 2, 4), (6, 4, 4, 4)])
def test_naik_force_matches_finite_differences(dims):
    """F = -dS_f/dw for random directions w, against symmetric finite
    differences (O(h^2)) of the improved operator's rational action, including
    a lattice whose z extent 2 makes a three-link path run over one link twice."""
    rng = synth.make_rng(930, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(dims, rng)
    F = naik.fermion_force(U, dims, 0.1, phi, rat, 1e-13)
    for trial in range(2):
        om = rng.standard_normal(F.shape)
        h = 1e-4
        fd = (naik.fermion_action(_move(U, om, h), dims, 0.1, phi, rat, 1e-13)
              - naik.fermion_action(_move(U, om, -h), dims, 0.1, phi, rat, 1e-13)) / (2 * h)
        an = -np.sum(om * F)
        assert abs(fd - an) <= 1e-6 * abs(an), (dims, trial, fd, an)


def test_naik_force_naive_limit():
    """(c1, c3) = (1, 0) is the one-hop operator: the same force as the plain
    operator's oracle (an independent derivation and code path)."""
    from oracle import fermion
    dims = (4, 4, 2, 4)
    rng = synth.make_rng(931, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(dims, rng)
    F = naik.fermion_force(U, dims, 0.1, phi, rat, 1e-13, c1=1.0, c3=0.0)
    F0 = fermion.fermion_force(U, dims, 0.1, phi, rat, 1e-13)
    assert np.abs(F - F0).max() < 1e-10 * np.abs(F0).max()


def test_naik_force_is_gauge_covariant():
    """F(U^Omega, Omega phi) = Omega F Omega^dag (as traceless Hermitian matrices)."""
    from oracle.su3 import to_coords, to_matrix
    dims = (4, 4, 2, 4)
    rng = synth.make_rng(932, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(dims, rng)
    Om = synth.haar_su3(dims, rng)[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    phig = L.full_to_half(np.einsum("...ij,...j->...i", Om, L.half_to_full(phi, dims, 0)), dims, 0)
    F = to_matrix(naik.fermion_force(U, dims, 0.1, phi, rat, 1e-13))
    Fg = to_matrix(naik.fermion_force(Ug, dims, 0.1, phig, rat, 1e-13))
    rot = np.einsum("...ij,...mjk,...lk->...mil", Om, F, Om.conj())
    assert np.abs(Fg - rot).max() < 1e-9 * np.abs(F).max()
