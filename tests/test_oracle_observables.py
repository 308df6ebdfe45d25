"""Pins for the oracle's observables.  Polyakov loop: unit links, a closed
form for constant diagonal time links, gauge invariance (which fails for the
reversed product) and the centre transformation (which tells tr P from its
conjugate).  Chiral condensate: the even-site reduction against the dense
full-lattice inverse, and the noise estimator against the exact trace."""
import numpy as np

import synth
from oracle import dirac, fermion, gauge, lattice as L, philox

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


def _dense_A(U, dims, mass):
    vh = L.volume(dims) // 2
    cols = []
    for j in range(3 * vh):
        e = np.zeros(3 * vh, dtype=complex)
        e[j] = 1.0
        cols.append(dirac.apply_A(U, e.reshape(vh, 3), dims, mass).reshape(-1))
    return np.array(cols).T


def test_condensate_reduction_to_the_even_sites():
    """(1/V) Tr (2m + D)^{-1} from the dense full-lattice matrix (built from
    the defining formula entry by entry) equals (4m/V) Tr_e A^{-1}."""
    dims, mass = (2, 2, 2, 4), 0.15
    U = synth.random_su3_near_identity(dims, 0.8, synth.make_rng(720, 0))
    V = L.volume(dims)
    M = 2 * mass * np.eye(3 * V) + dirac.dense_dslash(U, dims)
    full = np.trace(np.linalg.inv(M)).real / V
    even = 4 * mass * np.trace(np.linalg.inv(_dense_A(U, dims, mass))).real / V
    assert abs(full - even) < 1e-12 * abs(full)
    assert abs(np.trace(np.linalg.inv(M)).imag) < 1e-10


def test_condensate_estimator_converges_to_the_trace():
    dims, mass = (2, 2, 2, 2), 0.2
    U = synth.random_su3_near_identity(dims, 0.8, synth.make_rng(721, 0))
    exact = 4 * mass * np.trace(np.linalg.inv(_dense_A(U, dims, mass))).real / L.volume(dims)
    etas = [philox.noise(dims, 5, k) for k in range(400)]
    est, err = fermion.chiral_condensate(U, dims, mass, etas, 1e-13)
    assert 0 < err < 0.05 * abs(exact)
    assert abs(est - exact) < 4 * err


def test_estimator_noise_is_not_a_heat_bath_source():
    """The noise stream has its own field of the counter: with the chain's seed
    none of its vectors repeats the heat-bath source of any trajectory, and its
    moments are those of the source distribution."""
    dims = (4, 4, 2, 4)
    for k in range(4):
        eta = philox.noise(dims, 9, k)
        for traj in range(4):
            assert np.abs(eta - philox.source(dims, 9, traj)).max() > 0.1
    big = np.concatenate([philox.noise((8, 8, 8, 8), 3, k).ravel() for k in range(4)])
    assert abs(np.mean(np.abs(big) ** 2) - 1.0) < 0.02
    assert abs(np.mean(big)) < 0.02
