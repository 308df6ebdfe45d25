"""GPU parity of the molecular-dynamics pieces (Sec. 3.1) against the oracle:
gauge and pseudofermion forces, link update, actions, kinetic energy, and the
Philox random fields."""
import numpy as np
import pytest

import synth
from oracle import fermion, gauge, hmc, philox
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, lattice, log, rel_err

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (6, 4, 2, 8), (8, 6, 4, 10)]


@pytest.mark.parametrize("dims", DIMS)
def test_gauge_force_and_action(dims):
    log(f"gauge force parity dims={dims}")
    rng = synth.make_rng(200, 0)
    U = synth.random_su3_near_identity(dims, 0.6, rng)
    lat = lattice(dims, U)
    mom = lat.new_mom()
    lat.gauge_force(5.4, mom, 0.0)
    got = host(lat.mom_export(mom))
    exp = gauge.gauge_force(U, dims, 5.4)
    assert rel_err(got, exp) < 1e-13
    # fused kick: mom += dt F
    P = synth.gaussian_momentum(dims, rng)
    m2 = lat.mom_import(dev(P))
    lat.gauge_force(5.4, m2, 0.05)
    assert rel_err(host(lat.mom_export(m2)), P + 0.05 * exp) < 1e-14
    S, plaq = lat.gauge_action(5.4)
    assert abs(S - gauge.gauge_action(U, dims, 5.4)) < 1e-11 * abs(S)
    assert abs(plaq - gauge.mean_plaquette(U, dims)) < 1e-14
    K = lat.kinetic_energy(lat.mom_import(dev(P)))
    assert abs(K - hmc.kinetic(P)) < 1e-12 * K


@pytest.mark.parametrize("dims", DIMS)
def test_fermion_force_and_action(dims):
    log(f"fermion force parity dims={dims}")
    rng = synth.make_rng(201, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(dims, rng)
    lat = lattice(dims, U)
    mom = lat.new_mom()
    lat.fermion_force(0.1, rat, 1e-12, 100000, lat.vec_import(dev(phi), 0), mom, 0.0)
    got = host(lat.mom_export(mom))
    exp = fermion.fermion_force(U, dims, 0.1, phi, rat, 1e-12)
    assert rel_err(got, exp) < 1e-9
    S = lat.fermion_action(0.1, rat, 1e-12, 100000, lat.vec_import(dev(phi), 0))
    assert abs(S - fermion.fermion_action(U, dims, 0.1, phi, rat, 1e-12)) < 1e-10 * abs(S)


@pytest.mark.parametrize("improved", [False, True])
def test_fermion_force_of_a_zero_field(improved):
    """phi = 0: the solve returns zeros without iterating, the force is exactly
    zero and a kick leaves the momenta unchanged (plain and improved operator)."""
    dims = (4, 4, 2, 4)
    rng = synth.make_rng(201, 7)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    lat = lattice(dims, U)
    if improved:
        lat.set_naik(9.0 / 8.0, -1.0 / 24.0)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = lat.vec_import(dev(np.zeros((dims[0] * dims[1] * dims[2] * dims[3] // 2, 3), np.complex128)), 0)
    mom = lat.new_mom()
    lat.fermion_force(0.1, rat, 1e-12, 100, phi, mom, 0.0)
    assert not np.any(host(lat.mom_export(mom)))
    P = synth.gaussian_momentum(dims, rng)
    m2 = lat.mom_import(dev(P))
    lat.fermion_force(0.1, rat, 1e-12, 100, phi, m2, 0.05)
    assert np.array_equal(host(lat.mom_export(m2)), P)


def test_gauge_force_and_link_update_full_size_16c8():
    """Gauge force, action, plaquette and one link update at 16^3x8 against
    the oracle, every link."""
    dims = (16, 16, 16, 8)
    log("gauge force and link update parity at 16^3x8")
    rng = synth.make_rng(200, 16)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    lat = lattice(dims, U)
    mom = lat.new_mom()
    lat.gauge_force(5.4, mom, 0.0)
    assert rel_err(host(lat.mom_export(mom)), gauge.gauge_force(U, dims, 5.4)) < 1e-13
    S, plaq = lat.gauge_action(5.4)
    assert abs(S - gauge.gauge_action(U, dims, 5.4)) < 1e-11 * abs(S)
    assert abs(plaq - gauge.mean_plaquette(U, dims)) < 1e-14
    P = synth.gaussian_momentum(dims, rng)
    lat.link_update(lat.mom_import(dev(P)), 0.05)
    assert np.abs(host(lat.get_gauge()) - hmc.link_update(U, P, 0.05)).max() < 1e-13


def test_fermion_force_full_size_16c8():
    """Every link's pseudofermion force at the RHMC workload's 16^3x8 (the
    launch configuration the trajectories use) against the oracle's."""
    dims = (16, 16, 16, 8)
    log("fermion force parity at 16^3x8")
    rng = synth.make_rng(201, 16)
    U = synth.random_su3_near_identity(dims, 0.3, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phi = synth.gaussian_half_vector(dims, rng)
    lat = lattice(dims, U)
    mom = lat.new_mom()
    lat.fermion_force(0.1, rat, 1e-12, 100000, lat.vec_import(dev(phi), 0), mom, 0.0)
    exp = fermion.fermion_force(U, dims, 0.1, phi, rat, 1e-12)
    assert rel_err(host(lat.mom_export(mom)), exp) < 1e-9


@pytest.mark.parametrize("dims", DIMS[:2])
def test_link_update(dims):
    log(f"link update parity dims={dims}")
    rng = synth.make_rng(202, 0)
    U = synth.random_su3_near_identity(dims, 0.7, rng)
    P = synth.gaussian_momentum(dims, rng)
    lat = lattice(dims, U)
    for dt in (0.05, 0.7):
        lat.set_gauge(dev(U))
        lat.link_update(lat.mom_import(dev(P)), dt)
        got = host(lat.get_gauge())
        exp = hmc.link_update(U, P, dt)
        assert np.abs(got - exp).max() < 1e-13
        assert np.abs(np.einsum("...ji,...jk->...ik", got.conj(), got) - np.eye(3)).max() < 1e-14


def test_philox_known_answers_and_fields():
    import json, os
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        out = host(stag.philox([int(c, 16) for c in v["ctr"]], [int(k, 16) for k in v["key"]], 1))
        assert [int(o) & 0xFFFFFFFF for o in out] == [int(e, 16) for e in v["out"]]
    # a run of counters matches the oracle bit for bit
    ctr = np.zeros((1000, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1000) + 5
    ctr[:, 1], ctr[:, 2], ctr[:, 3] = 7, 11, 13
    ref = philox.philox4x32_10(ctr, (17, 19))
    got = host(stag.philox([5, 7, 11, 13], [17, 19], 1000)).astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(got.reshape(1000, 4), ref.astype(np.int64))
    dims = (6, 4, 2, 8)
    lat = lattice(dims, synth.random_su3_near_identity(dims, 0.1, synth.make_rng(203, 0)))
    seed, traj = 0x1234567890AB, 42
    P = host(lat.mom_export(lat.random_momentum(seed, traj)))
    assert np.abs(P - philox.momentum(dims, seed, traj)).max() < 1e-13
    xi = host(lat.vec_export(lat.random_source(seed, traj), 0))
    assert np.abs(xi - philox.source(dims, seed, traj)).max() < 1e-13


def test_leapfrog_reversible_at_16c8():
    """A property that holds at any size, checked at the RHMC workload's
    16^3x8: leapfrog (gauge and fermion forces, link updates) run forward,
    momenta flipped, run again, returns to the starting links and the
    negated starting momenta."""
    dims = (16, 16, 16, 8)
    log("leapfrog reversibility at 16^3x8")
    rng = synth.make_rng(310, 0)
    U0 = synth.random_su3_near_identity(dims, 0.3, rng)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n12_m0.02")
    lat = lattice(dims, U0)
    phid = lat.vec_import(dev(phi), 0)
    mom = lat.random_momentum(9, 1)
    P0 = host(lat.mom_export(mom))
    dt, n = 0.05, 4

    def kick(h):
        lat.gauge_force(5.4, mom, h)
        lat.fermion_force(0.02, rat, 1e-12, 100000, phid, mom, h)

    def leapfrog():
        kick(0.5 * dt)
        for s in range(n):
            lat.link_update(mom, dt)
            kick(dt if s < n - 1 else 0.5 * dt)

    leapfrog()
    U1 = host(lat.get_gauge())
    assert np.abs(U1 - U0).max() > 1e-3        # the links did move
    flipped = lat.mom_import(dev(-host(lat.mom_export(mom))))
    mom.copy_(flipped)
    leapfrog()
    U2 = host(lat.get_gauge())
    P2 = host(lat.mom_export(mom))
    assert np.abs(U2 - U0).max() < 1e-9, np.abs(U2 - U0).max()
    assert np.abs(P2 + P0).max() < 1e-8 * np.abs(P0).max(), np.abs(P2 + P0).max()
