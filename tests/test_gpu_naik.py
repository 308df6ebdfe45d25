"""GPU parity of the Naik-improved operator (Sec. 8 Summary, improved quarks;
reading: c1 = 9/8 one-hop plus c3 = -1/24 three-hop paths) against the
oracle's path definition: D_oe / D_eo and A element by element over several
tiles, ragged tails, lattices on which the three-hop wraps onto itself, every
work split and both FP64 link formats; solves against the oracle's solver on
the improved A; the sloppy formats within their roundoff bounds."""
import numpy as np
import pytest

import synth
from oracle import dirac, hmc, naik, philox
from oracle import lattice as L
from oracle.solvers import multishift_cg, true_residuals
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, lattice, log, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 0.3),      # three hops forward = one hop backward, along a different path
    ((2, 2, 2, 2), 0.5),      # every three-hop path returns to the neighbour
    ((8, 6, 4, 10), 0.4),     # Vh = 960: several tiles and a ragged tail
    ((6, 2, 8, 4), 1.0),      # strongly disordered links
    ((16, 16, 16, 8), 0.2),   # z-slab tile map
]


def _naik_lattice(dims, U, fmt=stag.LINKS_F64_18):
    lat = lattice(dims, U)
    lat.set_link_format(fmt)
    lat.set_naik(naik.C1, naik.C3)
    return lat


@pytest.mark.parametrize("dims,eps", CASES)
@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("fmt", [stag.LINKS_F64_18, stag.LINKS_F64_12])
def test_naik_dslash_matches_oracle(dims, eps, tps, fmt):
    log(f"naik dslash parity dims={dims} eps={eps} tps={tps} fmt={fmt}")
    rng = synth.make_rng(920, hash(dims) % 1000)
    U = synth.random_su3_near_identity(dims, eps, rng)
    lat = _naik_lattice(dims, U, fmt)
    lat.tune(tps, 16)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash(y, lat.vec_import(dev(vin), 1 - out_par), out_par)
        got = host(lat.vec_export(y, out_par))
        exp = naik.dslash_half(U, vin, dims, out_par)
        assert rel_err(got, exp) < 2e-14, (out_par, rel_err(got, exp))


@pytest.mark.parametrize("dims,eps", CASES[:3])
def test_naik_mdagm_matches_oracle(dims, eps):
    log(f"naik A parity dims={dims}")
    rng = synth.make_rng(921, 0)
    U = synth.random_su3_near_identity(dims, eps, rng)
    lat = _naik_lattice(dims, U)
    vin = synth.gaussian_half_vector(dims, rng)
    y = lat.new_vec()
    lat.mdagm(y, lat.vec_import(dev(vin), 0), 0.1)
    assert rel_err(host(lat.vec_export(y, 0)), naik.apply_A(U, vin, dims, 0.1)) < 2e-14


@pytest.mark.parametrize("fmt", [stag.LINKS_F64_18, stag.LINKS_F64_12])
def test_naik_full_size_32c8(fmt):
    """32^3x8, eps = 0.2, the launch configuration the benchmark times: every
    output element of D_oe and D_eo."""
    dims = (32, 32, 32, 8)
    log(f"naik dslash parity at 32^3x8 fmt={fmt}")
    rng = synth.make_rng(922, fmt)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = _naik_lattice(dims, U, fmt)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash(y, lat.vec_import(dev(vin), 1 - out_par), out_par)
        got = host(lat.vec_export(y, out_par))
        assert rel_err(got, naik.dslash_half(U, vin, dims, out_par)) < 2e-14


def test_long_links_follow_the_gauge_field():
    """A new gauge field (set_gauge) and a link update both rebuild the long
    links before the next operator call."""
    dims = (8, 6, 4, 10)
    rng = synth.make_rng(923, 0)
    U1 = synth.random_su3_near_identity(dims, 0.4, rng)
    U2 = synth.random_su3_near_identity(dims, 0.4, rng)
    lat = _naik_lattice(dims, U1)
    vin = synth.gaussian_half_vector(dims, rng)
    x = lat.vec_import(dev(vin), 0)
    y = lat.new_vec()
    lat.dslash(y, x, 1)
    assert rel_err(host(lat.vec_export(y, 1)), naik.dslash_half(U1, vin, dims, 1)) < 2e-14
    lat.set_gauge(dev(U2))
    lat.dslash(y, x, 1)
    assert rel_err(host(lat.vec_export(y, 1)), naik.dslash_half(U2, vin, dims, 1)) < 2e-14
    mom = lat.random_momentum(5, 0)
    lat.link_update(mom, 0.05)
    U3 = host(lat.get_gauge())
    lat.dslash(y, x, 1)
    assert rel_err(host(lat.vec_export(y, 1)), naik.dslash_half(U3, vin, dims, 1)) < 2e-14


def test_naik_off_restores_the_one_hop_operator():
    dims = (8, 6, 4, 10)
    rng = synth.make_rng(924, 0)
    U = synth.random_su3_near_identity(dims, 0.4, rng)
    lat = _naik_lattice(dims, U)
    vin = synth.gaussian_half_vector(dims, rng)
    x = lat.vec_import(dev(vin), 0)
    y = lat.new_vec()
    lat.set_naik(1.0, 0.0)
    lat.dslash(y, x, 1)
    plain = lattice(dims, U)
    y2 = plain.new_vec()
    plain.dslash(y2, plain.vec_import(dev(vin), 0), 1)
    assert np.array_equal(host(y), host(y2))
    # other weights: the operator is linear in (c1, c3)
    lat.set_naik(0.0, 1.0)
    lat.dslash(y, x, 1)
    exp = naik.dslash_half(U, vin, dims, 1, c1=0.0, c3=1.0)
    assert rel_err(host(lat.vec_export(y, 1)), exp) < 2e-14


FORCE_CASES = [
    ((4, 4, 2, 4), 0.5, stag.LINKS_F64_18),
    ((2, 2, 2, 2), 0.5, stag.LINKS_F64_18),    # a three-link path runs over one link twice
    ((4, 4, 4, 4), 0.4, stag.LINKS_F64_12),    # forward and backward three-link paths share links
    ((8, 6, 4, 10), 0.4, stag.LINKS_F64_18),   # several tiles and a ragged tail
]


@pytest.mark.parametrize("dims,eps,fmt", FORCE_CASES)
def test_naik_force_and_action_match_oracle(dims, eps, fmt):
    """Pseudofermion force and action of the improved operator against the
    oracle's (whose force is pinned by finite differences of its action):
    mom = F and the kick mom += dt F."""
    log(f"naik force parity dims={dims} fmt={fmt}")
    rng = synth.make_rng(925, hash(dims) % 1000)
    U = synth.random_su3_near_identity(dims, eps, rng)
    lat = _naik_lattice(dims, U, fmt)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    phid = lat.vec_import(dev(phi), 0)
    mom = lat.new_mom()
    lat.fermion_force(0.1, rat, 1e-12, 100000, phid, mom, 0.0)
    exp = naik.fermion_force(U, dims, 0.1, phi, rat, 1e-12)
    assert rel_err(host(lat.mom_export(mom)), exp) < 1e-9
    P = synth.gaussian_momentum(dims, rng)
    m2 = lat.mom_import(dev(P))
    lat.fermion_force(0.1, rat, 1e-12, 100000, phid, m2, 0.05)
    assert rel_err(host(lat.mom_export(m2)), P + 0.05 * exp) < 1e-9
    S = lat.fermion_action(0.1, rat, 1e-12, 100000, phid)
    assert abs(S - naik.fermion_action(U, dims, 0.1, phi, rat, 1e-12)) < 1e-10 * abs(S)


def test_naik_force_full_size_16c8():
    """Every link's improved-operator force at the RHMC workload's 16^3x8
    against the oracle's (the oracle's solve and force take ~30 s)."""
    dims = (16, 16, 16, 8)
    log("naik force parity at 16^3x8")
    rng = synth.make_rng(925, 16)
    U = synth.random_su3_near_identity(dims, 0.3, rng)
    lat = _naik_lattice(dims, U)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    mom = lat.new_mom()
    lat.fermion_force(0.1, rat, 1e-12, 100000, lat.vec_import(dev(phi), 0), mom, 0.0)
    exp = naik.fermion_force(U, dims, 0.1, phi, rat, 1e-12)
    assert rel_err(host(lat.mom_export(mom)), exp) < 1e-9


def test_naik_trajectory_matches_oracle():
    """One trajectory with the improved operator in heat bath, force and
    actions against the oracle trajectory with the same momenta, noise and
    uniform."""
    dims = (4, 4, 2, 4)
    log("naik trajectory parity 4x4x2x4")
    rng = synth.make_rng(927, 0)
    U0 = synth.random_su3_near_identity(dims, 0.4, rng)
    seed, traj = 2024, 5
    prm = hmc.HMCParams(beta=5.4, mass=0.1, tau=0.5, n_steps=6,
                        r_md=synth.load_rational("xm050_n8_m0.1"),
                        r_action=synth.load_rational("xm050_n8_m0.1"),
                        r_heatbath=synth.load_rational("xp025_n8_m0.1"),
                        tol_md=1e-12, tol_action=1e-12, naik=(naik.C1, naik.C3))
    P0 = philox.momentum(dims, seed, traj)
    xi = philox.source(dims, seed, traj)
    u = philox.uniform(seed, traj)
    ref = hmc.trajectory(U0, dims, prm, P0, xi, u)
    lat = _naik_lattice(dims, U0)
    out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                         tol_md=1e-12, tol_action=1e-12, seed=seed, traj_index=traj)
    log(f"  dH gpu {out['dH']:.12e} oracle {ref['dH']:.12e}")
    K0, Sg0, Sf0 = ref["H0"]
    K1, Sg1, Sf1 = ref["H1"]
    for a, b in [(out["K_old"], K0), (out["Sg_old"], Sg0), (out["Sf_old"], Sf0),
                 (out["K_new"], K1), (out["Sg_new"], Sg1), (out["Sf_new"], Sf1)]:
        assert abs(a - b) <= 1e-10 * abs(b)
    assert abs(out["dH"] - ref["dH"]) < 1e-8
    assert out["accepted"] == int(ref["accepted"])
    assert np.abs(host(lat.get_gauge()) - ref["U"]).max() < 1e-10


@pytest.mark.parametrize("fmt", [2, 3])
def test_naik_fp32_md_forces(fmt):
    """Improved-operator trajectories with the MD force solves in FP32 Krylov
    vectors (FP32-18 or FP16-12 long and one-hop links): deterministic, FP64
    actions, dH close to the oracle's FP64 trajectory with the same fields."""
    dims = (4, 4, 2, 4)
    log(f"naik trajectory, MD solves in link format {fmt}")
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(927, 1))
    seed, traj = 78, 3
    prm = hmc.HMCParams(beta=5.4, mass=0.1, tau=0.5, n_steps=6,
                        r_md=synth.load_rational("xm050_n8_m0.1"),
                        r_action=synth.load_rational("xm050_n8_m0.1"),
                        r_heatbath=synth.load_rational("xp025_n8_m0.1"),
                        tol_md=1e-12, tol_action=1e-12, naik=(naik.C1, naik.C3))
    ref = hmc.trajectory(U0, dims, prm, philox.momentum(dims, seed, traj), philox.source(dims, seed, traj),
                         philox.uniform(seed, traj))
    lat = _naik_lattice(dims, U0)
    outs = []
    for _ in range(2):
        lat.set_gauge(dev(U0))
        outs.append(lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action,
                                   prm.r_heatbath, tol_md=1e-8, tol_action=1e-12, seed=seed, traj_index=traj,
                                   md_link_format=fmt))
    assert outs[0]["dH"] == outs[1]["dH"]
    log(f"  fmt {fmt}: dH {outs[0]['dH']:.6e} oracle FP64 {ref['dH']:.6e}")
    assert abs(outs[0]["Sf_old"] - ref["H0"][2]) <= 1e-10 * abs(ref["H0"][2])
    tol = 1e-4 if fmt == 2 else 5e-2
    assert abs(outs[0]["dH"] - ref["dH"]) < tol * max(1.0, abs(ref["dH"]))


def test_naik_leapfrog_reversible_at_16c8():
    """At the RHMC workload's 16^3x8, a property that holds at any size:
    leapfrog with the improved operator's force, run forward, momenta
    flipped, run again, returns to the starting links and negated momenta."""
    dims = (16, 16, 16, 8)
    log("naik leapfrog reversibility at 16^3x8")
    rng = synth.make_rng(928, 0)
    U0 = synth.random_su3_near_identity(dims, 0.3, rng)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n12_m0.02")
    lat = _naik_lattice(dims, U0)
    phid = lat.vec_import(dev(phi), 0)
    mom = lat.random_momentum(9, 2)
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
    assert np.abs(U1 - U0).max() > 1e-3
    mom.copy_(lat.mom_import(dev(-host(lat.mom_export(mom)))))
    leapfrog()
    dU = np.abs(host(lat.get_gauge()) - U0).max()
    dP = np.abs(host(lat.mom_export(mom)) + P0).max()
    log(f"  |dU| {dU:.2e} |dP| {dP:.2e}")
    assert dU < 1e-9
    assert dP < 1e-8 * np.abs(P0).max()


def test_naik_multishift_matches_oracle():
    """8 poles, ragged lattice: every solution within 2 tol kappa_k of the
    oracle's solve of the improved A, true residuals (oracle operator) below tol."""
    dims = (8, 6, 4, 10)
    mass, tol = 0.1, 1e-10
    log("naik multi-shift solve 8x6x4x10")
    rng = synth.make_rng(926, 0)
    U = synth.random_su3_near_identity(dims, 0.4, rng)
    b = synth.gaussian_half_vector(dims, rng)
    poles = list(np.logspace(-4, 0, 8))
    lat = _naik_lattice(dims, U)
    xs = [lat.new_vec() for _ in poles]
    info = lat.multishift_solve(mass, {"c0": 0.0, "pole": poles, "residue": [1.0] * 8}, tol, 10000,
                                lat.vec_import(dev(b), 0), xs)
    A = lambda v: naik.apply_A(U, v, dims, mass)  # noqa: E731
    ref = multishift_cg(A, b, poles, tol)
    got = [host(lat.vec_export(x, 0)) for x in xs]
    res = true_residuals(A, b, poles, got)
    assert max(res) < tol, res
    lam_max = 4 * mass * mass + (8 * (naik.C1 - naik.C3)) ** 2
    for g, xr, s in zip(got, ref["x"], poles):
        kappa = (lam_max + s) / (4 * mass * mass + s)
        assert np.linalg.norm(g - xr) <= 2 * tol * kappa * np.linalg.norm(xr)
    log(f"  {info['iters']} iterations (oracle {ref['iters']}), max true residual {max(res):.2e}")


def test_naik_solve_32c8():
    """The 12-pole x^(-1/4) solve of the 32^3x8 workload with the improved
    operator: every pole's true residual, computed with the oracle's operator
    on the GPU solutions, below 1e-10."""
    dims = (32, 32, 32, 8)
    mass, tol = 0.005, 1e-10
    log("naik 12-pole solve at 32^3x8")
    rng = synth.make_rng(927, 0)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    b = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm025_n12_m0.005")
    lat = _naik_lattice(dims, U)
    xs = [lat.new_vec() for _ in rat["pole"]]
    info = lat.multishift_solve(mass, rat, tol, 100000, lat.vec_import(dev(b), 0), xs)
    got = [host(lat.vec_export(x, 0)) for x in xs]
    res = true_residuals(lambda v: naik.apply_A(U, v, dims, mass), b, rat["pole"], got)
    log(f"  {info['iters']} iterations, true residuals (oracle operator) max {max(res):.2e}, "
        f"GPU's own max {max(info['true_resid']):.2e}")
    assert max(res) < tol


def test_naik_mixed_solve_reaches_fp64_residual():
    dims = (8, 6, 4, 10)
    mass, tol = 0.05, 1e-10
    rng = synth.make_rng(928, 0)
    U = synth.random_su3_near_identity(dims, 0.4, rng)
    b = synth.gaussian_half_vector(dims, rng)
    poles = list(np.logspace(-4, 0, 8))
    lat = _naik_lattice(dims, U)
    xs = [lat.new_vec() for _ in poles]
    lat.multishift_solve_mixed(mass, {"c0": 0.0, "pole": poles, "residue": [1.0] * 8}, tol, 100000,
                               lat.vec_import(dev(b), 0), xs, sloppy=stag.LINKS_F32_18)
    got = [host(lat.vec_export(x, 0)) for x in xs]
    res = true_residuals(lambda v: naik.apply_A(U, v, dims, mass), b, poles, got)
    assert max(res) < tol, res


# ---- sloppy formats: roundoff bounds as for the one-hop operator, with the
# weighted neighbour sums c1 P1(x) + |c3| P3(x) and up to 96 + 4 rounded
# products per output real part
U32, U16 = 2.0 ** -24, 2.0 ** -11
BOUND_COEF = {stag.LINKS_F32_18: 100 * U32, stag.LINKS_F16_12: 2.1 * U16 * np.sqrt(2) + 100 * U32}


def _shift3(a, mu, d):
    for _ in range(3):
        a = L.fwd(a, mu) if d > 0 else L.bwd(a, mu)
    return a


def _weighted_neighbour_sum(v_half, dims, in_par):
    s = np.abs(v_half.real).sum(-1) + np.abs(v_half.imag).sum(-1)
    full = L.half_to_full(s[:, None], dims, in_par)[..., 0]
    p1 = sum(L.fwd(full, mu) + L.bwd(full, mu) for mu in range(4))
    p3 = sum(_shift3(full, mu, 1) + _shift3(full, mu, -1) for mu in range(4))
    tot = naik.C1 * p1 + abs(naik.C3) * p3
    return L.full_to_half(tot[..., None], dims, 1 - in_par)[:, 0]


@pytest.mark.parametrize("sloppy", [stag.LINKS_F32_18, stag.LINKS_F16_12])
def test_naik_sloppy_dslash_32c8(sloppy):
    dims = (32, 32, 32, 8)
    log(f"naik sloppy Dslash at 32^3x8 format={sloppy}")
    rng = synth.make_rng(929, sloppy)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = _naik_lattice(dims, U)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash_sloppy(y, lat.vec_import(dev(vin), 1 - out_par), out_par, sloppy)
        got = host(lat.vec_export(y, out_par))
        exp = naik.dslash_half(U, vin, dims, out_par)
        P = _weighted_neighbour_sum(vin, dims, 1 - out_par)[:, None]
        err = np.maximum(np.abs(got.real - exp.real), np.abs(got.imag - exp.imag))
        ratio = err / (BOUND_COEF[sloppy] * P)
        log(f"  out parity {out_par}: relative (max norm) {rel_err(got, exp):.3e}, max err / bound {ratio.max():.3f}")
        assert ratio.max() <= 1.0
