"""One RHMC trajectory on the GPU (Sec. 3.1: heat bath, leapfrog, Metropolis)
against the oracle trajectory with the same momenta, noise and uniform."""
import numpy as np
import pytest

import synth
from oracle import hmc, philox
from tests.gpu_util import dev, host, lattice, log

pytestmark = pytest.mark.gpu


def _params(n_steps, tau):
    return hmc.HMCParams(beta=5.4, mass=0.1, tau=tau, n_steps=n_steps,
                         r_md=synth.load_rational("xm050_n8_m0.1"),
                         r_action=synth.load_rational("xm050_n8_m0.1"),
                         r_heatbath=synth.load_rational("xp025_n8_m0.1"),
                         tol_md=1e-12, tol_action=1e-12)


@pytest.mark.parametrize("dims", [(4, 4, 2, 4), (6, 4, 4, 8)])
def test_trajectory_matches_oracle(dims):
    log(f"trajectory parity dims={dims}")
    rng = synth.make_rng(300, 0)
    U0 = synth.random_su3_near_identity(dims, 0.4, rng)
    seed, traj = 2024, 3
    prm = _params(6, 0.5)
    P0 = philox.momentum(dims, seed, traj)
    xi = philox.source(dims, seed, traj)
    u = philox.uniform(seed, traj)
    ref = hmc.trajectory(U0, dims, prm, P0, xi, u)
    lat = lattice(dims, U0)
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
    Ug = host(lat.get_gauge())
    assert np.abs(Ug - ref["U"]).max() < 1e-10
    assert abs(out["plaquette"] - ref["plaquette"]) < 1e-12


def test_accurate_action_tables_with_a_cheaper_md_set():
    """16-pole action and heat-bath tables (relative error ~2e-12) decide the
    Metropolis step while the 8-pole table (~2e-6) drives the molecular
    dynamics; the trajectory matches the oracle's with the same tables."""
    dims = (4, 4, 2, 4)
    log("trajectory with 16-pole action / heat bath and 8-pole MD tables")
    rng = synth.make_rng(300, 5)
    U0 = synth.random_su3_near_identity(dims, 0.4, rng)
    seed, traj = 2024, 7
    prm = hmc.HMCParams(beta=5.4, mass=0.1, tau=0.5, n_steps=6,
                        r_md=synth.load_rational("xm050_n8_m0.1"),
                        r_action=synth.load_rational("xm050_n16_m0.1"),
                        r_heatbath=synth.load_rational("xp025_n16_m0.1"),
                        tol_md=1e-12, tol_action=1e-12)
    P0 = philox.momentum(dims, seed, traj)
    xi = philox.source(dims, seed, traj)
    u = philox.uniform(seed, traj)
    ref = hmc.trajectory(U0, dims, prm, P0, xi, u)
    lat = lattice(dims, U0)
    out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                         tol_md=1e-12, tol_action=1e-12, seed=seed, traj_index=traj)
    K0, Sg0, Sf0 = ref["H0"]
    K1, Sg1, Sf1 = ref["H1"]
    for a, b in [(out["K_old"], K0), (out["Sg_old"], Sg0), (out["Sf_old"], Sf0),
                 (out["K_new"], K1), (out["Sg_new"], Sg1), (out["Sf_new"], Sf1)]:
        assert abs(a - b) <= 1e-10 * abs(b)
    assert abs(out["dH"] - ref["dH"]) < 1e-8
    assert out["accepted"] == int(ref["accepted"])
    assert np.abs(host(lat.get_gauge()) - ref["U"]).max() < 1e-10


def test_checkpoint_resume_is_bitwise(tmp_path):
    """A checkpoint is the canonical FP64 gauge field plus the (seed,
    trajectory index) of the counter-based random numbers: a fresh handle
    loaded from the file reproduces the next trajectory bit for bit."""
    dims = (4, 4, 2, 4)
    rng = synth.make_rng(300, 9)
    U0 = synth.random_su3_near_identity(dims, 0.4, rng)
    prm = _params(4, 0.5)
    args = (prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath)
    kw = dict(tol_md=1e-12, tol_action=1e-12, seed=77)
    lat = lattice(dims, U0)
    lat.trajectory(*args, traj_index=0, **kw)
    path = tmp_path / "ckpt.npz"
    np.savez(path, U=host(lat.get_gauge()), seed=77, next_traj=1)
    cont = lat.trajectory(*args, traj_index=1, **kw)
    U_cont = host(lat.get_gauge())
    ck = np.load(path)
    fresh = lattice(dims, ck["U"])
    res = fresh.trajectory(*args, traj_index=int(ck["next_traj"]), tol_md=1e-12, tol_action=1e-12,
                           seed=int(ck["seed"]))
    assert res["dH"] == cont["dH"] and res["accepted"] == cont["accepted"]
    assert np.array_equal(host(fresh.get_gauge()), U_cont)


def test_injected_fields_and_rejection_restores():
    dims = (4, 4, 2, 4)
    rng = synth.make_rng(301, 0)
    U0 = synth.random_su3_near_identity(dims, 0.4, rng)
    P0 = synth.gaussian_momentum(dims, rng)
    xi = synth.gaussian_half_vector(dims, rng, scale=np.sqrt(0.5))
    prm = _params(4, 0.5)
    ref = hmc.trajectory(U0, dims, prm, P0, xi, 0.999999)
    lat = lattice(dims, U0)
    out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                         tol_md=1e-12, tol_action=1e-12, inject_mom=lat.mom_import(dev(P0)),
                         inject_xi=lat.vec_import(dev(xi), 0), inject_u=0.999999)
    assert abs(out["dH"] - ref["dH"]) < 1e-8
    assert out["accepted"] == int(ref["accepted"])
    if not out["accepted"]:
        assert np.array_equal(host(lat.get_gauge()), U0)


def test_pure_gauge_trajectory():
    dims = (6, 4, 4, 8)
    rng = synth.make_rng(302, 0)
    U0 = synth.random_su3_near_identity(dims, 0.6, rng)
    seed, traj = 5, 0
    prm = _params(8, 1.0)
    P0 = philox.momentum(dims, seed, traj)
    ref = hmc.trajectory(U0, dims, prm, P0, None, philox.uniform(seed, traj), with_fermions=False)
    lat = lattice(dims, U0)
    out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                         seed=seed, traj_index=traj, no_fermions=True)
    assert abs(out["dH"] - ref["dH"]) < 1e-9
    assert np.abs(host(lat.get_gauge()) - ref["U"]).max() < 1e-11


@pytest.mark.parametrize("fmt", [2, 3])
def test_fp32_md_forces(fmt):
    """MD force solves with FP32 Krylov vectors (FP32-18 or FP16-12 links):
    the trajectory is deterministic (same dH twice) and its dH stays close
    to the oracle's FP64 trajectory with the same fields; the actions, and
    so the Metropolis test, are FP64 as before."""
    dims = (6, 4, 4, 8)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(300, 1))
    seed, traj = 77, 2
    prm = _params(6, 0.5)
    ref = hmc.trajectory(U0, dims, prm, philox.momentum(dims, seed, traj), philox.source(dims, seed, traj),
                         philox.uniform(seed, traj))
    lat = lattice(dims, U0)
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


def test_failed_solve_restores_the_links():
    """A momentum field with one NaN component passes the heat bath and the
    first kick, moves one link to NaN in the first link update, and the next
    force solve stops with NONFINITE: the handle's links are then those of the
    call, bit for bit, and the next trajectory runs normally."""
    from paper_1710_09178_amd import stag
    dims = (4, 4, 2, 4)
    log("trajectory error path restores the links")
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(300, 9))
    prm = _params(4, 0.5)
    lat = lattice(dims, U0)
    before = host(lat.get_gauge())
    P = philox.momentum(dims, 1, 0)
    P[1, 0, 1, 2, 3, 5] = np.nan
    bad = lat.mom_import(dev(P))
    with pytest.raises(stag.StagError) as ei:
        lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                       tol_md=1e-12, tol_action=1e-12, seed=1, traj_index=0, inject_mom=bad)
    assert ei.value.code == stag.STAG_ERR_NONFINITE
    assert np.array_equal(host(lat.get_gauge()), before)
    out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                         tol_md=1e-12, tol_action=1e-12, seed=1, traj_index=0)
    assert np.isfinite(out["dH"])


@pytest.mark.parametrize("improved", [False, True])
def test_mean_exp_minus_dH_is_one(improved):
    """Area preservation and reversibility of the leapfrog with the exact
    heat bath make <exp(-dH)> = 1 for every configuration: a 400-trajectory
    chain on 4^4 (tau 0.5, 10 steps, <|dH|> ~ 0.3) averages to 1 within four
    standard errors, with the one-hop and with the improved operator (whose
    force and action are then consistent at the level the statistic sees).
    The same chain's initial fermion actions average to 3 Vh, the mean of
    xi^dag xi for the heat bath's complex Gaussian noise."""
    from oracle import naik
    dims = (4, 4, 4, 4)
    log(f"<exp(-dH)> over a 400-trajectory chain, improved={improved}")
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(301, int(improved)))
    prm = _params(10, 0.5)
    lat = lattice(dims, U0)
    if improved:
        lat.set_naik(naik.C1, naik.C3)
    dH, Sf = [], []
    for t in range(400):
        out = lat.trajectory(prm.beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                             tol_md=1e-10, tol_action=1e-12, seed=77, traj_index=t)
        dH.append(out["dH"])
        Sf.append(out["Sf_old"])
    e = np.exp(-np.array(dH))
    mean, err = e.mean(), e.std() / np.sqrt(len(e) - 1)
    log(f"  <exp(-dH)> = {mean:.4f} +- {err:.4f}, <|dH|> = {np.mean(np.abs(dH)):.3f}")
    assert err < 0.05
    assert abs(mean - 1.0) < 4 * err
    # the heat bath: S_f at the start is xi^dag xi up to the tables' error,
    # whose mean is the number of complex components, 3 Vh
    vh3 = 3 * dims[0] * dims[1] * dims[2] * dims[3] // 2
    sm, se = np.mean(Sf), np.std(Sf) / np.sqrt(len(Sf) - 1)
    log(f"  <S_f> / (3 Vh) = {sm / vh3:.4f} +- {se / vh3:.4f}")
    assert abs(sm - vh3) < 4 * se


def test_pure_gauge_plaquette_at_strong_coupling():
    """Pure-gauge HMC at beta = 0.5 on 4^4 against the strong-coupling
    expansion of the Wilson action: the one-plaquette integral gives
    <Re tr P / 3> = beta/18 + beta^2/216 + O(beta^3) (the second-order term
    from <(Re tr U)^2> = 1/2 over SU(3)).  300 trajectories after 50 to
    equilibrate from a cold start; the chain mean (error from blocks of 25)
    within the larger of four standard errors and 1e-3 (a bound on the
    neglected higher orders at this beta)."""
    dims = (4, 4, 4, 4)
    beta = 0.5
    log("pure-gauge plaquette at beta 0.5")
    lat = lattice(dims, synth.random_su3_near_identity(dims, 0.0, synth.make_rng(303, 0)))
    prm = _params(10, 1.0)
    plaq = []
    for t in range(350):
        out = lat.trajectory(beta, prm.mass, prm.tau, prm.n_steps, prm.r_md, prm.r_action, prm.r_heatbath,
                             seed=9, traj_index=t, no_fermions=True)
        if t >= 50:
            plaq.append(out["plaquette"])
    blocks = np.array(plaq).reshape(12, 25).mean(axis=1)
    mean, err = blocks.mean(), blocks.std() / np.sqrt(len(blocks) - 1)
    expect = beta / 18 + beta ** 2 / 216
    log(f"  <P> = {mean:.5f} +- {err:.5f}, strong coupling {expect:.5f}")
    assert abs(mean - expect) < max(4 * err, 1e-3)
    assert err < 1e-3
