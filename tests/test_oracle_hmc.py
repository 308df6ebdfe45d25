"""Pins for the oracle's RHMC pieces (paper Sec. 3.1): reversibility of the
leapfrog integrator, dH ~ dt^2, the heat bath, and the energy bookkeeping."""
import numpy as np

import synth
from oracle import fermion, hmc, philox

DIMS = (4, 4, 2, 4)


def _params(n_steps, tau=0.5):
    return hmc.HMCParams(beta=5.4, mass=0.1, tau=tau, n_steps=n_steps,
                         r_md=synth.load_rational("xm050_n8_m0.1"),
                         r_action=synth.load_rational("xm050_n8_m0.1"),
                         r_heatbath=synth.load_rational("xp025_n8_m0.1"),
                         tol_md=1e-12, tol_action=1e-12)


def _state(kind):
    rng = synth.make_rng(903, kind)
    U = synth.random_su3_near_identity(DIMS, 0.4, rng)
    P = synth.gaussian_momentum(DIMS, rng)
    xi = synth.gaussian_half_vector(DIMS, rng, scale=np.sqrt(0.5))
    return U, P, xi


def test_reversibility():
    U0, P0, xi = _state(0)
    prm = _params(5)
    phi = hmc.heatbath(U0, DIMS, prm.mass, xi, prm.r_heatbath, 1e-12)
    U1, P1 = hmc.leapfrog(U0, P0, DIMS, prm, phi)
    U2, P2 = hmc.leapfrog(U1, -P1, DIMS, prm, phi)
    assert np.abs(U2 - U0).max() < 1e-10
    assert np.abs(P2 + P0).max() < 1e-10


def test_dH_scales_as_dt_squared():
    U0, P0, xi = _state(1)
    dh = []
    for n in (8, 16, 32):
        out = hmc.trajectory(U0, DIMS, _params(n), P0, xi, 0.5)
        dh.append(abs(out["dH"]))
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    assert 3.2 < r1 < 4.5 and 3.7 < r2 < 4.3


def test_heatbath_inverts_action():
    """phi = r_{1/4}(A) xi gives phi^dag r_{-1/2}(A) phi = xi^dag xi up to the
    rational approximation errors (~1e-6 relative for these tables)."""
    U0, _, xi = _state(2)
    prm = _params(4)
    phi = hmc.heatbath(U0, DIMS, prm.mass, xi, prm.r_heatbath, 1e-13)
    Sf = fermion.fermion_action(U0, DIMS, prm.mass, phi, prm.r_action, 1e-13)
    xx = float(np.vdot(xi, xi).real)
    assert abs(Sf - xx) < 1e-5 * xx


def test_trajectory_accounting_and_philox_draws():
    U0, _, _ = _state(3)
    seed, traj = 12345, 7
    P0 = philox.momentum(DIMS, seed, traj)
    xi = philox.source(DIMS, seed, traj)
    u = philox.uniform(seed, traj)
    out = hmc.trajectory(U0, DIMS, _params(6), P0, xi, u)
    K0, Sg0, Sf0 = out["H0"]
    assert abs(K0 - 0.5 * np.sum(P0 ** 2)) < 1e-9
    assert abs(Sf0 - np.vdot(xi, xi).real) < 1e-5 * Sf0
    assert out["accepted"] == (u < np.exp(-out["dH"]))
    assert abs(out["dH"]) < 1.0


NAIK = (9.0 / 8.0, -1.0 / 24.0)


def _naik_params(n_steps, weights=NAIK):
    prm = _params(n_steps)
    prm.naik = weights
    return prm


def test_naik_dH_scales_as_dt_squared():
    """The improved operator's force is the derivative of its action: the
    leapfrog energy error then falls as dt^2 (a force inconsistent with the
    action leaves an O(1) dH)."""
    U0, P0, xi = _state(1)
    dh = []
    for n in (8, 16, 32):
        out = hmc.trajectory(U0, DIMS, _naik_params(n), P0, xi, 0.5)
        dh.append(abs(out["dH"]))
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    assert 3.2 < r1 < 4.5 and 3.7 < r2 < 4.3


def test_naik_heatbath_inverts_action():
    """phi = r_{1/4}(A) xi with the improved A: phi^dag r_{-1/2}(A) phi = xi^dag xi
    up to the tables' approximation errors (the improved spectrum on these
    near-identity links, free-field maximum 4m^2 + 16 (c1 - c3)^2 = 21.8,
    lies inside the tables' interval [0.01, 64])."""
    from oracle import naik
    U0, _, xi = _state(2)
    prm = _naik_params(4)
    phi = hmc.heatbath(U0, DIMS, prm.mass, xi, prm.r_heatbath, 1e-13, NAIK)
    Sf = naik.fermion_action(U0, DIMS, prm.mass, phi, prm.r_action, 1e-13, *NAIK)
    xx = float(np.vdot(xi, xi).real)
    assert abs(Sf - xx) < 1e-5 * xx


def test_naik_one_hop_weights_reproduce_the_plain_trajectory():
    """(c1, c3) = (1, 0) takes the improved code path (heat bath, force,
    actions) and must reproduce the one-hop trajectory."""
    U0, P0, xi = _state(4)
    a = hmc.trajectory(U0, DIMS, _params(4), P0, xi, 0.5)
    b = hmc.trajectory(U0, DIMS, _naik_params(4, (1.0, 0.0)), P0, xi, 0.5)
    assert abs(a["dH"] - b["dH"]) < 1e-9
    assert np.abs(a["U_proposed"] - b["U_proposed"]).max() < 1e-11
