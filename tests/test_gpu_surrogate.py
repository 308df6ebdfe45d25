"""Learned force model on the GPU (bf16 matrix-core kernels) against the
oracle's bf16-emulating reference: forces, loss, gradients; covariance;
training reduces the loss; trajectories use it only on non-exact kicks."""
import numpy as np
import pytest

import synth
from oracle import lattice as L, surrogate as S
from oracle.su3 import to_coords, to_matrix
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, lattice, log

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 2, 4)
KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")


def _params(seed):
    rng = synth.make_rng(700, seed)
    p = S.init_params(rng)
    p["W3"] = rng.standard_normal(p["W3"].shape) * 0.3
    p["b1"] = rng.standard_normal(S.HID) * 0.1
    p["b3"] = rng.standard_normal(S.N_OUT) * 0.1
    # the library keeps FP32 parameters: compare against the same values
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in p.items()}


def _flat(p):
    return stag.surrogate_params_to_flat(p)


def _unflat(g):
    out, o = {}, 0
    shapes = {"W1": (64, 16), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (8, 64), "b3": (8,)}
    for k in KEYS:
        n = int(np.prod(shapes[k]))
        out[k] = g[o:o + n].reshape(shapes[k])
        o += n
    return out


def _aux(dims, seed):
    nx, ny, nz, nt = dims
    return synth.make_rng(704, seed).standard_normal((nt, nz, ny, nx, 4, 8))


@pytest.mark.parametrize("with_aux", [False, True])
@pytest.mark.parametrize("dims", [DIMS, (6, 4, 4, 8)])
def test_force_matches_bf16_oracle(dims, with_aux):
    log(f"surrogate force dims={dims} aux={with_aux}")
    U = synth.random_su3_near_identity(dims, 0.6, synth.make_rng(701, 0))
    lat = lattice(dims, U)
    sur = stag.Surrogate(lat, 1)
    p = _params(1)
    sur.set_params(_flat(p))
    aux = _aux(dims, 0) if with_aux else None
    if with_aux:
        aux_dev = lat.mom_import(dev(aux))
        sur.set_aux(aux_dev)
    mom = lat.new_mom()
    sur.force(mom, 0.0)
    got = host(lat.mom_export(mom))
    exp = S.surrogate_force(p, U, dims, mode="bf16", aux=aux)
    scale = np.abs(exp).max()
    assert np.abs(got - exp).max() < 3e-3 * scale, np.abs(got - exp).max() / scale
    assert np.sqrt(np.mean((got - exp) ** 2)) < 2e-4 * scale


def test_loss_and_gradient_match_bf16_oracle():
    U = synth.random_su3_near_identity(DIMS, 0.6, synth.make_rng(701, 1))
    lat = lattice(DIMS, U)
    sur = stag.Surrogate(lat, 1)
    p = _params(2)
    sur.set_params(_flat(p))
    nx, ny, nz, nt = DIMS
    target = synth.make_rng(701, 2).standard_normal((nt, nz, ny, nx, 4, 8))
    aux = _aux(DIMS, 1)
    aux_dev = lat.mom_import(dev(aux))
    sur.set_aux(aux_dev)
    loss, g = sur.eval(lat.mom_import(dev(target)), want_grad=True)
    f, loops = S.features(U, DIMS, aux)
    tf = target.reshape(-1, 8).astype(np.float32).astype(np.float64)
    B = S.basis(loops, aux).astype(np.float32).astype(np.float64)   # the device keeps the channels in FP32
    lref, gref = S.loss_and_grad(p, f, B, tf, mode="bf16")
    assert abs(loss - lref) < 1e-4 * lref
    gg = _unflat(g.astype(np.float64))
    for k in KEYS:
        err = np.abs(gg[k] - gref[k]).max() / max(np.abs(gref[k]).max(), 1e-30)
        assert err < 2e-2, (k, err)


def test_force_is_gauge_covariant():
    U = synth.random_su3_near_identity(DIMS, 0.6, synth.make_rng(701, 3))
    rng = synth.make_rng(701, 4)
    Om = synth.haar_su3(DIMS, rng)[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    lat = lattice(DIMS, U)
    sur = stag.Surrogate(lat, 1)
    sur.set_params(_flat(_params(3)))
    m1 = lat.new_mom()
    sur.force(m1, 0.0)
    F = host(lat.mom_export(m1))
    lat.set_gauge(dev(Ug))
    m2 = lat.new_mom()
    sur.force(m2, 0.0)
    Fg = host(lat.mom_export(m2))
    rot = to_coords(np.einsum("...ij,...mjk,...lk->...mil", Om, to_matrix(F), Om.conj()))
    # invariant inputs are bf16-rounded on both sides: equal up to that rounding
    assert np.abs(rot - Fg).max() < 2e-2 * np.abs(F).max()


def test_training_learns_a_representable_force():
    """The Wilson gauge force is the model's basis with every channel weight
    equal to -beta/3: training on it must drive the loss far down."""
    dims = (6, 4, 4, 8)
    lat = stag.Lattice(dims)
    sur = stag.Surrogate(lat, 4, seed=5)
    rng = synth.make_rng(702, 0)
    beta = 1.5
    for k in range(4):
        lat.set_gauge(dev(synth.random_su3_near_identity(dims, 0.5, rng)))
        mom = lat.new_mom()
        lat.gauge_force(beta, mom, 0.0)
        sur.add_pair(mom)
    l0, _ = sur.eval(mom)
    sur.train(60, 1e-2)
    l1, _ = sur.eval(mom)
    log(f"  gauge-force loss before {l0:.4e} after {l1:.4e}")
    assert l1 < 0.05 * l0


def test_training_on_fermion_forces_lowers_the_loss():
    dims = (6, 4, 4, 8)
    rat = synth.load_rational("xm050_n8_m0.1")
    lat = stag.Lattice(dims)
    sur = stag.Surrogate(lat, 4, seed=5)
    rng = synth.make_rng(702, 1)
    for k in range(4):
        U = synth.random_su3_near_identity(dims, 0.5, rng)
        lat.set_gauge(dev(U))
        phi = lat.vec_import(dev(synth.gaussian_half_vector(dims, rng)), 0)
        mom = lat.new_mom()
        lat.fermion_force(0.1, rat, 1e-10, 100000, phi, mom, 0.0)
        sur.add_pair(mom)
    l0, _ = sur.eval(mom)
    sur.train(30, 3e-3)
    l1, _ = sur.eval(mom)
    log(f"  fermion-force loss before {l0:.4e} after {l1:.4e}")
    assert l1 < l0


def test_trajectory_with_model_is_exact_when_every_kick_is_exact():
    dims = (4, 4, 2, 4)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(703, 0))
    r_f = synth.load_rational("xm050_n8_m0.1")
    r_h = synth.load_rational("xp025_n8_m0.1")
    lat = lattice(dims, U0)
    sur = stag.Surrogate(lat, 1)
    sur.set_params(_flat(_params(4)))
    a = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, seed=3, traj_index=1)
    Ua = host(lat.get_gauge())
    lat.set_gauge(dev(U0))
    b = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, seed=3, traj_index=1, surrogate=sur, exact_every=1)
    assert a["dH"] == b["dH"] and np.array_equal(Ua, host(lat.get_gauge()))
    lat.set_gauge(dev(U0))
    c = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, seed=3, traj_index=1, surrogate=sur, exact_every=2)
    assert np.isfinite(c["dH"]) and c["dH"] != a["dH"]


def test_trajectory_schedules_and_pair_recording():
    dims = (4, 4, 2, 4)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(703, 1))
    r_f = synth.load_rational("xm050_n8_m0.1")
    r_h = synth.load_rational("xp025_n8_m0.1")
    lat = lattice(dims, U0)
    kw = dict(seed=4, traj_index=2)
    a = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, **kw)
    lat.set_gauge(dev(U0))
    # the two-time-scale ablation with one fine step per coarse step is plain leapfrog
    c = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=1, **kw)
    assert c["dH"] == a["dH"]
    lat.set_gauge(dev(U0))
    d = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, **kw)
    assert np.isfinite(d["dH"]) and d["dH"] != a["dH"]
    assert d["n_solves"] < a["n_solves"]
    with pytest.raises(stag.StagError):
        lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=3, **kw)
    # model on the inner scale with the outer-scale correction: a zero model is the ablation
    zero = stag.Surrogate(lat, 1)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    lat.set_gauge(dev(U0))
    z = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, surrogate=zero, **kw)
    assert z["dH"] == d["dH"]
    live = stag.Surrogate(lat, 1)
    live.set_params(_flat(_params(5)))
    lat.set_gauge(dev(U0))
    m = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, surrogate=live, **kw)
    assert np.isfinite(m["dH"]) and m["dH"] != d["dH"] and m["n_solves"] == d["n_solves"]
    # recording stores the exact forces of the kicks until the dataset is full
    sur = stag.Surrogate(lat, 3)
    lat.set_gauge(dev(U0))
    rec = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, surrogate=sur, record_pairs=True, **kw)
    assert sur.pairs == 3 and sur.capacity == 3
    assert abs(rec["dH"] - a["dH"]) < 1e-9 * max(1.0, abs(a["dH"]))
    with pytest.raises(stag.StagError):
        lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, surrogate=sur, record_pairs=True, exact_every=2, **kw)


def test_truncated_force_matches_oracle():
    """The pseudofermion force of a multi-shift solve stopped after N
    iterations (the model's auxiliary channel in trajectories) against the
    oracle's solver stopped after the same N iterations."""
    from oracle import fermion
    dims = (6, 4, 4, 8)
    rng = synth.make_rng(705, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n8_m0.1")
    lat = lattice(dims, U)
    mom = lat.new_mom()
    for n in (5, 20):
        info = lat.fermion_force(0.1, rat, 1e-30, n, lat.vec_import(dev(phi), 0), mom, 0.0,
                                 allow_not_converged=True)
        assert info["code"] == stag.STAG_ERR_NOT_CONVERGED and info["iters"] == n
        got = host(lat.mom_export(mom))
        sol = fermion.rational_solve(U, dims, 0.1, phi, rat, 1e-30, maxiter=n)
        assert sol["iters"] == n
        exp = fermion.force_from_solutions(U, dims, sol["x"], rat["residue"])
        assert np.abs(got - exp).max() < 1e-10 * np.abs(exp).max(), n


def test_trajectory_with_truncated_inner_force():
    """Schedules with the auxiliary channel: a model that is the truncated
    force alone (c_6 = 1) on the inner scale, exact force correcting on the
    outer scale; recording stores the truncated force with every pair."""
    dims = (4, 4, 2, 4)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(706, 0))
    r_f = synth.load_rational("xm050_n8_m0.1")
    r_h = synth.load_rational("xp025_n8_m0.1")
    lat = lattice(dims, U0)
    kw = dict(seed=5, traj_index=3)
    ident = stag.Surrogate(lat, 2)
    p = {k: np.zeros_like(v) for k, v in _params(0).items()}
    p["b3"][6] = 1.0
    ident.set_params(_flat(p))
    a = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, **kw)
    lat.set_gauge(dev(U0))
    b = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, surrogate=ident,
                       inner_iters=10, **kw)
    assert np.isfinite(b["dH"]) and b["dH"] != a["dH"]
    # 5 kicks, exact on 0, 2, 4; the model on every kick: 5 truncated solves
    assert b["n_solves"] == a["n_solves"] + 5
    lat.set_gauge(dev(U0))
    rec = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, surrogate=ident, record_pairs=True, inner_iters=10, **kw)
    assert ident.pairs == 2 and np.isfinite(rec["dH"])
    with pytest.raises(stag.StagError):
        lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, inner_iters=10, **kw)


def test_model_error_paths():
    lat = lattice(DIMS, synth.random_su3_near_identity(DIMS, 0.3, synth.make_rng(707, 0)))
    sur = stag.Surrogate(lat, 1)
    with pytest.raises(stag.StagError):
        sur.train(1, 1e-3)                      # no training pairs yet
    mom = lat.new_mom()
    sur.add_pair(mom)
    with pytest.raises(stag.StagError):
        sur.add_pair(mom)                       # dataset full
    with pytest.raises(stag.StagError):
        sur.set_aux(mom[1:])                    # misaligned device pointer
    with pytest.raises(stag.StagError):
        sur.train(1, -1.0)                      # learning rate must be positive
    with pytest.raises(ValueError):
        sur.set_params(np.zeros(3, dtype=np.float32))
    assert sur.train(1, 1e-3) >= 0.0
