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
    # Without the auxiliary channel the inputs are functions of U alone, while
    # the force depends on the pseudofermion field drawn with it: the model
    # can only learn the part common to the four pairs, so the bar is a
    # decrease, not a factor.
    assert l1 < l0


def test_training_with_the_truncated_force_channel():
    """With the auxiliary channel set to the force of a solve stopped after 20
    iterations (13% off the exact force on these fields, measured with the
    oracle), c_6 = 1 alone already leaves (0.13)^2 = 1.8% of the loss of a
    zero model: training on the exact forces must get below 10% of it."""
    dims = (6, 4, 4, 8)
    rat = synth.load_rational("xm050_n8_m0.1")
    lat = stag.Lattice(dims)
    sur = stag.Surrogate(lat, 4, seed=5)
    rng = synth.make_rng(702, 1)
    keep = []
    for k in range(4):
        U = synth.random_su3_near_identity(dims, 0.5, rng)
        lat.set_gauge(dev(U))
        phi = lat.vec_import(dev(synth.gaussian_half_vector(dims, rng)), 0)
        mom, aux = lat.new_mom(), lat.new_mom()
        lat.fermion_force(0.1, rat, 1e-10, 100000, phi, mom, 0.0)
        lat.fermion_force(0.1, rat, 1e-30, 20, phi, aux, 0.0, allow_not_converged=True)
        sur.set_aux(aux)
        sur.add_pair(mom)
        keep.append(aux)
    zero = stag.Surrogate(lat, 1)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    l_zero, _ = zero.eval(mom)
    sur.train(60, 1e-2)
    l1, _ = sur.eval(mom)
    log(f"  loss of a zero model {l_zero:.4e}, trained with the channel {l1:.4e}")
    assert l1 < 0.1 * l_zero


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
    # judging the model at the exact kicks reuses their solves
    lat.set_gauge(dev(U0))
    j = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, coarse_force=True, exact_every=2, surrogate=ident,
                       inner_iters=10, judge_model=True, **kw)
    assert j["n_solves"] == b["n_solves"] and j["cg_iters_total"] == b["cg_iters_total"]
    assert abs(j["dH"] - b["dH"]) < 1e-9 * max(1.0, abs(b["dH"])) and 0.0 < j["model_force_err"] < np.inf
    lat.set_gauge(dev(U0))
    rec = lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, surrogate=ident, record_pairs=True, inner_iters=10, **kw)
    assert ident.pairs == 2 and np.isfinite(rec["dH"])
    with pytest.raises(stag.StagError):
        lat.trajectory(5.4, 0.1, 0.5, 4, r_f, r_f, r_h, inner_iters=10, **kw)


def test_judged_trajectory_reports_the_model_force_error():
    """judge_model: at the exact kick of a one-step trajectory (kick 0 on the
    starting links; kick 1 is the model's) the reported error is
    |F_model - F| / |F| of the model's and the exact force on those links,
    recomputed here from the same injected source; a zero model gives 1."""
    dims = (4, 4, 2, 4)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(708, 0))
    r_f = synth.load_rational("xm050_n8_m0.1")
    r_h = synth.load_rational("xp025_n8_m0.1")
    lat = lattice(dims, U0)
    sur = stag.Surrogate(lat, 1)
    sur.set_params(_flat(_params(6)))
    xi, mom0 = lat.random_source(11, 0), lat.random_momentum(11, 0)
    kw = dict(seed=3, traj_index=1, inject_mom=mom0, inject_xi=xi, inject_u=0.0, exact_every=2)
    t = lat.trajectory(5.4, 0.1, 0.5, 1, r_f, r_f, r_h, surrogate=sur, judge_model=True, **kw)
    assert t["used_model"] == 1
    lat.set_gauge(dev(U0))
    phi = lat.new_vec()
    lat.multishift_solve(0.1, r_h, 1e-10, 100000, xi, sum_out=phi)
    F, Fm = lat.new_mom(), lat.new_mom()
    lat.fermion_force(0.1, r_f, 1e-10, 100000, phi, F, 0.0)
    sur.force(Fm)
    f, fm = host(F), host(Fm)
    exp = np.sqrt(((fm - f) ** 2).sum() / (f ** 2).sum())
    log(f"  judged model force error {t['model_force_err']:.6e} (host {exp:.6e})")
    assert 0.0 < exp and abs(t["model_force_err"] - exp) < 1e-9 * exp
    # without the judge the trajectory is the same update up to the kick's rounding
    lat.set_gauge(dev(U0))
    u = lat.trajectory(5.4, 0.1, 0.5, 1, r_f, r_f, r_h, surrogate=sur, **kw)
    assert u["model_force_err"] == -1.0 and abs(u["dH"] - t["dH"]) < 1e-9 * max(1.0, abs(t["dH"]))
    zero = stag.Surrogate(lat, 1)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    lat.set_gauge(dev(U0))
    z = lat.trajectory(5.4, 0.1, 0.5, 2, r_f, r_f, r_h, surrogate=zero, judge_model=True, **kw)
    assert z["model_force_err"] == 1.0
    lat.set_gauge(dev(U0))
    e = lat.trajectory(5.4, 0.1, 0.5, 1, r_f, r_f, r_h, judge_model=True, **kw)
    assert e["used_model"] == 0 and e["model_force_err"] == -1.0


def _chain_reference(lat, U0, pattern, args, kw, sur):
    """The chain's trajectories replayed one by one with the given schedule."""
    lat.set_gauge(dev(U0))
    out = []
    for t, use in enumerate(pattern):
        extra = dict(surrogate=sur, exact_every=2, judge_model=True) if use else {}
        out.append(lat.trajectory(*args, seed=kw["seed"], traj_index=kw["traj_index"] + t, **extra))
    return out, host(lat.get_gauge())


def test_chain_falls_back_to_the_exact_force():
    """stag_md_chain: a model whose judged error exceeds the bound hands the
    next exact_trajectories trajectories to the exact force; a model whose
    trajectories are all rejected does so once the acceptance window fills;
    every trajectory equals the one-by-one call with the same schedule."""
    dims = (4, 4, 2, 4)
    U0 = synth.random_su3_near_identity(dims, 0.4, synth.make_rng(708, 1))
    r_f = synth.load_rational("xm050_n8_m0.1")
    r_h = synth.load_rational("xp025_n8_m0.1")
    lat = lattice(dims, U0)
    args = (5.4, 0.1, 0.5, 4, r_f, r_f, r_h)
    kw = dict(seed=7, traj_index=20)
    zero = stag.Surrogate(lat, 1)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    # the zero model's judged error is 1 > 0.5: model, exact, exact, model, ...
    got = lat.chain(7, *args, surrogate=zero, exact_every=2, max_model_err=0.5, min_acceptance=0.0,
                    exact_trajectories=2, **kw)
    Ug = host(lat.get_gauge())
    assert [g["used_model"] for g in got] == [1, 0, 0, 1, 0, 0, 1]
    assert all((g["model_force_err"] == 1.0) == bool(g["used_model"]) for g in got)
    ref, Ur = _chain_reference(lat, U0, [1, 0, 0, 1, 0, 0, 1], args, kw, zero)
    assert [g["dH"] for g in got] == [r["dH"] for r in ref]
    assert [g["accepted"] for g in got] == [r["accepted"] for r in ref]
    assert np.array_equal(Ug, Ur)
    # a wild model (large constant force): rejected, window 2 of acceptance 0
    wild = stag.Surrogate(lat, 1)
    p = {k: np.zeros_like(v) for k, v in _params(0).items()}
    p["b3"][:6] = 40.0
    wild.set_params(_flat(p))
    lat.set_gauge(dev(U0))
    got = lat.chain(7, *args, surrogate=wild, exact_every=2, max_model_err=1e30, min_acceptance=0.5, window=2,
                    exact_trajectories=2, **kw)
    assert [g["used_model"] for g in got] == [1, 1, 0, 0, 1, 1, 0]
    assert all(g["accepted"] == 0 for g in got if g["used_model"])
    # no model: plain RHMC, trajectory indices counting up
    lat.set_gauge(dev(U0))
    plain = lat.chain(3, *args, **kw)
    ref, _ = _chain_reference(lat, U0, [0, 0, 0], args, kw, None)
    assert [g["dH"] for g in plain] == [r["dH"] for r in ref] and not any(g["used_model"] for g in plain)
    # without a model the chain keeps the given schedule (here the two-time-scale ablation)
    lat.set_gauge(dev(U0))
    abl = lat.chain(2, *args, coarse_force=True, exact_every=2, **kw)
    lat.set_gauge(dev(U0))
    ref = [lat.trajectory(*args, seed=kw["seed"], traj_index=kw["traj_index"] + t, coarse_force=True,
                          exact_every=2) for t in range(2)]
    assert [g["dH"] for g in abl] == [r["dH"] for r in ref] and abl[0]["dH"] != plain[0]["dH"]
    with pytest.raises(stag.StagError):
        lat.chain(2, *args, surrogate=zero, window=0, **kw)
    with pytest.raises(stag.StagError):
        lat.chain(2, *args, surrogate=zero, max_model_err=0.0, **kw)


def test_model_error_paths():
    lat = lattice(DIMS, synth.random_su3_near_identity(DIMS, 0.3, synth.make_rng(707, 0)))
    sur = stag.Surrogate(lat, 1)
    with pytest.raises(stag.StagError):
        sur.train(1, 1e-3)                      # no training pairs yet
    mom = lat.new_mom()
    sur.add_pair(mom)
    with pytest.raises(stag.StagError):
        sur.add_pair(mom)                       # dataset full
    with pytest.raises(ValueError):
        sur.set_aux(mom[1:])                    # wrong size: refused by the binding
    import ctypes                               # misaligned device pointer: refused by the library
    assert sur.lib.stag_surrogate_set_aux(sur.h, ctypes.c_void_p(mom.data_ptr() + 8)) == stag.STAG_ERR_INVALID_ARG
    with pytest.raises(stag.StagError):
        sur.train(1, -1.0)                      # learning rate must be positive
    with pytest.raises(ValueError):
        sur.set_params(np.zeros(3, dtype=np.float32))
    assert sur.train(1, 1e-3) >= 0.0


# ---- the learned model at the size of the 16^3x8 RHMC workload -------------
# 131,072 links: every wave of the training and inference kernels walks 8
# tiles of 16 links, accumulating across tiles and reusing its LDS, which the
# small lattices above (at most one tile per wave) never do.

C4 = (16, 16, 16, 8)
U_BF16 = 2.0 ** -8          # unit roundoff of bfloat16 (8 significant bits)


def _c4_setup(with_aux, seed=0):
    U = synth.random_su3_near_identity(C4, 0.6, synth.make_rng(708, seed))
    nx, ny, nz, nt = C4
    rng = synth.make_rng(708, 100 + seed)
    target = rng.standard_normal((nt, nz, ny, nx, 4, 8))
    aux = rng.standard_normal((nt, nz, ny, nx, 4, 8)) if with_aux else None
    return U, target, aux


def _fp64_bounds(p, f, B, target):
    """First-order bounds on |model_bf16 - model_fp64| for the force and the
    gradient, from the bf16 unit roundoff u of the operands each matrix
    product rounds (both operands: 2u), propagated through SiLU (|silu'| <=
    1.1, |silu''| <= 0.5) and the backward products; 1e-5 of the absolute
    terms covers the FP32 accumulations.  Returns (e_F, e_grad dict)."""
    u = U_BF16
    a = np.abs
    W1, W2, W3 = p["W1"], p["W2"], p["W3"]
    z1 = f @ W1.T + p["b1"]
    h1 = S.silu(z1)
    z2 = h1 @ W2.T + p["b2"]
    h2 = S.silu(z2)
    c = h2 @ W3.T + p["b3"]
    F = np.einsum("nj,nja->na", c[:, :S.N_CH], B)
    e_z1 = 2 * u * (a(f) @ a(W1).T)
    e_h1 = 1.1 * e_z1
    e_z2 = 2 * u * (a(h1) @ a(W2).T) + e_h1 @ a(W2).T
    e_h2 = 1.1 * e_z2
    e_c = 2 * u * (a(h2) @ a(W3).T) + e_h2 @ a(W3).T
    absF = np.einsum("nj,nja->na", a(c[:, :S.N_CH]), a(B))
    e_F = np.einsum("nj,nja->na", e_c[:, :S.N_CH], a(B)) + 1e-5 * absF
    N = f.shape[0]
    dF = 2.0 * (F - target) / N
    e_dF = 2.0 * e_F / N
    dc = np.zeros((N, S.N_OUT))
    e_dc = np.zeros((N, S.N_OUT))
    dc[:, :S.N_CH] = np.einsum("na,nja->nj", dF, B)
    e_dc[:, :S.N_CH] = np.einsum("na,nja->nj", e_dF, a(B)) + 1e-5 * np.einsum("na,nja->nj", a(dF), a(B))
    s2, s1 = S.dsilu(z2), S.dsilu(z1)
    dh2 = dc @ W3
    e_dh2 = 2 * u * (a(dc) @ a(W3)) + e_dc @ a(W3)
    dz2 = dh2 * s2
    e_dz2 = e_dh2 * a(s2) + a(dh2) * 0.5 * e_z2
    dh1 = dz2 @ W2
    e_dh1 = 2 * u * (a(dz2) @ a(W2)) + e_dz2 @ a(W2)
    dz1 = dh1 * s1
    e_dz1 = e_dh1 * a(s1) + a(dh1) * 0.5 * e_z1
    acc = 1e-5
    e = {"W3": (2 * u * a(dc) + e_dc).T @ a(h2) + a(dc).T @ e_h2 + acc * (a(dc).T @ a(h2)),
         "b3": e_dc.sum(0) + acc * a(dc).sum(0),
         "W2": (2 * u * a(dz2) + e_dz2).T @ a(h1) + a(dz2).T @ e_h1 + acc * (a(dz2).T @ a(h1)),
         "b2": e_dz2.sum(0) + acc * a(dz2).sum(0),
         "W1": (2 * u * a(dz1) + e_dz1).T @ a(f) + acc * (a(dz1).T @ a(f)),
         "b1": e_dz1.sum(0) + acc * a(dz1).sum(0)}
    return e_F, e


@pytest.mark.parametrize("with_aux", [False, True])
def test_c4_size_force_matches_oracle(with_aux):
    """Model force at 16^3x8 against the oracle's bf16 mode (same rounding
    points) and against its FP64 mode within the bf16 roundoff bound."""
    log(f"surrogate force 16^3x8 aux={with_aux}")
    U, _, aux = _c4_setup(with_aux)
    lat = lattice(C4, U)
    sur = stag.Surrogate(lat, 1)
    p = _params(11)
    sur.set_params(_flat(p))
    if with_aux:
        aux_dev = lat.mom_import(dev(aux))
        sur.set_aux(aux_dev)
    mom = lat.new_mom()
    sur.force(mom, 0.0)
    got = host(lat.mom_export(mom)).reshape(-1, 8)
    f, loops = S.features(U, C4, aux)
    B = S.basis(loops, aux)
    exp_bf, _ = S.forward(p, f, B, mode="bf16")
    scale = np.abs(exp_bf).max()
    assert np.abs(got - exp_bf).max() < 3e-3 * scale
    assert np.sqrt(np.mean((got - exp_bf) ** 2)) < 2e-4 * scale
    exp64, _ = S.forward(p, f, B, mode="fp64")
    e_F, _ = _fp64_bounds(p, f, B, np.zeros_like(exp64))
    ratio = np.abs(got - exp64) / e_F
    log(f"  max |F_gpu - F_fp64| / bound = {ratio.max():.3f}")
    assert ratio.max() <= 1.0


def test_c4_size_loss_gradient_and_adam_match_oracle():
    """Loss and gradient at 16^3x8 (with the auxiliary channel) against the
    oracle's bf16 mode and, within the bf16 roundoff bound, its FP64 mode;
    then two Adam steps of the GPU trainer against the oracle's Adam applied
    to the same gradients."""
    log("surrogate loss / gradient / Adam 16^3x8")
    U, target, aux = _c4_setup(True, seed=1)
    lat = lattice(C4, U)
    sur = stag.Surrogate(lat, 1)
    p = _params(12)
    sur.set_params(_flat(p))
    aux_dev = lat.mom_import(dev(aux))
    sur.set_aux(aux_dev)
    tdev = lat.mom_import(dev(target))
    loss, g = sur.eval(tdev, want_grad=True)
    f, loops = S.features(U, C4, aux)
    tf = target.reshape(-1, 8).astype(np.float32).astype(np.float64)
    B = S.basis(loops, aux).astype(np.float32).astype(np.float64)
    lref, gref = S.loss_and_grad(p, f, B, tf, mode="bf16")
    assert abs(loss - lref) < 1e-4 * lref
    gg = _unflat(g.astype(np.float64))
    for k in KEYS:
        err = np.abs(gg[k] - gref[k]).max() / max(np.abs(gref[k]).max(), 1e-30)
        assert err < 2e-2, (k, err)
    l64, g64 = S.loss_and_grad(p, f, B, tf, mode="fp64")
    _, e_g = _fp64_bounds(p, f, B, tf)
    for k in KEYS:
        # zero bound: entries fed only by zero-padded features must be exactly zero
        diff, zero = np.abs(gg[k] - g64[k]), e_g[k] == 0
        assert (diff[zero] == 0).all(), k
        ratio = (diff[~zero] / e_g[k][~zero]).max()
        log(f"  {k}: max |g_gpu - g_fp64| / bound = {ratio:.3f}")
        assert ratio <= 1.0, k
    # Adam: the trainer's step on its one pair uses the gradient eval returns
    sur.add_pair(tdev)
    state = {}
    ref = {k: v.copy() for k, v in p.items()}
    lr = 3e-3
    for step in range(2):
        _, gs = sur.eval(tdev, want_grad=True)
        sur.train(1, lr)
        S.adam_step(ref, _unflat(gs.astype(np.float64)), state, lr=lr)
        got = _unflat(sur.get_params().astype(np.float64))
        for k in KEYS:
            d = np.abs(got[k] - ref[k])
            tol = 1e-5 * lr + 2.0 ** -23 * np.abs(ref[k])
            assert (d <= tol).all(), (step, k, d.max())
        moved = np.abs(got["W2"] - p["W2"]).max()
        assert 0.5 * lr * (step + 1) < moved <= 1.01 * lr * (step + 1)


def test_learned_inner_force_leapfrog_is_reversible():
    """The inner-scale force of the learned schedule -- the model applied to
    the force of a solve stopped after a fixed number of iterations -- is a
    deterministic function of the links and the pseudofermion, so a
    two-time-scale leapfrog with it (exact force on the outer kicks), run
    forward, momenta flipped and run again, returns to the starting links and
    the negated momenta: the property that keeps the schedules exact."""
    dims = (8, 8, 8, 8)
    log("learned-schedule leapfrog reversibility at 8^4")
    rng = synth.make_rng(708, 0)
    U0 = synth.random_su3_near_identity(dims, 0.3, rng)
    phi = synth.gaussian_half_vector(dims, rng)
    rat = synth.load_rational("xm050_n12_m0.02")
    lat = lattice(dims, U0)
    phid = lat.vec_import(dev(phi), 0)
    sur = stag.Surrogate(lat, 1)
    sur.set_params(_flat(_params(3)))
    aux = lat.new_mom()
    mom = lat.random_momentum(9, 2)
    P0 = host(lat.mom_export(mom))
    dt, n, every = 0.05, 4, 2

    def kick(h, exact):
        lat.gauge_force(5.4, mom, h)
        if exact:
            lat.fermion_force(0.02, rat, 1e-12, 100000, phid, mom, h)
        else:
            lat.fermion_force(0.02, rat, 1e-30, 30, phid, aux, 0.0, allow_not_converged=True)
            sur.set_aux(aux)
            sur.force(mom, h)
            sur.set_aux(None)

    def leapfrog():
        kick(0.5 * dt, True)
        for s in range(n):
            lat.link_update(mom, dt)
            k = s + 1
            kick(dt if k < n else 0.5 * dt, k % every == 0)

    leapfrog()
    U1 = host(lat.get_gauge())
    assert np.abs(U1 - U0).max() > 1e-3
    mom.copy_(lat.mom_import(dev(-host(lat.mom_export(mom)))))
    leapfrog()
    U2 = host(lat.get_gauge())
    P2 = host(lat.mom_export(mom))
    assert np.abs(U2 - U0).max() < 1e-8, np.abs(U2 - U0).max()
    assert np.abs(P2 + P0).max() < 1e-7 * np.abs(P0).max(), np.abs(P2 + P0).max()
