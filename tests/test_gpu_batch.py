"""Batched form: lattices of uneven volume x right-hand sides x poles in one
multi-shift solve, FP64 and mixed FP32/FP64, against the oracle."""
import numpy as np
import pytest

import synth
from oracle import dirac
from oracle.solvers import multishift_cg, true_residuals
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, log

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (6, 4, 2, 8), (8, 6, 4, 10), (2, 2, 2, 2), (4, 2, 6, 4)]
POLES = list(np.logspace(-4, 0, 5))


def _setup(nrhs, seed=0):
    rng = synth.make_rng(500, seed)
    Us = [synth.random_su3_near_identity(d, 0.4, rng) for d in DIMS]
    masses = list(rng.uniform(0.005, 0.05, len(DIMS)))
    bs = [[synth.gaussian_half_vector(d, rng) for _ in range(nrhs)] for d in DIMS]
    packed = np.concatenate([b.reshape(-1) for per in bs for b in per])
    B = stag.Batch(DIMS, nrhs)
    for i, U in enumerate(Us):
        B.set_gauge(i, dev(U))
    return B, Us, masses, bs, dev(packed)


def _unpack(x_pole, nrhs):
    out, off = [], 0
    for d in DIMS:
        vh = d[0] * d[1] * d[2] * d[3] // 2
        per = []
        for _ in range(nrhs):
            per.append(x_pole[off:off + 3 * vh].reshape(vh, 3))
            off += 3 * vh
        out.append(per)
    return out


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nrhs", [1, 3, 4])
def test_batch_matches_oracle(precision, nrhs):
    _check_against_oracle(precision, nrhs, None)


@pytest.mark.parametrize("precision,nrhs", [(0, 1), (0, 4), (1, 3)])
def test_eight_lanes_per_site_matches_oracle(precision, nrhs):
    """The hop-per-lane Dslash (8 lanes per site, lane exchanges instead of
    LDS), including the 2^4 lattice whose single tile is mostly off-lattice."""
    _check_against_oracle(precision, nrhs, 8)


@pytest.mark.parametrize("precision,nrhs,tps", [(0, 4, None), (1, 3, None), (0, 2, 8), (1, 1, 8)])
def test_twelve_real_link_reads_match_oracle(precision, nrhs, tps):
    """The batched operators reading rows 0-1 of every link and rebuilding row
    2 (FP64, and the mixed form's FP32 operator): solutions against the
    oracle as with all 18 reals, for the LDS and the hop-per-lane splits."""
    _check_against_oracle(precision, nrhs, tps, link12=True)


def _check_against_oracle(precision, nrhs, tps, link12=False):
    log(f"batched solve precision={precision} nrhs={nrhs} tps={tps} link12={link12}")
    B, Us, masses, bs, bdev_ = _setup(nrhs)
    if tps:
        B.set_tps(tps)
    if link12:
        B.set_link_format(stag.LINKS_F64_12)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    x, info = B.solve(masses, rat, bdev_, precision=precision, tol=1e-10)
    xh = host(x)
    sols = [_unpack(xh[k], nrhs) for k in range(len(POLES))]
    assert info["true_resid"].max() < 1e-10
    for i, (d, U, m) in enumerate(zip(DIMS, Us, masses)):
        op = lambda v: dirac.apply_A(U, v, d, m)
        for j in range(nrhs):
            xs = [sols[k][i][j] for k in range(len(POLES))]
            res = true_residuals(op, bs[i][j], POLES, xs)
            assert res.max() < 1e-10, (i, j, res)
            if j == 0:
                ref = multishift_cg(op, bs[i][j], POLES, 1e-12)
                for sig, xg, xr in zip(POLES, xs, ref["x"]):
                    kappa = (4 * m * m + 64 + sig) / (4 * m * m + sig)
                    assert np.linalg.norm(xg - xr) <= 1.1e-10 * kappa * np.linalg.norm(xr)
    assert all(v > 0 for v in info["latency"])


def test_graph_and_stream_paths_agree_bitwise():
    B, Us, masses, bs, bd = _setup(2, seed=1)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    xa, ia = B.solve(masses, rat, bd, use_graph=True)
    xb, ib = B.solve(masses, rat, bd, use_graph=False)
    assert ia["iters"] == ib["iters"]
    assert np.array_equal(host(xa), host(xb))


def test_tune_and_errors():
    B, Us, masses, bs, bd = _setup(2, seed=2)
    us = B.tune(0)
    assert len(us) == 4 and all(u > 0 for u in us)
    with pytest.raises(stag.StagError):
        B.set_tps(3)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    x, info = B.solve(masses, rat, bd)   # still correct after retiling
    assert info["true_resid"].max() < 1e-10
    with pytest.raises(stag.StagError):
        stag.Batch([(4, 4, 4, 3)], 1)
    with pytest.raises(stag.StagError):
        stag.Batch([(4, 4, 4, 4)], 5)
    C = stag.Batch([(4, 4, 4, 4), (2, 2, 2, 2)], 1)
    C.set_gauge(0, dev(Us[0]))
    with pytest.raises(stag.StagError) as e:
        C.solve([0.1, 0.1], rat, dev(np.zeros(C.vec_len(), dtype=np.complex128)))
    assert e.value.code == stag.STAG_ERR_NO_GAUGE


@pytest.mark.parametrize("precision", [0, 1])
def test_shift_window_does_not_change_results(precision):
    """Windows of 1, 2, 4 and 8 iterations give bitwise the same solutions."""
    B, Us, masses, bs, bd = _setup(3, seed=3)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    ref = None
    for lag in (1, 2, 4, 8):
        log(f"batched window {lag} precision={precision}")
        B.set_shift_window(lag)
        x, info = B.solve(masses, rat, bd, precision=precision)
        got = host(x)
        if ref is None:
            ref, ref_info = got, info
        else:
            assert info["iters_sys"] == ref_info["iters_sys"]
            assert np.array_equal(got, ref), lag
    with pytest.raises(stag.StagError):
        B.set_shift_window(3)


def test_eight_lanes_per_site_window_invariance_and_agreement():
    """With the hop-per-lane operator (32-site tiles) windows 1 and 8 agree
    bitwise, and the solutions agree with the 4-threads-per-site split (the
    two sum a site's hops in different orders; both reach the FP64 true
    residual, so they differ by at most tol times the condition number)."""
    B, Us, masses, bs, bd = _setup(4, seed=4)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    out = {}
    for tps in (4, 8):
        B.set_tps(tps)
        for lag in (1, 8):
            log(f"batched tps={tps} window {lag}")
            B.set_shift_window(lag)
            x, info = B.solve(masses, rat, bd)
            out[tps, lag] = host(x)
            assert info["true_resid"].max() < 1e-10
    assert np.array_equal(out[8, 1], out[8, 8])
    assert np.array_equal(out[4, 1], out[4, 8])
    ref = out[4, 8]
    assert np.abs(out[8, 8] - ref).max() <= 1e-6 * np.abs(ref).max()


def test_large_instances_window_and_residuals():
    """Many more tiles than the GPU runs at once (6 x 24^3x6 + 2 x 16^3x8 +
    8^4, 4 right-hand sides: 2216 tiles of 128 sites) and the 12-pole table:
    window 8 equals window 1 bitwise and every system reaches the FP64 true
    residual.  This is where a block that starts after another block of the
    same launch has recorded a stop must still apply the pending window."""
    dims = [(24, 24, 24, 6)] * 6 + [(16, 16, 16, 8)] * 2 + [(8, 8, 8, 8)]
    rng = synth.make_rng(501, 0)
    Us = [synth.random_su3_near_identity(d, 0.2, rng) for d in dims]
    masses = list(rng.uniform(0.005, 0.05, len(dims)))
    nrhs = 4
    b = np.concatenate([synth.gaussian_half_vector(d, rng).reshape(-1) for d in dims for _ in range(nrhs)])
    B = stag.Batch(dims, nrhs)
    for i, U in enumerate(Us):
        B.set_gauge(i, dev(U))
    rat = synth.load_rational("xm025_n12_m0.005")
    out = {}
    for lag in (1, 8):
        log(f"large batch, window {lag}")
        B.set_shift_window(lag)
        x, info = B.solve(masses, rat, dev(b), precision=0, tol=1e-10)
        out[lag] = (host(x), info)
        assert info["true_resid"].max() < 1e-10, info["true_resid"].max()
    assert out[1][1]["iters_sys"] == out[8][1]["iters_sys"]
    assert np.array_equal(out[1][0], out[8][0])


def test_full_size_64_lattices_against_oracle():
    """The batched workload at its full size: 64 lattices (16 each of 8^4,
    12^3x6, 16^3x8, 24^3x6) x 4 right-hand sides x the 12-pole x^(-1/4)
    table, masses uniform in [0.005, 0.05].  FP64: for every lattice (one
    right-hand side each, rotating) the oracle's operator gives every pole's
    true residual below 1e-10 and matches the library's own FP64 residual;
    mixed precision, and FP64 reading 12 reals per link: the same for one
    lattice of each volume."""
    from concurrent.futures import ThreadPoolExecutor
    classes = [(8, 8, 8, 8), (12, 12, 12, 6), (16, 16, 16, 8), (24, 24, 24, 6)]
    dims = [d for d in classes for _ in range(16)]
    nrhs = 4
    rng = synth.make_rng(502, 0)
    masses = list(rng.uniform(0.005, 0.05, len(dims)))
    with ThreadPoolExecutor(8) as ex:
        Us = list(ex.map(lambda i: synth.random_su3_near_identity(dims[i], 0.2, synth.make_rng(502, 1000 + i)),
                         range(len(dims))))
    srcs = [[synth.gaussian_half_vector(d, synth.make_rng(502, 5000 + 8 * i + j)) for j in range(nrhs)]
            for i, d in enumerate(dims)]
    B = stag.Batch(dims, nrhs)
    for i, U in enumerate(Us):
        B.set_gauge(i, dev(U))
    b = dev(np.concatenate([v.reshape(-1) for per in srcs for v in per]))
    rat = synth.load_rational("xm025_n12_m0.005")
    offs = np.cumsum([0] + [nrhs * 3 * (d[0] * d[1] * d[2] * d[3] // 2) for d in dims])

    def system(xh, i, j):
        vh = dims[i][0] * dims[i][1] * dims[i][2] * dims[i][3] // 2
        o = offs[i] + j * 3 * vh
        return [xh[k][o:o + 3 * vh].reshape(vh, 3) for k in range(len(rat["pole"]))]

    for precision, link12, sample in ((0, False, range(len(dims))), (1, False, [0, 16, 32, 48]),
                                      (0, True, [1, 17, 33, 49])):
        log(f"full-size batch precision={precision} link12={link12}")
        B.set_link_format(stag.LINKS_F64_12 if link12 else stag.LINKS_F64_18)
        x, info = B.solve(masses, rat, b, precision=precision, tol=1e-10)
        xh = host(x)
        for i in sample:
            j = i % nrhs
            op = lambda v, i=i: dirac.apply_A(Us[i], v, dims[i], masses[i])
            res = true_residuals(op, srcs[i][j], rat["pole"], system(xh, i, j))
            assert res.max() < 1e-10, (precision, i, j, res.max())
            lib = info["true_resid"][i * nrhs + j]
            # both residuals are computed in FP64; near 1e-10 their rounding
            # (about 1e-16 |A| |x|) is a visible fraction of the residual itself
            assert np.all(np.abs(lib - res) <= 0.1 * res + 1e-12), (precision, i, j)
        del x, xh


def test_autotune_cache_and_link_loads(tmp_path):
    """The autotuner times every candidate, appends its choice to the cache
    file and takes it from there on the next call; the solver's results are
    bitwise the same for plain and non-temporal link loads (choices forced
    through the cache file)."""
    B, Us, masses, bs, bd = _setup(2, seed=3)
    cache = str(tmp_path / "tune.txt")
    us, choice = B.autotune(0, cache)
    assert all(u > 0 for u in us) and choice[2] == 0
    lines = open(cache).read().split("\n")
    key = lines[0].split()[0]
    assert len([ln for ln in lines if ln.strip()]) == 1
    us2, choice2 = B.autotune(0, cache)
    assert choice2[:2] == choice[:2] and choice2[2] == 1 and all(u == -1.0 for u in us2)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    got = []
    for nt in (0, 1):
        forced = str(tmp_path / f"forced{nt}.txt")
        with open(forced, "w") as f:
            f.write(f"{key} 4 {nt} 1.0\n")
        _, ch = B.autotune(0, forced)
        assert ch == (4, nt, 1)
        x, info = B.solve(masses, rat, bd)
        assert info["true_resid"].max() < 1e-10
        got.append(host(x))
    assert np.array_equal(got[0], got[1])


def test_repeated_batched_solves_with_the_iteration_estimate():
    """Later solves of the same kind replay the cached chunk graphs and
    schedule their chunks from the previous iteration count: bitwise the
    first solve's solutions and counts, also right after a solve of the same
    kind stopped at maxiter = 6 (an estimate far too short)."""
    B, Us, masses, bs, bd = _setup(2, seed=4)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * len(POLES)}
    x0, i0 = B.solve(masses, rat, bd, true_resid=False)
    x0 = host(x0)
    for _ in range(2):
        x1, i1 = B.solve(masses, rat, bd, true_resid=False)
        assert i1["iters"] == i0["iters"]
        assert np.array_equal(host(x1), x0)
    _, ishort = B.solve(masses, rat, bd, maxiter=6, true_resid=False, allow_not_converged=True)
    assert ishort["iters"] == 6
    x2, i2 = B.solve(masses, rat, bd, true_resid=False)
    assert i2["iters"] == i0["iters"]
    assert np.array_equal(host(x2), x0)
