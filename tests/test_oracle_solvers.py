"""Pins for the oracle's CG and multi-shift CG (paper Sec. 4)."""
import numpy as np

import synth
from oracle import dirac, lattice as L
from oracle.solvers import cg, multishift_cg, true_residuals, vdot

DIMS = (4, 4, 4, 4)
SIGMAS = np.logspace(-4, 0, 8)


def _setup(eps=0.3, kind=0, mass=0.1):
    rng = synth.make_rng(901, kind)
    U = synth.random_su3_near_identity(DIMS, eps, rng)
    b = synth.gaussian_half_vector(DIMS, rng)
    return U, b, (lambda v: dirac.apply_A(U, v, DIMS, mass))


def _dense(op, vh):
    cols = []
    for k in range(3 * vh):
        e = np.zeros((vh, 3), dtype=np.complex128)
        e.reshape(-1)[k] = 1
        cols.append(op(e).reshape(-1))
    return np.array(cols).T


def test_multishift_matches_dense_solve():
    U, b, op = _setup()
    A = _dense(op, b.shape[0])
    sol = multishift_cg(op, b, SIGMAS, 1e-12)
    for s, x in zip(SIGMAS, sol["x"]):
        xd = np.linalg.solve(A + s * np.eye(A.shape[0]), b.reshape(-1))
        assert np.linalg.norm(x.reshape(-1) - xd) <= 1e-10 * np.linalg.norm(xd)
    assert true_residuals(op, b, SIGMAS, sol["x"]).max() < 1e-11


def test_collinear_shifted_residuals():
    """After any number of iterations the true residual of every shifted system
    equals zeta_i times the base residual."""
    U, b, op = _setup(eps=0.8, kind=1)
    bn = np.sqrt(vdot(b, b).real)
    for k in (1, 3, 7):
        sol = multishift_cg(op, b, SIGMAS, 1e-30, maxiter=k)
        for i, (s, x) in enumerate(zip(SIGMAS, sol["x"])):
            res = b - (op(x) + s * x)
            assert np.linalg.norm(res - sol["zeta"][i] * sol["r"]) <= 1e-12 * bn


def test_free_field_plane_wave_and_krylov_bound():
    """At U = 1 a plane-wave source gives x_i = b / (lambda(p) + sigma_i); on 4^4
    A has only 4 distinct eigenvalues so all shifts converge in <= 4 iterations."""
    nx, ny, nz, nt = DIMS
    U = np.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    m = 0.1
    op = lambda v: dirac.apply_A(U, v, DIMS, m)
    x, y, z, t = L.coords(DIMS)
    p = (np.pi / 2, 0.0, np.pi, 3 * np.pi / 4)
    lam = 4 * m * m + 4 * sum(np.sin(q) ** 2 for q in p)
    wave = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None] * np.array([1.0, 0.5j, -0.25])
    b = L.full_to_half(wave, DIMS, 0)
    sol = multishift_cg(op, b, SIGMAS, 1e-12)
    for s, xs in zip(SIGMAS, sol["x"]):
        assert np.abs(xs - b / (lam + s)).max() < 1e-12
    rng = synth.make_rng(901, 7)
    b2 = synth.gaussian_half_vector(DIMS, rng)
    sol2 = multishift_cg(op, b2, SIGMAS, 1e-12)
    assert sol2["iters"] <= 4
    assert true_residuals(op, b2, SIGMAS, sol2["x"]).max() < 1e-12


def test_each_pole_matches_single_shift_cg():
    U, b, op = _setup(eps=0.5, kind=2)
    sol = multishift_cg(op, b, SIGMAS, 1e-11)
    for s, x in zip(SIGMAS, sol["x"]):
        xc, _ = cg(lambda v: op(v) + s * v, b, 1e-12)
        assert np.linalg.norm(x - xc) <= 1e-9 * np.linalg.norm(xc)


def test_zero_source_and_tolerance_semantics():
    U, b, op = _setup(kind=3)
    sol = multishift_cg(op, np.zeros_like(b), SIGMAS, 1e-10)
    assert sol["iters"] == 0 and all(np.all(x == 0) for x in sol["x"])
    sol = multishift_cg(op, b, SIGMAS, 1e-6)
    res = true_residuals(op, b, SIGMAS, sol["x"])
    assert res.max() < 2e-6
    # heavier shifts freeze earlier
    assert sol["iters_per_pole"][-1] <= sol["iters_per_pole"][0]
