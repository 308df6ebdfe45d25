"""Precision form: 12-real FP64 link compression (exact for SU(3)) and the
mixed-precision multi-shift solve (FP32 Krylov vectors, FP32 or FP16-12 links,
FP64 reliable updates) reaching the FP64 true residual, against the oracle."""
import numpy as np
import pytest

import synth
from oracle import dirac
from oracle.solvers import multishift_cg, true_residuals
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, lattice, log, rel_err

pytestmark = pytest.mark.gpu

POLES = list(np.logspace(-4, 0, 8))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 6, 4, 10)])
def test_fp64_12real_dslash(dims):
    log(f"12-real FP64 Dslash dims={dims}")
    rng = synth.make_rng(400, 0)
    U = synth.random_su3_near_identity(dims, 0.5, rng)
    lat = lattice(dims, U)
    lat.set_link_format(stag.LINKS_F64_12)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash(y, lat.vec_import(dev(vin), 1 - out_par), out_par)
        assert rel_err(host(lat.vec_export(y, out_par)), dirac.dslash_half(U, vin, dims, out_par)) < 1e-13


@pytest.mark.parametrize("sloppy", [stag.LINKS_F32_18, stag.LINKS_F16_12])
@pytest.mark.parametrize("dims,eps,mass", [((4, 4, 4, 4), 0.3, 0.1), ((8, 6, 4, 10), 0.4, 0.05)])
def test_mixed_solve_reaches_fp64_residual(sloppy, dims, eps, mass):
    log(f"mixed solve sloppy={sloppy} dims={dims}")
    rng = synth.make_rng(401, 0)
    U = synth.random_su3_near_identity(dims, eps, rng)
    b = synth.gaussian_half_vector(dims, rng)
    lat = lattice(dims, U)
    rat = {"c0": 0.0, "pole": POLES, "residue": [1.0] * 8}
    xs = [lat.new_vec() for _ in POLES]
    info = lat.multishift_solve_mixed(mass, rat, 1e-10, 100000, lat.vec_import(dev(b), 0), xs, sloppy=sloppy)
    xh = [host(lat.vec_export(x, 0)) for x in xs]
    op = lambda v: dirac.apply_A(U, v, dims, mass)
    res = true_residuals(op, b, POLES, xh)
    assert res.max() < 1e-10, res
    ref = multishift_cg(op, b, POLES, 1e-12)
    lmin, lmax = 4 * mass * mass, 4 * mass * mass + 64
    for sig, x, xr in zip(POLES, xh, ref["x"]):
        kappa = (lmax + sig) / (lmin + sig)
        assert np.linalg.norm(x - xr) <= 1.1e-10 * kappa * np.linalg.norm(xr)


@pytest.mark.parametrize("sloppy", [stag.LINKS_F32_18, stag.LINKS_F16_12])
def test_mixed_full_size_32c8(sloppy):
    dims = (32, 32, 32, 8)
    log(f"mixed solve at 32^3x8 sloppy={sloppy}")
    rng = synth.make_rng(1, 0)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    b = synth.gaussian_half_vector(dims, synth.make_rng(1, 1))
    rat = synth.load_rational("xm025_n12_m0.005")
    lat = lattice(dims, U)
    xs = [lat.new_vec() for _ in rat["pole"]]
    info = lat.multishift_solve_mixed(0.005, rat, 1e-10, 100000, lat.vec_import(dev(b), 0), xs, sloppy=sloppy)
    log(f"  iterations {info['iters']} seconds {info['seconds']:.3f} per pole {info['iters_per_pole']}")
    xh = [host(lat.vec_export(x, 0)) for x in xs]
    res = true_residuals(lambda v: dirac.apply_A(U, v, dims, 0.005), b, rat["pole"], xh)
    assert res.max() < 1e-10, res
    assert max(info["true_resid"]) < 1e-10
