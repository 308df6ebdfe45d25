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


# ---- element-wise error of the sloppy operators against the FP64 oracle ----
# Bounds from the roundoff of each format, per output element x:
#   P(x) = sum over the 8 neighbours y of sum_b (|Re psi_b(y)| + |Im psi_b(y)|)
# (|U_ab| <= 1 for SU(3)).  An output real part is a sum of 48 real products
# of a rounded link entry and a rounded vector entry, so FP32 arithmetic with
# FP32-18 links errs by at most (48 + 2) u32 P(x) with u32 = 2^-24.  FP16-12
# links hold rows 0-1 with relative error u16 = 2^-11 each, and row 2 rebuilt
# as conj(row0 x row1) errs by at most 2 u16 (1 + u16) in absolute value
# (two products of unit-row entries, both rounded), so the link error adds
# 2.1 u16 sqrt(2) P(x).
U32, U16 = 2.0 ** -24, 2.0 ** -11
BOUND_COEF = {stag.LINKS_F32_18: 50 * U32, stag.LINKS_F16_12: 2.1 * U16 * np.sqrt(2) + 50 * U32}


def _neighbour_sum(v_half, dims, in_par):
    """P(x) on the sites of the other parity, from a half vector of parity in_par."""
    from oracle import lattice as L
    s = np.abs(v_half.real).sum(-1) + np.abs(v_half.imag).sum(-1)
    full = L.half_to_full(s[:, None], dims, in_par)[..., 0]
    tot = sum(L.fwd(full, mu) + L.bwd(full, mu) for mu in range(4))
    return L.full_to_half(tot[..., None], dims, 1 - in_par)[:, 0]


@pytest.mark.parametrize("sloppy", [stag.LINKS_F32_18, stag.LINKS_F16_12])
def test_sloppy_dslash_elementwise_32c8(sloppy):
    """D_oe and D_eo of the sloppy formats at 32^3x8, every output element
    within the roundoff bound of its format, and the measured error stated."""
    dims = (32, 32, 32, 8)
    log(f"sloppy Dslash at 32^3x8 format={sloppy}")
    rng = synth.make_rng(402, sloppy)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = lattice(dims, U)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash_sloppy(y, lat.vec_import(dev(vin), 1 - out_par), out_par, sloppy)
        got = host(lat.vec_export(y, out_par))
        exp = dirac.dslash_half(U, vin, dims, out_par)
        P = _neighbour_sum(vin, dims, 1 - out_par)[:, None]
        err = np.maximum(np.abs(got.real - exp.real), np.abs(got.imag - exp.imag))
        ratio = err / (BOUND_COEF[sloppy] * P)
        log(f"  out parity {out_par}: max |err| / P = {(err / P).max():.3e}, "
            f"relative (max norm) {rel_err(got, exp):.3e}, max err / bound {ratio.max():.3f}")
        assert ratio.max() <= 1.0


@pytest.mark.parametrize("sloppy", [stag.LINKS_F32_18, stag.LINKS_F16_12])
def test_sloppy_mdagm_32c8(sloppy):
    """A = 4m^2 - D_eo D_oe in the sloppy formats at 32^3x8.  w = D_oe psi errs
    by e_w(x) <= c P_psi(x) (above); D_eo then adds its own c P_w(x) and passes
    e_w through links of norm <= 1: e_A(x) <= c P_w(x) + sum over neighbours
    of 3 sqrt(2) e_w(y) + u32 (4m^2 |psi(x)| + |A psi(x)|) for the final axpy."""
    dims = (32, 32, 32, 8)
    mass = 0.005
    log(f"sloppy A at 32^3x8 format={sloppy}")
    rng = synth.make_rng(403, sloppy)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = lattice(dims, U)
    vin = synth.gaussian_half_vector(dims, rng)
    y = lat.new_vec()
    lat.mdagm_sloppy(y, lat.vec_import(dev(vin), 0), mass, sloppy)
    got = host(lat.vec_export(y, 0))
    exp = dirac.apply_A(U, vin, dims, mass)
    c = BOUND_COEF[sloppy]
    w = dirac.dslash_half(U, vin, dims, 1)
    e_w = c * _neighbour_sum(vin, dims, 0)
    from oracle import lattice as L
    full = L.half_to_full(e_w[:, None], dims, 1)[..., 0]
    prop = L.full_to_half(sum(L.fwd(full, mu) + L.bwd(full, mu) for mu in range(4))[..., None], dims, 0)[:, 0]
    bound = (c * _neighbour_sum(w, dims, 1) + 3 * np.sqrt(2) * prop)[:, None] \
        + U32 * (4 * mass * mass * np.abs(vin) + 2 * np.abs(exp))
    err = np.maximum(np.abs(got.real - exp.real), np.abs(got.imag - exp.imag))
    log(f"  relative (max norm) {rel_err(got, exp):.3e}, max err / bound {(err / bound).max():.3f}")
    assert (err <= bound).all()


def test_fp64_12real_dslash_32c8():
    """FP64 12-real links at full size: exact to FP64 rounding, like 18-real."""
    dims = (32, 32, 32, 8)
    log("12-real FP64 Dslash at 32^3x8")
    rng = synth.make_rng(404, 0)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = lattice(dims, U)
    lat.set_link_format(stag.LINKS_F64_12)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        y = lat.new_vec()
        lat.dslash(y, lat.vec_import(dev(vin), 1 - out_par), out_par)
        assert rel_err(host(lat.vec_export(y, out_par)), dirac.dslash_half(U, vin, dims, out_par)) < 1e-13
    x = lat.vec_import(dev(vin), 0)
    lat.mdagm(y, x, 0.005)
    assert rel_err(host(lat.vec_export(y, 0)), dirac.apply_A(U, vin, dims, 0.005)) < 1e-13
