"""GPU parity of the even-odd Dslash and the half-lattice operator against the
oracle (Sec. 3.2), element by element, over several tiles, ragged tails, every
work split, and the full 32^3x8 lattice."""
import numpy as np
import pytest

import synth
from oracle import dirac
from tests.gpu_util import dev, host, lattice, log, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 0.3),      # 4^4 configuration
    ((2, 2, 2, 2), 0.5),      # smallest lattice: every neighbour wraps
    ((8, 6, 4, 10), 0.4),     # Vh = 960: several tiles and a ragged tail
    ((6, 2, 8, 4), 1.0),      # strongly disordered links
    ((8, 8, 16, 4), 0.3),     # z-slab tile map with two (z, t) planes per tile (4 threads per site)
    ((16, 16, 16, 8), 0.2),   # z-slab tile map for every work split
]


@pytest.mark.parametrize("dims,eps", CASES)
@pytest.mark.parametrize("tps", [1, 2, 4])
def test_dslash_matches_oracle(dims, eps, tps):
    log(f"dslash parity dims={dims} eps={eps} tps={tps}")
    rng = synth.make_rng(100, hash(dims) % 1000)
    U = synth.random_su3_near_identity(dims, eps, rng)
    lat = lattice(dims, U)
    lat.tune(tps, 16)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        x = lat.vec_import(dev(vin), 1 - out_par)
        y = lat.new_vec()
        lat.dslash(y, x, out_par)
        got = host(lat.vec_export(y, out_par))
        exp = dirac.dslash_half(U, vin, dims, out_par)
        assert rel_err(got, exp) < 1e-14, (out_par, rel_err(got, exp))


@pytest.mark.parametrize("dims,eps", CASES[:3])
def test_mdagm_matches_oracle(dims, eps):
    log(f"mdagm parity dims={dims}")
    rng = synth.make_rng(101, 0)
    U = synth.random_su3_near_identity(dims, eps, rng)
    lat = lattice(dims, U)
    vin = synth.gaussian_half_vector(dims, rng)
    x = lat.vec_import(dev(vin), 0)
    y = lat.new_vec()
    lat.mdagm(y, x, 0.1)
    got = host(lat.vec_export(y, 0))
    exp = dirac.apply_A(U, vin, dims, 0.1)
    assert rel_err(got, exp) < 1e-14


@pytest.mark.parametrize("tps", [1, 2, 4])
def test_full_size_32c8(tps):
    """32^3x8, eps = 0.2: every output element of D_oe and D_eo."""
    dims = (32, 32, 32, 8)
    log(f"dslash parity at 32^3x8 tps={tps}")
    rng = synth.make_rng(1, 0)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = lattice(dims, U)
    lat.tune(tps, 16)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        x = lat.vec_import(dev(vin), 1 - out_par)
        y = lat.new_vec()
        lat.dslash(y, x, out_par)
        got = host(lat.vec_export(y, out_par))
        exp = dirac.dslash_half(U, vin, dims, out_par)
        assert rel_err(got, exp) < 1e-14


def test_layout_roundtrips_are_exact():
    dims = (8, 6, 4, 10)
    rng = synth.make_rng(102, 0)
    U = synth.haar_su3(dims, rng)
    lat = lattice(dims, U)
    assert np.array_equal(host(lat.get_gauge()), U)
    v = synth.gaussian_half_vector(dims, rng)
    for par in (0, 1):
        assert np.array_equal(host(lat.vec_export(lat.vec_import(dev(v), par), par)), v)
    P = synth.gaussian_momentum(dims, rng)
    assert np.array_equal(host(lat.mom_export(lat.mom_import(dev(P)))), P)


def test_large_lattice_48c12():
    """48^3x12 (V = 1.3M sites, 4x the 32^3x8 volume; z-slab map with 18
    tiles per plane): every output element of D_oe and D_eo."""
    dims = (48, 48, 48, 12)
    log("dslash parity at 48^3x12")
    rng = synth.make_rng(102, 0)
    U = synth.random_su3_near_identity(dims, 0.2, rng)
    lat = lattice(dims, U)
    for out_par in (1, 0):
        vin = synth.gaussian_half_vector(dims, rng)
        x = lat.vec_import(dev(vin), 1 - out_par)
        y = lat.new_vec()
        lat.dslash(y, x, out_par)
        got = host(lat.vec_export(y, out_par))
        exp = dirac.dslash_half(U, vin, dims, out_par)
        assert rel_err(got, exp) < 1e-14


@pytest.mark.parametrize("naik", [False, True])
def test_link_streaming_modes_are_bitwise_equal(naik):
    """Non-temporal and plain link loads give bitwise the same operator, for
    the one-hop and the improved stencil, and a solve with either matches."""
    dims = (8, 6, 4, 10)
    rng = synth.make_rng(103, int(naik))
    U = synth.random_su3_near_identity(dims, 0.4, rng)
    lat = lattice(dims, U)
    if naik:
        lat.set_naik()
    vin = synth.gaussian_half_vector(dims, rng)
    x = lat.vec_import(dev(vin), 0)
    outs = []
    for mode in (0, 2):
        lat.set_link_streaming(mode)
        y = lat.new_vec()
        lat.dslash(y, x, 1)
        xs = [lat.new_vec() for _ in range(3)]
        lat.multishift_solve(0.1, {"c0": 0.0, "pole": [1e-3, 1e-2, 1e-1], "residue": [1.0] * 3}, 1e-10, 10000, x, xs)
        outs.append([host(y)] + [host(v) for v in xs])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
