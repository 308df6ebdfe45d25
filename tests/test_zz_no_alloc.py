"""The allocation-free operator entry point (stag_mdagm_noalloc) called through
the C ABI against stag_mdagm: bitwise equal results on two calls in a row, the
second on a smaller lattice (both share the static scratch array), no change
of the device's free memory, and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_1710_09178_amd import stag
from tests.gpu_util import dev, host, lattice, log

pytestmark = pytest.mark.gpu


def _call_noalloc(lat, out, inp, mass):
    return lat.lib.stag_mdagm_noalloc(lat.h, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inp.data_ptr()),
                                      ctypes.c_double(mass))


@pytest.mark.parametrize("fmt,naik", [(stag.LINKS_F64_18, False), (stag.LINKS_F64_12, True)])
def test_noalloc_matches_mdagm_on_two_sizes(fmt, naik):
    mass = 0.05
    runs = []
    for dims, seed in [((16, 16, 16, 8), 1), ((8, 6, 4, 10), 2)]:   # the second call is smaller
        log(f"noalloc mdagm dims={dims} fmt={fmt} naik={naik}")
        rng = synth.make_rng(950, seed)
        U = synth.random_su3_near_identity(dims, 0.3, rng)
        lat = lattice(dims, U)
        lat.set_link_format(fmt)
        if naik:
            lat.set_naik()
        x = lat.vec_import(dev(synth.gaussian_half_vector(dims, rng)), 0)
        ref = lat.new_vec()
        lat.mdagm(ref, x, mass)
        torch.cuda.synchronize()
        runs.append((lat, x, ref))
    outs = [torch.full_like(ref, float("nan")) for _, _, ref in runs]   # caller-owned outputs, made first
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (lat, x, ref), out in zip(runs, outs):
        assert _call_noalloc(lat, out, x, mass) == stag.STAG_OK, lat.lib.stag_last_error(lat.h)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for (lat, x, ref), out in zip(runs, outs):
        assert np.array_equal(host(out), host(ref))


def test_noalloc_rejects_lattices_beyond_the_scratch_size():
    dims = (64, 64, 32, 12)   # odd half vector 37.7 MB > 32 MiB
    lat = lattice(dims)
    lat.set_gauge(torch.zeros(lat.field_bytes(stag.FIELD_CANON_GAUGE) // 16, dtype=torch.complex128,
                              device="cuda"))
    v = lat.new_vec()
    w = lat.new_vec()
    assert _call_noalloc(lat, w, v, 0.1) == stag.STAG_ERR_INVALID_ARG
    assert b"scratch" in lat.lib.stag_last_error(lat.h)
