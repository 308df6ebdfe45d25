"""GPU Polyakov loop against the oracle on random fields (several tiles of
spatial sites, odd extents along x in blocks, 16^3x8) and the centre
transformation on the GPU."""
import numpy as np
import pytest

import synth
from oracle import gauge
from tests.gpu_util import lattice, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,eps", [((4, 4, 2, 4), 0.7), ((6, 4, 4, 8), 1.0), ((16, 16, 16, 8), 0.5),
                                      ((18, 10, 6, 4), 0.8)])
def test_polyakov_loop_matches_oracle(dims, eps):
    log(f"polyakov loop dims={dims}")
    U = synth.random_su3_near_identity(dims, eps, synth.make_rng(710, sum(dims)))
    lat = lattice(dims, U)
    got = lat.polyakov_loop()
    exp = gauge.polyakov_loop(U, dims)
    assert abs(got - exp) < 1e-13, (got, exp)
    # centre transformation of the t = 0 time links: P -> z P
    z = np.exp(2j * np.pi / 3)
    Uz = U.copy()
    Uz[0, ..., 3, :, :] *= z
    lz = lattice(dims, Uz)
    assert abs(lz.polyakov_loop() - z * got) < 1e-13
