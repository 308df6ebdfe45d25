"""GPU observables against the oracle: the Polyakov loop on random fields
(several blocks of spatial sites, 16^3x8) and under the centre
transformation; the stochastic chiral condensate with the same sources."""
import numpy as np
import pytest

import synth
from oracle import fermion, gauge, philox
from paper_1710_09178_amd import stag
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


def test_chiral_condensate_matches_oracle():
    """Same noise vectors (estimator-noise stream (seed, k)), same estimator:
    the GPU mean and standard error agree with the oracle's to the solver
    tolerance."""
    dims, mass, seed, n = (4, 4, 2, 4), 0.1, 5, 8
    log("chiral condensate")
    U = synth.random_su3_near_identity(dims, 0.6, synth.make_rng(711, 0))
    lat = lattice(dims, U)
    mean, err = lat.chiral_condensate(mass, 1e-12, 100000, n, seed)
    etas = [philox.noise(dims, seed, k) for k in range(n)]
    ref, ref_err = fermion.chiral_condensate(U, dims, mass, etas, 1e-12)
    assert abs(mean - ref) < 1e-9 * abs(ref), (mean, ref)
    assert abs(err - ref_err) < 1e-6 * ref_err, (err, ref_err)
    with pytest.raises(stag.StagError):
        lat.chiral_condensate(mass, 1e-12, 100000, 0, seed)
