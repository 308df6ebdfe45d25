"""The oracle's spectral range of A against what the mathematics fixes: the
free-field spectrum in closed form, the dense matrix's eigenvalues (brute
force, built entry by entry from the Dirac operator's definition), the
Rayleigh bound, and the interval rule of the paper's Appendix."""
import numpy as np

import synth
from oracle import dirac, lattice as L, philox, spectrum


def _dense_A_from_D(U, dims, mass):
    """4m^2 - D_eo D_oe from the dense hopping matrix (no use of apply_A)."""
    D = dirac.dense_dslash(U, dims)
    par = L.parity(dims).reshape(-1)
    ev = np.repeat(par == 0, 3)
    od = ~ev
    D_eo = D[np.ix_(ev, od)]
    D_oe = D[np.ix_(od, ev)]
    return 4 * mass * mass * np.eye(ev.sum()) - D_eo @ D_oe


def test_free_field_top_eigenvalue():
    """U = 1 on 4^4 with antiperiodic t: A e^{ipx} = (4m^2 + 4 sum sin^2 p) e^{ipx},
    the largest value 4m^2 + 4 (3 + 1/2) = 14.04 at m = 0.1 (p_i = pi/2 in space,
    p_t = pi/4 in time); the power iteration from a Gaussian vector reaches it."""
    dims = (4, 4, 4, 4)
    U = np.broadcast_to(np.eye(3, dtype=complex), (4, 4, 4, 4, 4, 3, 3)).copy()
    lam = spectrum.power_rayleigh(U, dims, 0.1, philox.noise(dims, 1, 0), 200)
    assert abs(lam - 14.04) < 1e-12


def test_power_estimate_against_dense_eigenvalues():
    dims, mass = (2, 2, 2, 4), 0.05
    U = synth.random_su3_near_identity(dims, 0.9, synth.make_rng(730, 0))
    evals = np.linalg.eigvalsh(_dense_A_from_D(U, dims, mass))
    lam_max = evals.max()
    assert evals.min() >= 4 * mass * mass - 1e-12           # A = 4m^2 + D_oe^dag D_oe
    assert lam_max <= 4 * mass * mass + 64 + 1e-12           # |D_oe| <= 8
    v0 = philox.noise(dims, 2, 0)
    prev = 0.0
    for k in (1, 10, 100, 3000):
        lam = spectrum.power_rayleigh(U, dims, mass, v0, k)
        assert lam <= lam_max * (1 + 1e-12)                  # Rayleigh quotient bound
        assert lam >= prev - 1e-12 * lam_max                 # rises with k
        prev = lam
    assert lam > lam_max * (1 - 1e-6)


def test_interval_rule():
    m = 0.02
    lo = 4 * m * m
    assert spectrum.interval_covers(m, lo, 64.0, 20.0, 0.1)
    assert not spectrum.interval_covers(m, 1.5 * lo, 64.0, 20.0, 0.1)        # misses the bottom
    assert not spectrum.interval_covers(m, lo, 21.0, 20.0, 0.1)              # too close to the estimate
    assert spectrum.interval_covers(m, lo, lo + 64.0, 1e9, 0.1)              # certain bound reached
