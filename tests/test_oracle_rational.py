"""Pins for the oracle's minimax rational approximation (eq. ratapprx, Appendix).

The Chebyshev alternation theorem certifies optimality: a type (n, n) rational
whose relative error reaches +-E alternately at 2n+2 points and never exceeds E
on the interval is the unique best approximation."""
import glob
import json
import os

import numpy as np
import pytest

import synth
from oracle.rational import Rational, relative_error, remez

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_appendix_rational.json")
TABLES = sorted(glob.glob(os.path.join(os.path.dirname(synth.__file__), "rational", "*.json")))


def _check_alternation(r: Rational, grid=3000, rtol=1e-3):
    """Equal-magnitude alternation at the 2n+2 reference points.  The stored
    coefficients are rounded to double, which perturbs r/f by ~1e-14; that
    absolute floor is added to the tolerance."""
    ref = np.array(r.reference)
    assert len(ref) == 2 * r.n + 2
    e_ref = relative_error(r, ref)
    signs = np.sign(e_ref)
    assert np.all(signs[1:] == -signs[:-1]), "error does not alternate on the reference"
    tol = max(rtol * r.error, 2e-14)
    assert np.all(np.abs(np.abs(e_ref) - r.error) <= tol)
    x = np.geomspace(r.lo, r.hi, grid)
    assert np.abs(relative_error(r, x)).max() <= r.error + tol


@pytest.mark.parametrize("power,lo,hi,n", [(-0.5, 1e-3, 1.0, 4), (0.25, 1e-2, 10.0, 3), (-0.25, 1e-4, 64.0, 5)])
def test_remez_is_minimax(power, lo, hi, n):
    r = remez(power, lo, hi, n)
    _check_alternation(r, grid=1500, rtol=1e-6)
    assert all(d > 0 for d in r.pole)
    if power < 0:
        assert all(c > 0 for c in r.residue) and r.c0 > 0
    # more poles -> smaller error
    assert remez(power, lo, hi, n + 1).error < r.error


def test_partial_fractions_reproduce_ratio():
    """c0 + sum c_k/(x+d_k) equals the optimised P/Q: its error on the
    reference is exactly +-E (checked above) and it matches x^p to E."""
    r = remez(-0.5, 1e-2, 1.0, 3)
    x = np.geomspace(1e-2, 1.0, 50)
    assert np.abs(r(x) / x ** -0.5 - 1).max() <= r.error * (1 + 1e-6)


@pytest.mark.parametrize("path", TABLES, ids=[os.path.basename(t) for t in TABLES])
def test_stored_tables_are_minimax(path):
    with open(path) as f:
        r = Rational.from_json(json.load(f))
    _check_alternation(r, grid=2000 if r.n <= 12 else 1000)
    assert sorted(r.pole) == list(r.pole) and r.pole[0] > 0


def test_paper_appendix_example():
    """The paper's Appendix: degree 24/24 for x^(1/4) on [5e-5, 34] gives an
    error below 1e-12; the interval covers the spectrum [(2ma)^2, ...] for ma=0.005."""
    with open(GOLDEN) as f:
        g = json.load(f)
    with open(os.path.join(os.path.dirname(synth.__file__), "rational", "xp025_n24_paper.json")) as f:
        r = Rational.from_json(json.load(f))
    assert (r.power, r.lo, r.hi, r.n) == (g["power"], g["lo"], g["hi"], g["degree"])
    assert r.error < g["max_error_below"]
    assert g["lo"] < (2 * g["ma"]) ** 2 and g["hi"] > 32
    x = np.geomspace(r.lo, r.hi, 800)
    assert np.abs(relative_error(r, x)).max() < g["max_error_below"]
