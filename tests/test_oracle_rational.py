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
    """Equal-magnitude alternation at the 2n+2 reference points (2n+1 for the
    (n-1, n) type).  The stored coefficients are rounded to double, which
    perturbs r/f by ~1e-14; that absolute floor is added to the tolerance."""
    ref = np.array(r.reference)
    assert len(ref) == 2 * r.n + (1 if r.c0_zero else 2)
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


@pytest.mark.parametrize("power,lo,hi,n", [(-0.5, 4e-4, 64.0, 6), (0.25, 5e-5, 34.0, 6)])
def test_c0_zero_form_and_keeping_c0_halves_the_error(power, lo, hi, n):
    """Appendix: a numerator of degree n-1 sets c_0 = 0, and keeping c_0
    halved the error at the same number of shifts.  The (n-1, n) optimum is
    certified by alternation at 2n+1 points; its error is 1.8-2.3 times the
    (n, n) error for the action power x^(-1/2) on the 16^3x8 RHMC interval and
    for the Appendix's x^(1/4) on [5e-5, 34].  For the negative power every
    pole and residue is positive; for the positive power (a growing function
    that a sum of decaying terms cannot follow alone) one pole lies at a
    negative shift beyond the interval, standing in for the missing constant,
    which a shifted solve of A + d_k cannot take."""
    r0 = remez(power, lo, hi, n, c0_zero=True)
    r = remez(power, lo, hi, n)
    assert r0.c0 == 0.0 and r0.n == n
    _check_alternation(r0, grid=1500, rtol=1e-6)
    assert 1.8 < r0.error / r.error < 2.3, r0.error / r.error
    x = np.geomspace(lo, hi, 400)
    assert np.abs(r0(x) / x ** power - 1).max() <= r0.error * (1 + 1e-6)
    if power < 0:
        assert all(d > 0 for d in r0.pole) and all(c > 0 for c in r0.residue)
    else:
        neg = [d for d in r0.pole if d < 0]
        assert len(neg) == 1 and neg[0] < -hi
        assert all(d > 0 for d in r0.pole if d not in neg)
