"""Minimax rational approximation of x^p and its partial fractions
(paper eq. ratapprx; Appendix).

The paper writes (M^dag M)^{1/b} = c_0 + sum_k c_k / (M^dag M + d_k) and obtains
the coefficients from a high-precision minimax approximation of type (n, n)
followed by a partial-fraction split.  Here the same two steps are done in
mpmath:

1. Remez exchange for the best approximation r = P/Q (deg P = deg Q = n) to
   f(x) = x^p on [a, b] in the *relative* sense, i.e. minimising
   max |r(x)/f(x) - 1| (reading: the paper does not say absolute or relative;
   relative is the usual choice for matrix powers and Mathematica's default).
   By the Chebyshev alternation theorem the optimum is unique and its error
   takes the value +-E alternately at 2n+2 points.
2. Poles d_k = -roots(Q) and residues c_k = P(-d_k)/Q'(-d_k), c_0 = lim r(x).
   The paper's listing fits the residues by a linear solve at random points;
   the residue formula gives the same numbers directly.

The x variable is scaled to y = x/b in [a/b, 1] for the linear algebra, the
degree is raised one step at a time from n = 1 (each step seeds its reference
from the previous optimum), and the working precision grows with n log10(b/a).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import mpmath as mp
import numpy as np


@dataclass
class Rational:
    """r(x) = c0 + sum_k residue[k] / (x + pole[k])."""
    power: float
    lo: float
    hi: float
    c0: float
    residue: list
    pole: list
    error: float                      # max relative error on [lo, hi]
    reference: list = field(default_factory=list)  # alternation points
    c0_zero: bool = False             # type (n - 1, n): c0 = 0, 2n + 1 alternation points

    @property
    def n(self) -> int:
        return len(self.pole)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.full_like(x, self.c0)
        for c, d in zip(self.residue, self.pole):
            out = out + c / (x + d)
        return out

    def to_json(self) -> dict:
        return {"power": self.power, "lo": self.lo, "hi": self.hi, "n": self.n,
                "c0": self.c0, "residue": list(self.residue), "pole": list(self.pole),
                "error": self.error, "reference": list(self.reference), "c0_zero": self.c0_zero}

    @staticmethod
    def from_json(d: dict) -> "Rational":
        return Rational(d["power"], d["lo"], d["hi"], d["c0"], list(d["residue"]),
                        list(d["pole"]), d["error"], list(d.get("reference", [])), bool(d.get("c0_zero", False)))


def _horner(coef, y):
    acc = mp.mpf(0)
    for c in reversed(coef):
        acc = acc * y + c
    return acc


class _Remez:
    """Type (nd, n) with nd = n (the paper's form with c_0) or nd = n - 1
    (the Appendix's alternative whose constant term vanishes)."""

    def __init__(self, p, a_scaled, n, nd=None):
        self.p = mp.mpf(p)
        self.a = mp.mpf(a_scaled)
        self.n = n
        self.nd = n if nd is None else nd

    def f(self, y):
        return mp.power(y, self.p)

    def err(self, pc, qc, y):
        return _horner(pc, y) / (_horner(qc, y) * self.f(y)) - 1

    def solve(self, ref):
        """Coefficients (P, Q with Q(0) = 1) and E such that r/f - 1 = (-1)^j E
        on the reference.  Linearised passes (E*Q taken from the previous
        pass) give a starting point close to the wanted root; Newton's method on the full nonlinear
        system P(y_j) - f_j (1 + (-1)^j E) Q(y_j) = 0 then converges quadratically."""
        n, nd = self.n, self.nd
        m = nd + n + 2            # unknowns: nd + 1 of P, n of Q (Q(0) = 1), E
        iq, ie = nd + 1, nd + n + 1   # first Q column, E column
        fj = [self.f(y) for y in ref]
        pw = [[y ** i for i in range(max(n, nd) + 1)] for y in ref]
        sg = [(-1) ** j for j in range(m)]
        qprev = [mp.mpf(1)]
        E_prev = None
        for _ in range(200):
            A = mp.matrix(m, m)
            rhs = mp.matrix(m, 1)
            for j in range(m):
                for i in range(nd + 1):
                    A[j, i] = pw[j][i]
                for i in range(1, n + 1):
                    A[j, iq + i - 1] = -fj[j] * pw[j][i]
                A[j, ie] = -sg[j] * fj[j] * _horner(qprev, ref[j])
                rhs[j] = fj[j]
            sol = mp.lu_solve(A, rhs)
            qprev = [mp.mpf(1)] + [sol[iq + i] for i in range(n)]
            E_new = sol[ie]
            if E_prev is not None and abs(E_new - E_prev) <= mp.mpf(1e-5) * abs(E_new):
                break
            E_prev = E_new
        v = [sol[k] for k in range(m)]
        for _ in range(30):
            pc = v[:nd + 1]
            qc = [mp.mpf(1)] + v[iq:ie]
            E = v[ie]
            J = mp.matrix(m, m)
            F = mp.matrix(m, 1)
            for j in range(m):
                w = fj[j] * (1 + sg[j] * E)
                qv = _horner(qc, ref[j])
                F[j] = _horner(pc, ref[j]) - w * qv
                for i in range(nd + 1):
                    J[j, i] = pw[j][i]
                for i in range(1, n + 1):
                    J[j, iq + i - 1] = -w * pw[j][i]
                J[j, ie] = -sg[j] * fj[j] * qv
            dv = mp.lu_solve(J, F)
            v = [v[k] - dv[k] for k in range(m)]
            if abs(dv[m - 1]) <= abs(v[m - 1]) * mp.mpf(10) ** (-30):
                break
        pc = v[:nd + 1]
        qc = [mp.mpf(1)] + v[iq:ie]
        return pc, qc, v[ie]

    def _zero(self, pc, qc, lo, hi):
        elo = self.err(pc, qc, lo)
        llo, lhi = mp.log(lo), mp.log(hi)
        for _ in range(56):
            mid = (llo + lhi) / 2
            em = self.err(pc, qc, mp.exp(mid))
            if (em > 0) == (elo > 0):
                llo, elo = mid, em
            else:
                lhi = mid
        return mp.exp((llo + lhi) / 2)

    def _argmax(self, pc, qc, lo, hi):
        """Golden-section search for the maximum of |err| on [lo, hi] (log scale),
        compared with the two end points."""
        g = (mp.sqrt(5) - 1) / 2
        a, b = mp.log(lo), mp.log(hi)
        c = b - g * (b - a)
        d = a + g * (b - a)
        fc = abs(self.err(pc, qc, mp.exp(c)))
        fd = abs(self.err(pc, qc, mp.exp(d)))
        for _ in range(48):
            if fc > fd:
                b, d, fd = d, c, fc
                c = b - g * (b - a)
                fc = abs(self.err(pc, qc, mp.exp(c)))
            else:
                a, c, fc = c, d, fd
                d = a + g * (b - a)
                fd = abs(self.err(pc, qc, mp.exp(d)))
        best = mp.exp((a + b) / 2)
        vb = abs(self.err(pc, qc, best))
        for y in (lo, hi):
            v = abs(self.err(pc, qc, y))
            if v > vb:
                best, vb = y, v
        return best, vb

    def exchange(self, pc, qc, ref):
        one = mp.mpf(1)
        zeros = [self._zero(pc, qc, ref[j], ref[j + 1]) for j in range(len(ref) - 1)]
        bounds = [self.a] + zeros + [one]
        new_ref, vals = [], []
        for j in range(len(bounds) - 1):
            y, v = self._argmax(pc, qc, bounds[j], bounds[j + 1])
            new_ref.append(y)
            vals.append(v)
        return new_ref, vals


def _roots_negative_axis(qc, lo, hi, count):
    """The real roots of Q, all on the negative axis, bracketed by sign changes
    of Q(-t) on a fine logarithmic grid in t and refined by bisection."""
    grid_n = 4000
    while True:
        ts = [mp.exp(mp.log(lo) + (mp.log(hi) - mp.log(lo)) * k / grid_n) for k in range(grid_n + 1)]
        vals = [_horner(qc, -t) for t in ts]
        brackets = [(ts[k], ts[k + 1]) for k in range(grid_n) if (vals[k] > 0) != (vals[k + 1] > 0)]
        if len(brackets) == count or grid_n > 64000:
            break
        grid_n *= 4
    if len(brackets) != count:
        raise RuntimeError(f"found {len(brackets)} of {count} poles")
    roots = []
    for t0, t1 in brackets:
        q0 = _horner(qc, -t0)
        for _ in range(mp.mp.prec + 20):
            tm = (t0 + t1) / 2
            qm = _horner(qc, -tm)
            if (qm > 0) == (q0 > 0):
                t0, q0 = tm, qm
            else:
                t1 = tm
        roots.append((t0 + t1) / 2)
    return roots


def remez(power: float, lo: float, hi: float, n: int, rel_tol: float = 1e-8,
          max_iter: int = 60, verbose: bool = False, c0_zero: bool = False) -> Rational:
    """Best relative (n, n) rational approximation to x^power on [lo, hi];
    with c0_zero the best (n - 1, n) one, whose partial fractions have no
    constant term (the alternative of the Appendix, which reports that the
    (n, n) form halves the error at the same number of shifts).  The error
    equioscillates at 2n + 2 points, or 2n + 1 for the (n - 1, n) type."""
    if not (0 < lo < hi):
        raise ValueError("need 0 < lo < hi")
    if n < 1:
        raise ValueError("need n >= 1")
    kappa = hi / lo
    dps = 40 + int(math.ceil(1.3 * n * math.log10(kappa)))
    with mp.workdps(dps):
        a = mp.mpf(lo) / mp.mpf(hi)
        la = mp.log(a)
        ref = None
        for deg in range(1, n + 1):
            ndeg = deg - 1 if c0_zero else deg
            m = ndeg + deg + 2
            if ref is None:
                ref = [mp.exp(la * (1 + mp.cos(mp.pi * j / (m - 1))) / 2) for j in range(m)]
                ref = sorted(ref)
            else:
                # stretch the previous alternation set (2deg points) to 2deg+2 points
                old = [mp.log(y) for y in ref]
                told = np.linspace(0.0, 1.0, len(old))
                tnew = np.linspace(0.0, 1.0, m)
                ref = []
                for t in tnew:
                    k = min(int(np.searchsorted(told, t, side="right")) - 1, len(old) - 2)
                    w = mp.mpf((t - told[k]) / (told[k + 1] - told[k]))
                    ref.append(mp.exp(old[k] + w * (old[k + 1] - old[k])))
                ref[0], ref[-1] = a, mp.mpf(1)
            R = _Remez(power, a, deg, ndeg)
            for it in range(max_iter):
                pc, qc, E = R.solve(ref)
                ref, vals = R.exchange(pc, qc, ref)
                spread = (max(vals) - min(vals)) / max(vals)
                if verbose:
                    print(f"deg {deg} it {it} E={mp.nstr(E, 8)} spread={mp.nstr(spread, 3)}")
                if spread < (rel_tol if deg == n else 1e-3):
                    break
            pc, qc, E = R.solve(ref)
        # partial fractions in the scaled variable, then undo the scaling
        if c0_zero:
            # The (n - 1, n) form of a positive power puts one root of Q on the
            # positive axis beyond the interval (a pole at a negative shift
            # that stands in for the missing constant): take every root of Q
            # (all real) from mpmath's polynomial solver.
            roots = mp.polyroots(list(reversed(qc)), maxsteps=400, extraprec=4 * mp.mp.prec)
            if any(abs(mp.im(z)) > mp.mpf(10) ** (-dps // 2) * abs(z) for z in roots):
                raise RuntimeError("denominator has complex roots")
            poles_y = [-mp.re(z) for z in roots]
        else:
            poles_y = _roots_negative_axis(qc, a * mp.mpf(10) ** -8, mp.mpf(10) ** 8, n)
        dq = [i * qc[i] for i in range(1, n + 1)]
        c0_y = mp.mpf(0) if c0_zero else pc[n] / qc[n]
        res_y = [_horner(pc, -d) / _horner(dq, -d) for d in poles_y]
        scale = mp.mpf(hi)
        pw = mp.mpf(power)
        c0 = c0_y * mp.power(scale, pw)
        residue = [c * mp.power(scale, pw + 1) for c in res_y]
        pole = [d * scale for d in poles_y]
        order = sorted(range(n), key=lambda k: pole[k])
        err = abs(E)
        return Rational(float(power), float(lo), float(hi), float(c0),
                        [float(residue[k]) for k in order], [float(pole[k]) for k in order],
                        float(err), [float(y * scale) for y in ref], c0_zero)


def relative_error(r: Rational, x: np.ndarray, power: float | None = None) -> np.ndarray:
    """r(x)/x^p - 1 evaluated in mpmath (exact enough to see 1e-13 errors)."""
    p = r.power if power is None else power
    out = []
    with mp.workdps(40):
        for xv in np.asarray(x, dtype=np.float64).reshape(-1):
            xm = mp.mpf(xv)
            val = mp.mpf(r.c0) + mp.fsum(mp.mpf(c) / (xm + mp.mpf(d)) for c, d in zip(r.residue, r.pole))
            out.append(float(val / mp.power(xm, p) - 1))
    return np.array(out)
