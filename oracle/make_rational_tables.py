"""Write the rational-approximation tables used as solver inputs.

Run from the repository root:  python -m oracle.make_rational_tables [names...]

Each table is the minimax (n, n) relative approximation of x^p on [lo, hi]
computed by ``oracle.rational.remez`` (paper eq. ratapprx, Appendix) and is
stored as JSON under ``synth/rational/``.  The GPU library only ever receives
the numbers (c0, residues, poles); it never computes them.
"""
from __future__ import annotations

import json
import os
import sys
import time

from oracle.rational import remez

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth", "rational")

# name: (power, lo, hi, n, purpose)
TABLES = {
    # 32^3x8, m = 0.005: 12 poles of x^(-1/4) on [m^2, 64]
    "xm025_n12_m0.005": (-0.25, 0.005 ** 2, 64.0, 12, "32^3x8 multi-shift workload"),
    # 2-flavour RHMC with m = 0.02 on [m^2, 64]: action/force x^(-1/2), heat bath x^(+1/4)
    "xm050_n12_m0.02": (-0.5, 0.02 ** 2, 64.0, 12, "RHMC action and MD force"),
    "xp025_n12_m0.02": (0.25, 0.02 ** 2, 64.0, 12, "RHMC heat bath"),
    # heavier mass for small-lattice trajectory tests (m = 0.1)
    "xm050_n8_m0.1": (-0.5, 0.1 ** 2, 64.0, 8, "small trajectory tests, action/force"),
    "xp025_n8_m0.1": (0.25, 0.1 ** 2, 64.0, 8, "small trajectory tests, heat bath"),
    # higher-accuracy action and heat-bath tables beside the 8-pole MD set
    # (m = 0.1): the accurate tables decide the Metropolis step, the cheaper
    # one drives the molecular dynamics
    "xm050_n16_m0.1": (-0.5, 0.1 ** 2, 64.0, 16, "small trajectory tests, accurate action"),
    "xp025_n16_m0.1": (0.25, 0.1 ** 2, 64.0, 16, "small trajectory tests, accurate heat bath"),
    # accurate action and heat-bath tables for the m = 0.02 RHMC (relative
    # error < 1e-11, the accuracy eq. ratapprx asks of them), beside the
    # 12-pole MD table
    "xm050_n20_m0.02": (-0.5, 0.02 ** 2, 64.0, 20, "RHMC action, accurate"),
    "xp025_n20_m0.02": (0.25, 0.02 ** 2, 64.0, 20, "RHMC heat bath, accurate"),
    # the same three tables on [m^2, 88] for the improved (Naik) operator,
    # whose A is bounded by 4m^2 + (8 (|c1| + |c3|))^2 = 87.1 at (9/8, -1/24)
    "xm050_n12_m0.02_h88": (-0.5, 0.02 ** 2, 88.0, 12, "improved-operator RHMC MD force"),
    "xm050_n20_m0.02_h88": (-0.5, 0.02 ** 2, 88.0, 20, "improved-operator RHMC action, accurate"),
    "xp025_n20_m0.02_h88": (0.25, 0.02 ** 2, 88.0, 20, "improved-operator RHMC heat bath, accurate"),
    # the paper's Appendix example: degree 24/24 for x^(1/4) on [5e-5, 34]
    "xp025_n24_paper": (0.25, 5e-5, 34.0, 24, "paper Appendix example (error < 1e-12)"),
}


def main(names):
    os.makedirs(OUT, exist_ok=True)
    for name in names or TABLES:
        p, lo, hi, n, purpose = TABLES[name]
        t0 = time.time()
        r = remez(p, lo, hi, n)
        d = r.to_json()
        d["name"] = name
        d["purpose"] = purpose
        d["generator"] = "oracle.rational.remez"
        with open(os.path.join(OUT, name + ".json"), "w") as f:
            json.dump(d, f, indent=1)
        print(f"{name}: n={n} error={r.error:.3e} ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
