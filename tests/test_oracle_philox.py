"""Pins for the oracle's Philox4x32-10 and Box-Muller draws."""
import json
import os

import numpy as np

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_known_answer_vectors():
    """Known-answer vectors published with the Random123 library (Salmon et al. 2011)."""
    with open(GOLDEN) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        ctr = np.array([[int(c, 16) for c in v["ctr"]]], dtype=np.uint64)
        key = [int(k, 16) for k in v["key"]]
        out = philox.philox4x32_10(ctr, key)[0]
        assert [int(o) for o in out] == [int(e, 16) for e in v["out"]]


def test_gaussian_moments_and_ranges():
    idx = np.arange(200000, dtype=np.uint64)
    u = philox.uniforms(idx, philox.FIELD_MOMENTUM, 99, 3)
    assert u.min() > 0 and u.max() < 1
    g = philox.gaussians(idx, philox.FIELD_MOMENTUM, 99, 3).reshape(-1)
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1) < 0.01
    assert abs(np.mean(g ** 4) - 3) < 0.05
    xi = philox.source((8, 8, 8, 8), 99, 3)
    assert abs(np.mean(np.abs(xi) ** 2) - 1.0) < 0.02   # e^{-xi^dag xi}: <|xi_c|^2> = 1


def test_streams_distinct():
    a = philox.momentum((2, 2, 2, 2), 1, 0)
    b = philox.momentum((2, 2, 2, 2), 1, 1)
    c = philox.momentum((2, 2, 2, 2), 2, 0)
    assert not np.allclose(a, b) and not np.allclose(a, c)
