"""The Python binding checks every buffer's size and dtype before it calls the
C ABI (which takes raw pointers, so a wrong buffer would make a kernel read or
write outside it).  The library is replaced by a recorder: no GPU is needed,
and a rejected call must never reach it."""
import ctypes

import pytest
import torch

from paper_1710_09178_amd import stag


class _Recorder:
    """Stands in for the loaded library: every attribute is a function that
    records its call and returns STAG_OK."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def fn(*args):
            self.calls.append(name)
            return 0
        return fn


def _lattice(dims=(4, 4, 4, 4)):
    lat = object.__new__(stag.Lattice)
    lat.lib = _Recorder()
    lat.dims = dims
    V = dims[0] * dims[1] * dims[2] * dims[3]
    lat.V, lat.Vh = V, V // 2
    lat.h = ctypes.c_void_p(0)
    # the library's sizes: internal vec 48 B/site, mom 64 B/link, canonical as in stag.h
    lat._nb = {stag.FIELD_HALF_VEC: 48 * lat.Vh, stag.FIELD_MOM: 64 * 4 * V,
               stag.FIELD_CANON_HALF_VEC: 48 * lat.Vh, stag.FIELD_CANON_GAUGE: 144 * 4 * V,
               stag.FIELD_CANON_MOM: 64 * 4 * V}
    return lat


def test_wrong_sizes_and_dtypes_never_reach_the_library():
    lat = _lattice()
    vh, V = lat.Vh, lat.V
    short_vec = torch.zeros(6 * vh - 2, dtype=torch.float64)
    mom_sized = torch.zeros(32 * V, dtype=torch.float64)
    vec_f32 = torch.zeros(12 * vh, dtype=torch.float32)
    cases = [
        lambda: lat.dslash(short_vec, short_vec, 1),
        lambda: lat.mdagm(vec_f32, vec_f32, 0.1),
        lambda: lat.dslash(mom_sized, mom_sized, 1),           # a momentum field where a vector belongs
        lambda: lat.set_gauge(torch.zeros((V, 4, 3, 3), dtype=torch.complex64)),
        lambda: lat.set_gauge(torch.zeros((V, 4, 3, 2), dtype=torch.complex128)),
        lambda: lat.gauge_force(5.4, short_vec, 0.0),
        lambda: lat.kinetic_energy(short_vec),
        lambda: lat.link_update(torch.zeros(32 * V - 1, dtype=torch.float64), 0.1),
        lambda: lat.fermion_force(0.1, {"pole": [1.0], "residue": [1.0]}, 1e-10, 10, short_vec, mom_sized),
        lambda: lat.multishift_solve(0.1, {"pole": [1.0, 2.0], "residue": [1.0, 1.0]}, 1e-10, 10,
                                     short_vec, None),
        lambda: lat.trajectory(5.4, 0.1, 1.0, 4, {"pole": [1.0], "residue": [1.0]},
                               {"pole": [1.0], "residue": [1.0]}, {"pole": [1.0], "residue": [1.0]},
                               inject_mom=short_vec),
    ]
    for i, f in enumerate(cases):
        with pytest.raises((ValueError, TypeError)):
            f()
        assert lat.lib.calls == [], f"case {i} reached the library"


def test_solution_list_must_match_the_pole_count():
    lat = _lattice()
    vec = torch.zeros(6 * lat.Vh, dtype=torch.float64)
    with pytest.raises(ValueError, match="expected 2 solution vectors"):
        lat.multishift_solve(0.1, {"pole": [1.0, 2.0], "residue": [1.0, 1.0]}, 1e-10, 10, vec, [vec])
    assert lat.lib.calls == []


def test_right_sizes_pass_the_checks_up_to_the_device_test():
    # host tensors of the right size and dtype get as far as the device check
    lat = _lattice()
    vec = torch.zeros(6 * lat.Vh, dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):
        lat.dslash(vec, vec.clone(), 1)
    cvec = torch.zeros(3 * lat.Vh, dtype=torch.complex128)
    with pytest.raises(ValueError, match="device"):
        lat.mdagm(cvec, cvec.clone(), 0.1)
    assert lat.lib.calls == []


def test_batch_masses_and_instance_are_checked():
    b = object.__new__(stag.Batch)
    b.lib = _Recorder()
    b.dims = [(4, 4, 4, 4), (6, 4, 4, 4)]
    b.nrhs = 1
    b.vh = [128, 192]
    b.h = ctypes.c_void_p(0)
    with pytest.raises(ValueError, match="inst"):
        b.set_gauge(2, torch.zeros(1, dtype=torch.complex128))
    with pytest.raises(ValueError, match="bytes"):
        b.set_gauge(1, torch.zeros((256, 4, 3, 3), dtype=torch.complex128))
    assert b.lib.calls == []


def test_trajectory_log_appends_one_json_line_per_trajectory(tmp_path):
    """The per-trajectory log: one JSON object per call with the info fields
    and the trajectory's parameters (library replaced by the recorder, so
    the info is all zeros)."""
    import io
    import json
    lat = _lattice()
    rat = {"c0": 0.1, "residue": [0.5, 0.25], "pole": [0.01, 1.0]}
    path = tmp_path / "chain.jsonl"
    for t in range(2):
        out = lat.trajectory(5.4, 0.02, 1.0, 20, rat, rat, rat, seed=7, traj_index=t, log=str(path))
    buf = io.StringIO()
    lat.trajectory(5.4, 0.02, 1.0, 20, rat, rat, rat, seed=7, traj_index=2, log=buf)
    lines = path.read_text().splitlines() + buf.getvalue().splitlines()
    assert lat.lib.calls.count("stag_md_trajectory") == 3
    recs = [json.loads(x) for x in lines]
    assert [r["traj_index"] for r in recs] == [0, 1, 2]
    for r in recs:
        assert set(out) <= set(r)
        assert (r["seed"], r["beta"], r["mass"], r["tau"], r["n_steps"]) == (7, 5.4, 0.02, 1.0, 20)
        assert r["model"] is False and r["accepted"] == 0
