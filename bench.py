"""Benchmark: FP64 multi-shift CG with the staggered Dslash at 32^3x8.

One step = one complete multi-shift solve of (A + pole_k) x_k = b for the 12
poles of the minimax x^(-1/4) approximation on [m^2, 64], m = 0.005,
tolerance 1e-10, with all 12 solutions written out.  Inputs (links
exp(i 0.2 H) projected to SU(3), Gaussian source) are synthetic, seeded, and
resident in HBM before timing starts.

value    = algorithmic HBM bytes of the whole solve / wall time of the solve
           (GB/s; bytes counted per kernel from the data each one must move).
roofline = the D_oe Dslash kernel inside the solve: 1248 algorithmic bytes per
           output site / its average launch duration (hipEvents around every
           launch of one extra profiled solve), against 8 TB/s.
Also reported: the other solver kernels, iterations, true residuals, the
precision forms (12-real FP64 links; mixed FP32/FP64 with FP32-18 or FP16-12
links), the batched form (64 lattices x 4 right-hand sides), the seconds per
thermalised RHMC trajectory at 16^3x8, and RHMC with and without the learned
force model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 8)
MASS = 0.005
TOL = 1e-10
TABLE = "xm025_n12_m0.005"
# algorithmic bytes per output site (FP64, 18-real links)
B_DOE = 1248            # 8 links x 144 B + in 48 B + out 48 B
B_DEO_CG = 1344         # D_eo 1248 + read p and r (96) for the fused mass term and dots
B_UPD_FIXED = 336       # r (rw) 96, Ap 48, p (rw) 96, x_base (rw) 96
B_UPD_SHIFT = 192       # per active shifted system: x_k and p_k read and written


class no_gc:
    """Python's cyclic garbage collector off inside a timed region (collected
    just before): a full collection in this process takes ~40 ms and would
    otherwise land in a random timed step.  The GPU work is unchanged."""

    def __enter__(self):
        import gc
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        import gc
        gc.enable()
        return False


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# fused loop: D_oe launch j also forms p_j from r_{j-1}, Ap_{j-1}, p_{j-1}
# (read once each) and writes r_j and p_j (x_base read and written while the
# base system is active); the first launch reads p_0 and r_0 = b
B_FUSED_DOE = 1152 + 3 * 48 + 48 + 2 * 48     # links, r/Ap/p in, w out, r and p out
B_FUSED_DOE_FIRST = 1152 + 48 + 48 + 48       # links, p_0 in, w out, r_0 read for |r_0|^2


def fused_solve_bytes(vh, iters, ipp, base, lag):
    """Algorithmic bytes of one solve in the fused loop that stops at step
    S = iters: iteration 0 (first D_oe + D_eo), iterations 1..S (fused D_oe
    + D_eo), S // lag window flushes and the final partial flush; each flush
    reads its window's residuals once and every shifted system active at the
    window's start (x_k, p_k read and written)."""
    def shifts_from(j0):
        return sum(1 for k, f in enumerate(ipp) if k != base and f > j0)
    total = (B_FUSED_DOE_FIRST + B_DEO_CG) * vh
    for j in range(1, iters + 1):
        total += (B_FUSED_DOE + (96 if ipp[base] > j - 1 else 0) + B_DEO_CG) * vh
    for w0 in range(0, iters, lag):
        npend = min(lag, iters - w0)
        total += (48 * npend + B_UPD_SHIFT * shifts_from(w0)) * vh
    return total


def flush_bytes(vh, iters, ipp, base, lag):
    def shifts_from(j0):
        return sum(1 for k, f in enumerate(ipp) if k != base and f > j0)
    return sum((48 * lag + B_UPD_SHIFT * shifts_from(w0)) * vh for w0 in range(0, iters - lag + 1, lag))


def solve_bytes(vh, iters, ipp, base, lag=1, fused=False):
    """Algorithmic bytes of one solve from the per-pole freeze iterations
    (shift k is active in iterations j < ipp[k]).  The shifted solutions and
    directions are read and written once per window of `lag` iterations, and
    the window's residuals are read back once (two of them are in registers)."""
    if fused:
        return fused_solve_bytes(vh, iters, ipp, base, lag)

    def shifts_from(j0):
        return sum(1 for k, f in enumerate(ipp) if k != base and f > j0)
    total = 0
    for j in range(iters):
        upd = B_UPD_FIXED - (0 if ipp[base] > j else 96)
        if j % lag == lag - 1:
            upd += max(0, lag - 2) * 48 + B_UPD_SHIFT * shifts_from(j - j % lag)
        total += (B_DOE + B_DEO_CG + upd) * vh
    slot = iters % lag
    if slot:  # the stopping launch applies the pending part of the last window
        total += (48 * slot + B_UPD_SHIFT * shifts_from(iters - slot)) * vh
    return total


def cpu_baseline(U, b, rat, vh, lag, target_s=20.0):
    """Time the CPU oracle's multi-shift CG on the same workload for a bounded
    number of iterations and express it in the same unit (GB/s of algorithmic
    solver traffic)."""
    import numpy as np
    from oracle import dirac
    from oracle.solvers import multishift_cg
    op = lambda v: dirac.apply_A(U, v, DIMS, MASS)
    t0 = time.perf_counter()
    multishift_cg(op, b, rat["pole"], 1e-30, maxiter=1)
    one = time.perf_counter() - t0
    iters = max(2, int(target_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    multishift_cg(op, b, rat["pole"], 1e-30, maxiter=iters)
    dt = time.perf_counter() - t0
    # the same bytes per iteration as the GPU solve with every pole active
    n = len(rat["pole"])
    per_iter = solve_bytes(vh, 8 * lag, [10 ** 9] * n, 0, lag) / (8 * lag)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": per_iter * iters / dt / 1e9, "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} multi-shift CG iterations of the same 32^3x8 12-pole solve (all shifts active), "
                      f"{dt:.1f} s; numpy element-wise code runs on one core ({cores} available)",
            "seconds": dt, "iterations": iters}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "dslash_oe_fp64_32c3x8_hbm_traffic.md")
DSLASH_SOURCES = ["paper_1710_09178_amd/csrc/dslash.hip", "paper_1710_09178_amd/csrc/dslash.h",
                  "paper_1710_09178_amd/csrc/common.h", "paper_1710_09178_amd/csrc/msfused.h"]


def measured_traffic(fused=True):
    """Bytes per D_oe launch (FETCH_SIZE + WRITE_SIZE, calibrated; L2-to-fabric
    requests, which include Infinity-Cache hits) from the committed summary
    of the same loop, or None once the Dslash sources differ from the ones
    profiled."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        h = hashlib.sha256()
        for f in DSLASH_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    import re
    t = re.search(r"traffic_bytes_per_launch %s (\d+)" % ("dslash_oe_fused" if fused else "dslash_oe"), text)
    src = re.search(r"dslash_sources_sha256 ([0-9a-f]{64})", text)
    if not t or not src or src.group(1) != h.hexdigest():
        return None
    return float(t.group(1))


def _short(name: str) -> str:
    import re
    n = name.replace("stag::(anonymous namespace)::", "").replace("HIP_vector_type<double, 2u>", "double2")
    n = n.replace("HIP_vector_type<float, 2u>", "float2")
    m = re.match(r"(void )?([^(]*)", n)
    return m.group(2).strip()


def summarize_trace(path):
    """Per-kernel summary of a rocprofv3 kernel_trace.csv: all launches, and the
    launches that did the full work.  Once a solve has converged, the launches
    still queued behind it return early (1-5 us); a launch counts as full when
    it takes at least half the median of the kernel's longer half."""
    import csv
    from collections import defaultdict
    d = defaultdict(list)
    spans = []
    for row in csv.DictReader(open(path)):
        s0, s1 = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
        d[_short(row["Kernel_Name"])].append((s1 - s0) / 1e3)
        spans.append((s0, s1))
    # share of the traced span with a kernel running, and the mean idle gap
    spans.sort()
    busy, end = 0, spans[0][0] if spans else 0
    for s0, s1 in spans:
        busy += max(0, s1 - max(s0, end))
        end = max(end, s1)
    wall = (end - spans[0][0]) if spans else 0
    lines = [f"traced span {wall / 1e6:.2f} ms, kernels running {100.0 * busy / max(wall, 1):.1f}% of it, "
             f"{len(spans)} launches, mean gap {(wall - busy) / max(len(spans), 1) / 1e3:.2f} us",
             f"{'kernel':70s} {'launches':>8s} {'worked':>7s} {'avg_us(all)':>11s} {'avg_us(worked)':>14s} "
             f"{'min_us':>8s} {'max_us':>8s}"]
    for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        top = sorted(v)[len(v) // 2:]
        cut = 0.5 * top[len(top) // 2]
        w = [t for t in v if t >= cut]
        lines.append(f"{k[:70]:70s} {len(v):8d} {len(w):7d} {sum(v) / len(v):11.3f} "
                     f"{(sum(w) / len(w) if w else 0):14.3f} {min(v):8.3f} {max(v):8.3f}")
    return "\n".join(lines), d


def summarize_pmc(path, counter, copy_bytes):
    """Per-kernel average of a rocprofv3 --pmc counter (KiB per dispatch) and
    the scale factor that maps the counter onto the known bytes of the plain
    copy kernel run in --pmc-mode."""
    import csv
    from collections import defaultdict
    d = defaultdict(list)
    for row in csv.DictReader(open(path)):
        if row.get("Counter_Name", counter) != counter:
            continue
        d[_short(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return d


def pmc_mode():
    """One FP64 solve of the benchmark workload and a plain 512 MiB device copy
    (the calibration kernel for the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice
    torch.cuda.set_device(0)
    U = synth.random_su3_near_identity(DIMS, 0.2, synth.make_rng(1, 0))
    b = synth.gaussian_half_vector(DIMS, synth.make_rng(1, 1))
    rat = synth.load_rational(TABLE)
    lat = Lattice(DIMS)
    lat.set_gauge(torch.from_numpy(U).cuda())
    bd = lat.vec_import(torch.from_numpy(b).cuda(), 0)
    xs = [lat.new_vec() for _ in rat["pole"]]
    info = lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
    src = torch.ones(512 * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_mode": True, "iters": info["iters"], "copy_bytes": 512 * 2 ** 20}), flush=True)


def force_channel_probe(n_samples=6):
    """How much of the truncated-solve force error could covariant channels
    built from truncated solves remove?  The thermalised 16^3x8 RHMC
    configuration (as in rhmc()); for n_samples pseudofermions (one RHMC
    trajectory apart): the exact force F, the forces of solves stopped after
    100, 150 and 200 iterations, and of the 200-iteration solve split into the
    4 lightest and the 8 heavier poles; the share of the 200-iteration error
    carried by the light poles; and global least-squares combinations of
    these channels fitted on half of the samples and evaluated on the other
    half (relative errors |F_fit - F| / |F|)."""
    import numpy as np
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice
    torch.cuda.set_device(0)
    dims = (16, 16, 16, 8)
    beta, mass = 5.4, 0.02
    r_f = synth.load_rational("xm050_n12_m0.02")
    r_a = synth.load_rational("xm050_n20_m0.02")
    r_h = synth.load_rational("xp025_n20_m0.02")
    lat = Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.haar_su3(dims, synth.make_rng(5, 0))).cuda())
    kw = dict(tol_md=1e-8, tol_action=1e-10, seed=11)
    t = 0
    for _ in range(60):
        lat.trajectory(beta, mass, 0.5, 20, r_f, r_a, r_h, no_fermions=True, inject_u=0.0, traj_index=t, **kw)
        t += 1
    for _ in range(5):
        lat.trajectory(beta, mass, 1.0, 20, r_f, r_a, r_h, inject_u=0.0, traj_index=t, **kw)
        t += 1
    order = list(np.argsort(r_f["pole"]))

    def sub(idx):
        return {"c0": 0.0, "pole": [r_f["pole"][i] for i in idx], "residue": [r_f["residue"][i] for i in idx]}

    samples = []
    for j in range(n_samples):
        xs = [lat.new_vec() for _ in r_h["pole"]]
        phi = lat.new_vec()
        lat.multishift_solve(mass, r_h, 1e-10, 100000, lat.random_source(99, 100000 + j), xs, phi, true_resid=False)

        def force(rat, tol, maxiter):
            m = lat.new_mom()
            lat.fermion_force(mass, rat, tol, maxiter, phi, m, 0.0, allow_not_converged=True)
            return lat.mom_export(m).cpu().numpy().reshape(-1)
        samples.append({"F": force(r_f, 1e-10, 100000), "T200": force(r_f, 1e-30, 200),
                        "T150": force(r_f, 1e-30, 150), "T100": force(r_f, 1e-30, 100),
                        "L200": force(sub(order[:4]), 1e-30, 200), "H200": force(sub(order[4:]), 1e-30, 200),
                        "Lex": force(sub(order[:4]), 1e-10, 100000)})
        lat.trajectory(beta, mass, 1.0, 20, r_f, r_a, r_h, inject_u=0.0, traj_index=t, **kw)
        t += 1
        log(f"sample {j}")

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    half = n_samples // 2
    out = {"force_channel_probe": True,
           "truncated_200_rel_error": [round(rel(s["T200"], s["F"]), 5) for s in samples],
           "truncated_100_rel_error": [round(rel(s["T100"], s["F"]), 5) for s in samples],
           "light_poles_share_of_truncation_error": [
               round(float(np.linalg.norm(s["L200"] - s["Lex"]) / np.linalg.norm(s["T200"] - s["F"])), 6)
               for s in samples]}
    for name, cols in {"T200": ["T200"], "L200+H200": ["L200", "H200"], "T200+T100": ["T200", "T100"],
                       "T200+T150+T100": ["T200", "T150", "T100"]}.items():
        A = np.concatenate([np.stack([s[c] for c in cols], 1) for s in samples[:half]])
        y = np.concatenate([s["F"] for s in samples[:half]])
        coef = np.linalg.lstsq(A, y, rcond=None)[0]
        out["fit_" + name] = {"coefficients": [round(float(c), 5) for c in coef],
                              "held_out_rel_error": [round(rel(np.stack([s[c] for c in cols], 1) @ coef, s["F"]), 5)
                                                     for s in samples[half:]]}
    print(json.dumps(out), flush=True)


def surrogate_trace_mode(n_pairs=64, epochs=4):
    """The learned force model's kernels at 16^3x8 (131,072 links), for a
    kernel trace: n_pairs stored (gauge field, force) pairs with the
    auxiliary channel (random force fields stand in for the targets: the
    kernels' work does not depend on the values), `epochs` training epochs
    (one forward, backward and Adam step per pair), one evaluation with
    gradients and 20 applications of the model to a momentum field."""
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice, Surrogate
    torch.cuda.set_device(0)
    dims = (16, 16, 16, 8)
    lat = Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.random_su3_near_identity(dims, 0.5, synth.make_rng(6, 0))).cuda())
    sur = Surrogate(lat, n_pairs, seed=1)
    aux = lat.random_momentum(7, 0)
    sur.set_aux(aux)
    for k in range(n_pairs):
        sur.add_pair(lat.random_momentum(7, 1 + k))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = sur.train(epochs, 1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sur.eval(lat.random_momentum(7, 10 ** 6), want_grad=True)
    mom = lat.new_mom()
    t0 = time.perf_counter()
    for _ in range(20):
        sur.force(mom, 0.05)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t0) / 20
    print(json.dumps({"surrogate_trace_mode": True, "links": lat.V * 4, "pairs": n_pairs, "epochs": epochs,
                      "train_s": round(t_train, 4), "us_per_pair_step": round(1e6 * t_train / (n_pairs * epochs), 2),
                      "apply_us": round(1e6 * t_apply, 2), "loss": loss}), flush=True)


def trajectory_trace_mode(n_traj=3, improved=False):
    """A few RHMC trajectories at 16^3x8 (beta 5.4, m 0.02, the 12-pole MD
    table with 20-pole action and heat-bath tables, tau 1, 20 steps) from a near-identity start, after one untimed one: a
    short program for a kernel trace of the trajectory's launches.  improved:
    the Naik-improved operator with the tables on [m^2, 88]."""
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice
    torch.cuda.set_device(0)
    dims = (16, 16, 16, 8)
    lat = Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.random_su3_near_identity(dims, 0.5, synth.make_rng(5, 0))).cuda())
    suffix = "_h88" if improved else ""
    if improved:
        lat.set_naik(9.0 / 8.0, -1.0 / 24.0)
    r_f = synth.load_rational("xm050_n12_m0.02" + suffix)
    r_a = synth.load_rational("xm050_n20_m0.02" + suffix)
    r_h = synth.load_rational("xp025_n20_m0.02" + suffix)
    kw = dict(tol_md=1e-8, tol_action=1e-10, seed=11)
    lat.trajectory(5.4, 0.02, 1.0, 20, r_f, r_a, r_h, inject_u=0.0, traj_index=0, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [lat.trajectory(5.4, 0.02, 1.0, 20, r_f, r_a, r_h, inject_u=0.0, traj_index=1 + i, **kw)
           for i in range(n_traj)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n_traj
    print(json.dumps({"trajectory_trace_mode": True, "improved": improved, "sec_per_traj": round(dt, 4),
                      "cg_iters": [r["cg_iters_total"] for r in res]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tps", type=int, default=0, help="Dslash threads per site (0 = library default)")
    ap.add_argument("--lag", type=int, default=8, help="shift-update window of the solver (1..8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trajectory", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-naik", action="store_true")
    ap.add_argument("--no-memory-check", action="store_true")
    ap.add_argument("--no-fused", action="store_true", help="three launches per CG iteration instead of two")
    ap.add_argument("--c1-hot", action="store_true", help="also the 32^3x8 solve on Haar links (long solves)")
    ap.add_argument("--learned-long", action="store_true",
                    help="learned-force chains at 20 leapfrog steps (exact, and exact every 4th kick with the "
                         "truncated solve or the model between); use with --chain-traj 400")
    ap.add_argument("--chain-traj", type=int, default=24, help="trajectories per learned-force comparison chain")
    ap.add_argument("--improved-traj", type=int, default=10,
                    help="timed trajectories of the improved-operator chain")
    ap.add_argument("--inner-iters", type=int, default=200,
                    help="iterations of the truncated solve that feeds the learned model's auxiliary channel")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--pmc-mode", action="store_true", help="one solve + a 512 MiB copy, for counter runs")
    ap.add_argument("--trajectory-trace-mode", action="store_true",
                    help="a few 16^3x8 RHMC trajectories, for a kernel trace")
    ap.add_argument("--improved", action="store_true",
                    help="with --trajectory-trace-mode: the Naik-improved operator")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV")
    ap.add_argument("--surrogate-trace-mode", action="store_true",
                    help="the learned model's kernels at 16^3x8, for a kernel trace")
    ap.add_argument("--force-channel-probe", action="store_true",
                    help="truncated-solve force channels against the exact force at 16^3x8 (one JSON line)")
    args = ap.parse_args()
    if args.summarize_trace:
        text, _ = summarize_trace(args.summarize_trace)
        print(text)
        return
    if args.trajectory_trace_mode:
        trajectory_trace_mode(improved=args.improved)
        return
    if args.force_channel_probe:
        force_channel_probe()
        return
    if args.surrogate_trace_mode:
        surrogate_trace_mode()
        return
    if args.pmc_mode:
        pmc_mode()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (one process, one device).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice

    torch.cuda.set_device(0)
    rng = synth.make_rng(1, 0)
    U = synth.random_su3_near_identity(DIMS, 0.2, rng)
    b = synth.gaussian_half_vector(DIMS, synth.make_rng(1, 1))
    rat = synth.load_rational(TABLE)
    n = len(rat["pole"])
    base = int(np.argmin(rat["pole"]))
    lat = Lattice(DIMS)
    if args.tps:
        lat.tune(args.tps, 16)
    lat.set_shift_window(args.lag)
    # the library's default loop choice: fused on Dslash grids of <= 512
    # blocks of 64 sites, so three launches per iteration at 32^3x8
    fused = not args.no_fused and args.lag >= 2 and (vh_of(DIMS) + 63) // 64 <= 512
    lat.set_fused_iteration(1 if not args.no_fused else 0)
    lat.set_gauge(torch.from_numpy(U).cuda())
    bd = lat.vec_import(torch.from_numpy(b).cuda(), 0)
    xs = [lat.new_vec() for _ in range(n)]
    vh = lat.Vh

    def step(resid=False):
        return lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=resid)

    log(f"warmup {args.warmup} solves")
    info = None
    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} solves")
    with no_gc():
        t0 = time.perf_counter()
        infos, step_ms = [], []
        for _ in range(args.steps):
            ts = time.perf_counter()
            infos.append(step())      # returns after the solve has finished (host-side info)
            step_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    bytes_total = sum(solve_bytes(vh, i["iters"], i["iters_per_pole"], base, args.lag, fused) for i in infos)
    value = bytes_total / elapsed / 1e9

    # one more solve: true residuals, and hipEvents around every kernel launch
    log("profiled solve")
    lat.profile_enable(3 * (infos[0]["iters"] + 64))
    chk = step(resid=True)
    ms, cnt = lat.profile_read()
    doe_samples = lat.profile_samples(0)
    lat.profile_enable(0)
    avg_us = [1e3 * ms[i] / max(cnt[i], 1) for i in range(3)]
    ipp_c = chk["iters_per_pole"]
    if fused:
        # D_oe with the folded base update: its bytes averaged over its launches
        b_doe = (B_FUSED_DOE * cnt[0] + 96 * sum(1 for j in range(1, cnt[0] + 1) if ipp_c[base] > j - 1)) \
            / max(cnt[0], 1)
        upd_bytes = flush_bytes(vh, chk["iters"], ipp_c, base, args.lag)
    else:
        b_doe = B_DOE
        upd_bytes = solve_bytes(vh, chk["iters"], ipp_c, base, args.lag) - (B_DOE + B_DEO_CG) * vh * chk["iters"]
    doe_gbs = b_doe * vh / (avg_us[0] * 1e-6) / 1e9
    deo_gbs = B_DEO_CG * vh / (avg_us[1] * 1e-6) / 1e9
    upd_gbs = upd_bytes / max(cnt[2], 1) / (avg_us[2] * 1e-6) / 1e9

    forms = {}
    if not args.no_forms:
        log("precision forms")
        forms = precision_forms(lat, rat, bd, xs, vh, base, ms_per_step)

    hot = None
    if args.c1_hot:
        log("32^3x8 on Haar links")
        hot = c1_hot()

    memory = None
    if not args.no_memory_check:
        log("memory check: stream ceilings, isolated D_oe after a read sweep, 48^3x16 solve")
        memory = memory_check(lat, bd, vh)

    improved = None
    if not args.no_naik:
        log("Naik-improved operator")
        improved = improved_operator(lat, rat, bd, xs, vh)

    batched = None
    if not args.no_batch:
        log("batched form")
        batched = batched_form()

    rh = None
    if not args.no_trajectory:
        log("RHMC at 16^3x8" + ("" if args.no_surrogate else " with and without the learned force model"))
        if args.learned_long:
            # the workload's 20 leapfrog steps, long chains: exact force, and the
            # exact force on every 4th kick with the truncated solve or the model between
            rh = rhmc(with_model=True, n_traj=args.chain_traj, inner_iters=args.inner_iters, chain_steps=20,
                      n_improved=args.improved_traj,
                      every_list=(4,), ablation=False)
        else:
            rh = rhmc(with_model=not args.no_surrogate, n_traj=args.chain_traj, inner_iters=args.inner_iters,
                      n_improved=args.improved_traj)

    out = {
        "metric": "multishift-CG Dslash GB/s (% HBM peak) at 32^3x8; sec/RHMC trajectory",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64 multi-shift CG, staggered even-odd operator, 32^3x8, 12 poles of x^(-1/4), "
                               "m=0.005, tol=1e-10",
                   "lattice": list(DIMS), "poles": n, "mass": MASS, "tol": TOL, "links": "exp(i 0.2 H) in SU(3)"},
        "roofline": {"bound": "hbm",
                     "kernel": ("D_oe Dslash with the folded base-system update (fused CG iteration)" if fused
                                else "D_oe Dslash (in the multi-shift CG)"),
                     "achieved": round(doe_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(doe_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(fused),
                     "avg_launch_us": round(avg_us[0], 3), "algorithmic_bytes_per_launch": round(b_doe * vh)},
        "fused_iteration": fused,
        "kernels": {"dslash_oe" + ("_fused" if fused else ""): {"avg_us": round(avg_us[0], 3),
                                                                 "GB/s": round(doe_gbs, 1), "launches": cnt[0],
                                                                 "bytes_per_site": round(b_doe, 1)},
                    "dslash_eo_cg": {"avg_us": round(avg_us[1], 3), "GB/s": round(deo_gbs, 1), "launches": cnt[1]},
                    ("window_flush" if fused else "shift_update"): {"avg_us": round(avg_us[2], 3),
                                                                     "GB/s": round(upd_gbs, 1),
                                                                     "launches": cnt[2]}},
        "ms_per_step_pct": _pct(step_ms),
        "dslash_oe_us_pct": _pct(doe_samples),
        "iterations": infos[0]["iters"],
        "true_resid_max": max(chk["true_resid"]),
        "dslash_gflops": round(570 * vh * 1e-9 / (avg_us[0] * 1e-6), 1),
    }
    if rh:
        out.update(rh)
    if forms:
        out["precision_forms"] = forms
    if batched:
        out["batched_form"] = batched
    if improved:
        out["naik_operator"] = improved
    if hot:
        out["c1_hot"] = hot
    if memory:
        out["memory_check"] = memory
        out["roofline"]["beyond_cache"] = {
            "dslash_oe_48c3x16_frac": memory["solve_48c3x16"]["dslash_oe_frac_at_p50"],
            "dslash_oe_32c3x8_after_read_sweep_GB/s":
                memory["dslash_oe_32c3x8_isolated_after_2GiB_read_sweep_us"]["GB/s_at_p50"]}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(U, b, rat, vh, args.lag, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def precision_forms(lat, rat, bd, xs, vh, base, fp64_ms, reps=3):
    """The same 32^3x8 solve with 12-real FP64 links, and in mixed precision
    (FP32 Krylov vectors with FP32-18 or FP16-12 links, FP64 reliable updates,
    every pole to the FP64 true residual 1e-10)."""
    import torch
    from paper_1710_09178_amd import stag
    out = {}
    # FP64 reference solutions (18-real links), for the per-pole errors below
    lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
    x64 = [x.clone() for x in xs]

    def pole_errors():
        return [float(torch.linalg.vector_norm(x - r) / torch.linalg.vector_norm(r)) for x, r in zip(xs, x64)]

    # operator errors against the FP64 operator (itself equal to the oracle
    # to 1e-14): relative max-norm error of D_oe on a Gaussian even vector
    ref = lat.new_vec()
    lat.dslash(ref, bd, 1)
    op_err = {}
    for name, fmt in (("fp32_links18", stag.LINKS_F32_18), ("fp16_links12", stag.LINKS_F16_12)):
        y = lat.new_vec()
        lat.dslash_sloppy(y, bd, 1, fmt)
        op_err[name] = float((y - ref).abs().max() / ref.abs().max())
    lat.set_link_format(stag.LINKS_F64_12)
    y = lat.new_vec()
    lat.dslash(y, bd, 1)
    op_err["fp64_links12"] = float((y - ref).abs().max() / ref.abs().max())
    out["dslash_oe_rel_error_vs_fp64"] = op_err
    lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        i12 = lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
    torch.cuda.synchronize()
    ms12 = (time.perf_counter() - t0) / reps * 1e3
    chk = lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=True)
    out["fp64_links12"] = {"ms_per_solve": round(ms12, 3), "speedup_vs_fp64_18": round(fp64_ms / ms12, 3),
                           "iterations": i12["iters"], "true_resid_max": max(chk["true_resid"]),
                           "solution_rel_error_per_pole": [float("%.2e" % e) for e in pole_errors()]}
    lat.set_link_format(stag.LINKS_F64_18)
    for name, fmt in [("mixed_fp32_links18", stag.LINKS_F32_18), ("mixed_fp32_fp16links12", stag.LINKS_F16_12)]:
        lat.multishift_solve_mixed(MASS, rat, TOL, 100000, bd, xs, None, sloppy=fmt, true_resid=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            im = lat.multishift_solve_mixed(MASS, rat, TOL, 100000, bd, xs, None, sloppy=fmt, true_resid=False)
        torch.cuda.synchronize()
        msm = (time.perf_counter() - t0) / reps * 1e3
        chk = lat.multishift_solve_mixed(MASS, rat, TOL, 100000, bd, xs, None, sloppy=fmt, true_resid=True)
        out[name] = {"ms_per_solve": round(msm, 3), "speedup_vs_fp64_18": round(fp64_ms / msm, 3),
                     "iterations_total": im["iters"], "iterations_per_pole": im["iters_per_pole"],
                     "true_resid_max": max(chk["true_resid"]), "tol_sloppy": 1e-5, "reliable_every": 50,
                     "solution_rel_error_per_pole": [float("%.2e" % e) for e in pole_errors()]}
    return out


def vh_of(dims):
    return dims[0] * dims[1] * dims[2] * dims[3] // 2


def _pct(v):
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    return {"p10": round(float(np.percentile(v, 10)), 3), "p50": round(float(np.percentile(v, 50)), 3),
            "p90": round(float(np.percentile(v, 90)), 3), "n": int(v.size)}


def memory_check(lat, bd, vh, reps=20):
    """Which memory serves the D_oe kernel.  (1) STREAM-like ceilings of this
    GPU: a read-only sum of 4 GiB and a 2 GiB copy (torch kernels, events on
    torch's stream).  (2) The isolated 32^3x8 D_oe, back to back and each one
    right after a read-only 2 GiB sweep (no dirty lines left to write back),
    which evicts the 151 MB of links from the 256 MB Infinity Cache.  (3) The
    12-pole solve at 48^3x16, whose 1.02 GB of links cannot stay in any cache:
    its D_oe is served by HBM.  The 48^3x16 links are the 24^3x8 eps = 0.2
    field repeated 2x2x2x2 (bandwidth does not depend on the values); the
    source is drawn at full size."""
    import numpy as np
    import torch

    import synth
    from paper_1710_09178_amd.stag import Lattice
    out = {}
    big = torch.ones(4 * 2 ** 30 // 8, dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    big.sum()
    sums, copies = [], []
    half = big[: big.numel() // 2]
    dst = torch.empty_like(half)
    for _ in range(5):
        e0.record()
        big.sum()
        e1.record()
        torch.cuda.synchronize()
        sums.append(big.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        e0.record()
        dst.copy_(half)
        e1.record()
        torch.cuda.synchronize()
        copies.append(2 * half.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del dst
    out["stream_ceiling_GB/s"] = {"read_sum_4GiB": round(max(sums), 1), "copy_2GiB": round(max(copies), 1)}
    sweep = big[: 2 * 2 ** 30 // 8]
    y = lat.new_vec()
    for mode in ("back_to_back", "after_2GiB_read_sweep"):
        lat.profile_enable(4)
        for _ in range(reps):
            if mode != "back_to_back":
                sweep.sum()
            lat.dslash(y, bd, 1)
        us = lat.profile_samples(0)
        lat.profile_enable(0)
        pc = _pct(us)
        pc["GB/s_at_p50"] = round(B_DOE * vh / (pc["p50"] * 1e-6) / 1e9, 1)
        out[f"dslash_oe_32c3x8_isolated_{mode}_us"] = pc
    del big, sweep
    torch.cuda.empty_cache()
    dims = (48, 48, 48, 16)
    small = synth.random_su3_near_identity((24, 24, 24, 8), 0.2, synth.make_rng(1, 0))
    U = np.tile(small, (2, 2, 2, 2, 1, 1, 1))
    b = synth.gaussian_half_vector(dims, synth.make_rng(1, 2))
    rat = synth.load_rational(TABLE)
    big_lat = Lattice(dims)
    big_lat.set_gauge(torch.from_numpy(U).cuda())
    del U, small
    bdev = big_lat.vec_import(torch.from_numpy(b).cuda(), 0)
    xs = [big_lat.new_vec() for _ in rat["pole"]]
    solve_ms = {}
    for fz in (True, False):
        big_lat.set_fused_iteration(2 if fz else 0)
        big_lat.multishift_solve(MASS, rat, TOL, 100000, bdev, xs, None, true_resid=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = big_lat.multishift_solve(MASS, rat, TOL, 100000, bdev, xs, None, true_resid=False)
        solve_ms[fz] = ((time.perf_counter() - t0) * 1e3, info)
    ms, info = solve_ms[False]
    # the plain D_oe kernel inside the three-launch loop, links streamed
    # non-temporally (the default at this size) and with plain loads
    vh48 = big_lat.Vh
    doe_plain = None
    for mode in (0, 1):
        big_lat.set_link_streaming(mode)
        big_lat.profile_enable(3 * (info["iters"] + 64))
        chk = big_lat.multishift_solve(MASS, rat, TOL, 100000, bdev, xs, None, true_resid=True)
        doe = _pct(big_lat.profile_samples(0))
        deo = _pct(big_lat.profile_samples(1))
        big_lat.profile_enable(0)
        if mode == 0:
            doe_plain = doe
    base = int(np.argmin(rat["pole"]))
    out["solve_48c3x16"] = {
        "ms_per_solve_fused": round(solve_ms[True][0], 3), "ms_per_solve": round(ms, 3),
        "iterations": info["iters"], "true_resid_max": max(chk["true_resid"]),
        "value_GB/s": round(solve_bytes(vh48, info["iters"], info["iters_per_pole"], base, 8) / (ms * 1e-3) / 1e9, 1),
        "links_GB": round(2 * 4 * 144 * vh48 / 1e9, 3),
        "dslash_oe_us": doe, "dslash_oe_GB/s_at_p50": round(B_DOE * vh48 / (doe["p50"] * 1e-6) / 1e9, 1),
        "dslash_oe_plain_link_loads_us": doe_plain,
        "dslash_oe_plain_link_loads_GB/s_at_p50": round(B_DOE * vh48 / (doe_plain["p50"] * 1e-6) / 1e9, 1),
        "dslash_oe_frac_at_p50": round(B_DOE * vh48 / (doe["p50"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
        "dslash_eo_cg_us": deo, "dslash_eo_cg_GB/s_at_p50": round(B_DEO_CG * vh48 / (deo["p50"] * 1e-6) / 1e9, 1)}
    del big_lat, xs, bdev
    torch.cuda.empty_cache()
    return out


def c1_hot(reps=2):
    """The 32^3x8 12-pole solve (m = 0.005, tol 1e-10) on Haar-random links,
    whose dense low spectrum makes the solves long (the regime of the paper's
    production runs, thousands of iterations): FP64 with 18- and 12-real links
    against the mixed FP32/FP64 solve with FP32-18 links, every pole to the
    FP64 true residual 1e-10."""
    import torch

    import synth
    from paper_1710_09178_amd import stag
    from paper_1710_09178_amd.stag import Lattice
    U = synth.haar_su3(DIMS, synth.make_rng(1, 7))
    b = synth.gaussian_half_vector(DIMS, synth.make_rng(1, 1))
    rat = synth.load_rational(TABLE)
    lat = Lattice(DIMS)
    lat.set_gauge(torch.from_numpy(U).cuda())
    bd = lat.vec_import(torch.from_numpy(b).cuda(), 0)
    xs = [lat.new_vec() for _ in rat["pole"]]
    out = {"workload": "32^3x8 Haar links, m 0.005, 12 poles of x^(-1/4), tol 1e-10"}
    for name, fmt, mixed in (("fp64_links18", stag.LINKS_F64_18, False), ("fp64_links12", stag.LINKS_F64_12, False),
                             ("mixed_fp32_links18", stag.LINKS_F64_18, True)):
        lat.set_link_format(fmt)
        solve = (lambda tr: lat.multishift_solve_mixed(MASS, rat, TOL, 400000, bd, xs, None, sloppy=stag.LINKS_F32_18,
                                                       true_resid=tr)) if mixed else \
            (lambda tr: lat.multishift_solve(MASS, rat, TOL, 400000, bd, xs, None, true_resid=tr))
        solve(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            info = solve(False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        chk = solve(True)
        out[name] = {"ms_per_solve": round(ms, 2), "iterations": info["iters"],
                     "iterations_per_pole": info["iters_per_pole"], "true_resid_max": max(chk["true_resid"])}
    lat.set_link_format(stag.LINKS_F64_18)
    for k in ("fp64_links12", "mixed_fp32_links18"):
        out[k]["speedup_vs_fp64_links18"] = round(out["fp64_links18"]["ms_per_solve"] / out[k]["ms_per_solve"], 3)
    return out


# Naik-improved operator: 16 links per output site (8 one-hop, 8 long links)
B_NAIK_DOE = {"f64_links18": 16 * 144 + 96, "f64_links12": 16 * 96 + 96}
NAIK_FLOP = 16 * 66 + 15 * 6 + 2 * 6   # 16 SU(3) x vector, the sums, the two weights


def improved_operator(lat, rat, bd, xs, vh, reps=3):
    """The 32^3x8 12-pole solve with the Naik-improved operator (c1 = 9/8,
    c3 = -1/24), FP64 18-real and 12-real links: solve time, iterations, true
    residuals, and its D_oe kernel timed with events inside a profiled solve
    (algorithmic bytes: 16 links + in + out per output site)."""
    import torch
    from paper_1710_09178_amd import stag
    out = {}
    lat.set_naik(9.0 / 8.0, -1.0 / 24.0)
    for name, fmt in [("f64_links18", stag.LINKS_F64_18), ("f64_links12", stag.LINKS_F64_12)]:
        lat.set_link_format(fmt)
        lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            info = lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        lat.profile_enable(3 * (info["iters"] + 64))
        chk = lat.multishift_solve(MASS, rat, TOL, 100000, bd, xs, None, true_resid=True)
        pms, cnt = lat.profile_read()
        lat.profile_enable(0)
        us = 1e3 * pms[0] / max(cnt[0], 1)
        gbs = B_NAIK_DOE[name] * vh / (us * 1e-6) / 1e9
        out[name] = {"ms_per_solve": round(ms, 3), "iterations": info["iters"],
                     "true_resid_max": max(chk["true_resid"]),
                     "dslash_oe_avg_us": round(us, 3), "dslash_oe_GB/s": round(gbs, 1),
                     "dslash_oe_frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "dslash_oe_gflops": round(NAIK_FLOP * vh * 1e-9 / (us * 1e-6), 1),
                     "algorithmic_bytes_per_site": B_NAIK_DOE[name]}
    lat.set_link_format(stag.LINKS_F64_18)
    lat.set_naik(1.0, 0.0)
    return out


BATCH_DIMS = [(8, 8, 8, 8), (12, 12, 12, 6), (16, 16, 16, 8), (24, 24, 24, 6)]


def batch_bytes(dims, nrhs, iters_per_pole, base, lag):
    """Algorithmic FP64 bytes of one batched multi-shift solve: per instance and
    iteration the two Dslash launches read the links once for all right-hand
    sides; the shift update is counted per system from its per-pole stops."""
    total = 0
    for i, d in enumerate(dims):
        vh = d[0] * d[1] * d[2] * d[3] // 2
        ipp = iters_per_pole[i * nrhs:(i + 1) * nrhs]
        iters_inst = int(ipp.max())
        total += iters_inst * (1152 + 96 * nrhs + 1152 + 192 * nrhs) * vh
        for sys_ipp in ipp:
            total += solve_bytes(vh, int(sys_ipp.max()), list(sys_ipp), base, lag) \
                - (B_DOE + B_DEO_CG) * vh * int(sys_ipp.max())
    return total


def batched_form(per_class=16, nrhs=4, reps=2):
    """64 lattices (16 each of 8^4, 12^3x6, 16^3x8, 24^3x6) x 4 right-hand sides
    x the 12 poles of the x^(-1/4) table, masses uniform in [0.005, 0.05], in
    one batched multi-shift solve; FP64, mixed FP32/FP64, and FP64 reading 12
    reals per link; the same systems solved one after another."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import synth
    from paper_1710_09178_amd.stag import Batch
    dims = [d for d in BATCH_DIMS for _ in range(per_class)]
    rng = synth.make_rng(3, 0)
    masses = list(rng.uniform(0.005, 0.05, len(dims)))
    rat = synth.load_rational(TABLE)
    base = int(np.argmin(rat["pole"]))
    B = Batch(dims, nrhs)
    with ThreadPoolExecutor(8) as ex:
        fields = ex.map(lambda i: synth.random_su3_near_identity(dims[i], 0.2, synth.make_rng(3, 1000 + i)),
                        range(len(dims)))
        for i, U in enumerate(fields):
            B.set_gauge(i, torch.from_numpy(U).cuda())
    srcs = [synth.gaussian_half_vector(d, synth.make_rng(3, 5000 + 8 * i + j))
            for i, d in enumerate(dims) for j in range(nrhs)]
    b = torch.from_numpy(np.concatenate([v.reshape(-1) for v in srcs])).cuda()
    B.set_shift_window(8)
    tuned, choice = B.autotune(0)
    out = {"workload": f"{len(dims)} lattices (16 each of 8^4, 12^3x6, 16^3x8, 24^3x6) x {nrhs} right-hand "
                       f"sides x 12 poles of x^(-1/4), masses U[0.005, 0.05], tol 1e-10",
           "systems": len(dims) * nrhs, "sites": int(sum(np.prod(d) for d in dims)),
           "autotune_us": dict(zip(["tps1", "tps2", "tps4", "tps1_nt", "tps2_nt", "tps4_nt", "tps8"],
                                   [round(u, 2) for u in tuned])),
           "autotune_choice": {"threads_per_site": choice[0], "nontemporal_links": choice[1]}}
    for name, prec in (("fp64", 0), ("mixed_fp32_fp64", 1)):
        B.solve(masses, rat, b, precision=prec, true_resid=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, info = B.solve(masses, rat, b, precision=prec, true_resid=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        x, chk = B.solve(masses, rat, b, precision=prec, true_resid=True)
        lat_ms = np.array(info["latency"]) * 1e3
        row = {"ms_per_solve": round(dt * 1e3, 3), "iterations": info["iters"],
               "refine_iterations": info["refine_iters"],
               "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
               "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
               "true_resid_max": float(chk["true_resid"].max())}
        if prec == 0:
            row["GB/s"] = round(batch_bytes(dims, nrhs, info["iters_per_pole"], base, 8) / dt / 1e9, 1)
        out[name] = row
        del x
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["ms_per_solve"] / out["mixed_fp32_fp64"]["ms_per_solve"], 3)
    # FP64 reading 12 reals per link (rows 0-1, row 2 rebuilt), same work split
    from paper_1710_09178_amd import stag
    B.set_link_format(stag.LINKS_F64_12)
    B.solve(masses, rat, b, precision=0, true_resid=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, info = B.solve(masses, rat, b, precision=0, true_resid=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    x, chk = B.solve(masses, rat, b, precision=0, true_resid=True)
    out["fp64_links12"] = {"ms_per_solve": round(dt * 1e3, 3), "iterations": info["iters"],
                           "true_resid_max": float(chk["true_resid"].max()),
                           "speedup_vs_links18": round(out["fp64"]["ms_per_solve"] / (dt * 1e3), 3)}
    del x
    B.set_link_format(stag.LINKS_F64_18)
    # the same 256 systems one after another, one single-lattice handle per
    # lattice (FP64, library defaults), for the batched form's speedup
    from paper_1710_09178_amd.stag import Lattice
    del B, b
    torch.cuda.empty_cache()
    lats, vecs = [], []
    for i, d in enumerate(dims):
        lat = Lattice(d)
        lat.set_gauge(torch.from_numpy(synth.random_su3_near_identity(d, 0.2, synth.make_rng(3, 1000 + i))).cuda())
        lats.append(lat)
        vecs.append([lat.vec_import(torch.from_numpy(srcs[i * nrhs + j]).cuda(), 0) for j in range(nrhs)])
    del srcs
    xs = {}

    def sequential():
        iters = 0
        for i, lat in enumerate(lats):
            x = xs.setdefault(dims[i], [lat.new_vec() for _ in rat["pole"]])
            for j in range(nrhs):
                iters += lat.multishift_solve(masses[i], rat, 1e-10, 100000, vecs[i][j], x, None,
                                              true_resid=False)["iters"]
        return iters

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_iters = sequential()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    out["sequential_fp64"] = {"ms_for_all_systems": round(seq_ms, 3), "iterations_total": seq_iters,
                              "batched_speedup": round(seq_ms / out["fp64"]["ms_per_solve"], 3)}
    # the same with 12-real links on both sides
    for lat in lats:
        lat.set_link_format(stag.LINKS_F64_12)
    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    seq12 = (time.perf_counter() - t0) * 1e3
    out["sequential_fp64_links12"] = {"ms_for_all_systems": round(seq12, 3),
                                      "batched_speedup": round(seq12 / out["fp64_links12"]["ms_per_solve"], 3)}
    del lats, vecs, xs
    torch.cuda.empty_cache()
    return out


def improved_rhmc(lat, U_therm, summary, t_first, n_traj, beta, mass, tau, n_steps, kw, n_therm=8):
    """The same RHMC with the Naik-improved operator (c1 = 9/8, c3 = -1/24) in
    heat bath, force and actions, tables on [m^2, 88] (A is bounded by 87.1):
    n_therm accepted trajectories from the one-hop chain's configuration, then
    n_traj timed ones."""
    import torch

    import synth
    r_f = synth.load_rational("xm050_n12_m0.02_h88")
    r_a = synth.load_rational("xm050_n20_m0.02_h88")
    r_h = synth.load_rational("xp025_n20_m0.02_h88")
    lat.set_gauge(U_therm)
    lat.set_naik(9.0 / 8.0, -1.0 / 24.0)
    t = t_first + 1000
    for _ in range(n_therm):
        lat.trajectory(beta, mass, tau, n_steps, r_f, r_a, r_h, inject_u=0.0, traj_index=t, **kw)
        t += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = []
    for k in range(n_traj):
        res.append(lat.trajectory(beta, mass, tau, n_steps, r_f, r_a, r_h, traj_index=t, **kw))
        t += 1
        if (k + 1) % 50 == 0:
            log(f"improved-operator chain: {k + 1} of {n_traj} trajectories")
    torch.cuda.synchronize()
    out = summary(res, (time.perf_counter() - t1) / n_traj)
    lat.set_naik(1.0, 0.0)
    out["workload"] = ("as the one-hop chain, Naik-improved operator, tables on [m^2, 88], "
                       f"{n_therm} trajectories from the one-hop chain's configuration before timing")
    return out


def rhmc(with_model=True, n_exact=10, n_pairs=2000, n_traj=24, train_seconds=25.0, inner_iters=200,
         chain_steps=40, every_list=(2, 4), ablation=True, n_improved=10):
    """RHMC at 16^3x8 (beta 5.4, m 0.02, the 12-pole MD table with 20-pole
    action and heat-bath tables, tau 1, 20 leapfrog steps, MD tolerance 1e-8,
    action 1e-10) from a seeded hot start,
    thermalised by 60 pure-gauge and 5 dynamical trajectories (all accepted).
    sec_per_trajectory: n_exact exact-force trajectories continuing the chain.

    With the learned force model: exact-force trajectories record n_pairs
    (U, force) pairs, each with the force of a solve stopped after
    inner_iters iterations as the model's auxiliary channel; the model is
    trained on them on the GPU; then chains of n_traj trajectories of
    chain_steps leapfrog steps (a step size at which the exact force accepts
    well) start from the same configuration with the same momenta and
    pseudofermions: exact force on every kick, and for exact_every in (2, 4)
    a two-time-scale leapfrog with the exact force on the outer scale and on
    the inner scale (a) nothing (the ablation), (b) the truncated-solve force
    alone, (c) the trained model (which also sees the truncated-solve force);
    then the model's chain once more under stag_md_chain, the exact force
    judging the model at its exact kicks and taking over on a policy.
    Accept/reject always uses the exact action."""
    import numpy as np
    import torch

    import synth
    from paper_1710_09178_amd import stag
    from paper_1710_09178_amd.stag import Lattice, Surrogate
    dims = (16, 16, 16, 8)
    beta, mass, tau, n_steps = 5.4, 0.02, 1.0, 20
    r_f = synth.load_rational("xm050_n12_m0.02")     # MD force
    r_a = synth.load_rational("xm050_n20_m0.02")     # action (Metropolis), error 4.9e-12
    r_h = synth.load_rational("xp025_n20_m0.02")     # heat bath, error 3.4e-12
    lat = Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.haar_su3(dims, synth.make_rng(5, 0))).cuda())
    kw = dict(tol_md=1e-8, tol_action=1e-10, seed=11)
    t = 0
    for _ in range(60):
        lat.trajectory(beta, mass, 0.5, 20, r_f, r_a, r_h, no_fermions=True, inject_u=0.0, traj_index=t, **kw)
        t += 1
    for _ in range(5):
        lat.trajectory(beta, mass, tau, n_steps, r_f, r_a, r_h, inject_u=0.0, traj_index=t, **kw)
        t += 1

    def summary(res, sec):
        dH = np.array([r["dH"] for r in res])
        acc = np.array([r["accepted"] for r in res], dtype=np.float64)
        pmet = np.minimum(1.0, np.exp(-np.minimum(dH, 700.0)))
        edh = np.exp(-np.minimum(dH, 700.0))
        return {"sec_per_traj": round(sec, 4), "traj_per_s": round(1.0 / sec, 3),
                "acceptance": round(float(acc.mean()), 3),
                "acceptance_stderr": round(float(acc.std() / np.sqrt(max(len(acc) - 1, 1))), 3),
                "mean_min1_exp_minus_dH": round(float(pmet.mean()), 4),
                "mean_min1_exp_minus_dH_stderr": round(float(pmet.std() / np.sqrt(max(len(pmet) - 1, 1))), 4),
                "mean_abs_dH": round(float(np.mean(np.abs(dH))), 4),
                "mean_exp_minus_dH": round(float(edh.mean()), 4),
                "mean_exp_minus_dH_stderr": round(float(edh.std() / np.sqrt(max(len(edh) - 1, 1))), 4),
                "cg_iters_per_traj": int(np.mean([r["cg_iters_total"] for r in res])),
                "plaquette_end": round(res[-1]["plaquette"], 5), "trajectories": len(res)}

    U_therm = lat.get_gauge()
    pl = lat.polyakov_loop()
    t_first = t

    def timed_chain(**extra):
        lat.set_gauge(U_therm)
        torch.cuda.synchronize()
        with no_gc():
            t1 = time.perf_counter()
            res = [lat.trajectory(beta, mass, tau, n_steps, r_f, r_a, r_h, traj_index=t_first + i, **kw, **extra)
                   for i in range(n_exact)]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / n_exact
        return summary(res, dt)

    out = {"sec_per_trajectory": dict(timed_chain(), polyakov_loop_thermalised=[round(pl.real, 6), round(pl.imag, 6)],
                                      workload="RHMC 16^3x8, beta 5.4, m 0.02, 12-pole x^(-1/2) MD table, "
                                               "20-pole x^(-1/2) action and x^(1/4) heat-bath tables, tau 1, "
                                               "20 leapfrog steps, thermalised from a hot start")}
    # the same chain with three launches per CG iteration (no fused base update)
    lat.set_fused_iteration(False)
    out["sec_per_trajectory_three_launch_loop"] = timed_chain()
    lat.set_fused_iteration(True)
    # precision form in the trajectory: MD force solves with FP32 Krylov vectors
    md = {"fp32_links18": timed_chain(md_link_format=2), "fp32_fp16links12": timed_chain(md_link_format=3)}
    # every solve of the trajectory with FP64 12-real links (row 2 rebuilt; exact to rounding)
    lat.set_link_format(stag.LINKS_F64_12)
    md["fp64_links12_all_solves"] = timed_chain()
    lat.set_link_format(stag.LINKS_F64_18)
    for v in md.values():
        v["speedup_vs_fp64"] = round(out["sec_per_trajectory"]["sec_per_traj"] / v["sec_per_traj"], 3)
    out["md_precision_forms"] = md
    out["improved_operator"] = improved_rhmc(lat, U_therm, summary, t_first, n_improved, beta, mass, tau, n_steps,
                                             kw)
    out["improved_operator"]["sec_per_traj_vs_one_hop"] = round(
        out["improved_operator"]["sec_per_traj"] / out["sec_per_trajectory"]["sec_per_traj"], 3)
    t = t_first + n_exact
    if not with_model:
        return out

    log(f"recording {n_pairs} training pairs")
    sur = Surrogate(lat, n_pairs, seed=1)
    rec = []
    t0 = time.perf_counter()
    while sur.pairs < n_pairs:
        rec.append(lat.trajectory(beta, mass, tau, n_steps, r_f, r_a, r_h, surrogate=sur, record_pairs=True,
                                  inner_iters=inner_iters, traj_index=t, **kw))
        t += 1
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses, epochs, lr = [], 0, 1e-3
    while time.perf_counter() - t0 < train_seconds and epochs < 30:
        losses.append(sur.train(1, lr))
        epochs += 1
        if epochs == 10:
            lr = 3e-4
    t_train = time.perf_counter() - t0
    # the model that is the truncated-solve force alone (c_6 = 1)
    ident = Surrogate(lat, 0)
    p = np.zeros(ident.n_params, dtype=np.float32)
    p[-8 + 6] = 1.0
    ident.set_params(p)

    def force_errors(n=4):
        out_m, out_t = [], []
        xs = [lat.new_vec() for _ in r_h["pole"]]
        phi = lat.new_vec()
        mom, aux = lat.new_mom(), lat.new_mom()
        for j in range(n):
            xi = lat.random_source(99, 100000 + j)
            lat.multishift_solve(mass, r_h, 1e-10, 100000, xi, xs, phi, true_resid=False)
            lat.fermion_force(mass, r_f, 1e-10, 100000, phi, mom, 0.0)
            lat.fermion_force(mass, r_f, 1e-30, inner_iters, phi, aux, 0.0, allow_not_converged=True)
            sur.set_aux(aux)
            loss, _ = sur.eval(mom)
            sur.set_aux(None)
            ref = float((mom * mom).sum().item())
            out_m.append(float(np.sqrt(loss * lat.V * 4 / ref)))
            out_t.append(float(torch.linalg.vector_norm(mom - aux).item() / np.sqrt(ref)))
        return out_m, out_t

    U_start = lat.get_gauge()
    err_model, err_trunc = force_errors()

    def chain(**extra):
        log(f"chain of {n_traj} trajectories: " + ", ".join(f"{k}={v}" for k, v in extra.items() if k != "surrogate"))
        lat.set_gauge(U_start)
        torch.cuda.synchronize()
        res = []
        t1 = time.perf_counter()
        for i in range(n_traj):
            res.append(lat.trajectory(beta, mass, tau, chain_steps, r_f, r_a, r_h, traj_index=10 ** 6 + i,
                                      **kw, **extra))
            if (i + 1) % 50 == 0:
                log(f"  {i + 1} trajectories")
        torch.cuda.synchronize()
        return summary(res, (time.perf_counter() - t1) / n_traj)

    chains = {"exact": chain()}
    for every in every_list:
        ms = dict(exact_every=every, coarse_force=True)
        if ablation:
            chains[f"ablation_no_inner_force_exact_every_{every}"] = chain(**ms)
        chains[f"inner_truncated_solve_exact_every_{every}"] = chain(surrogate=ident, inner_iters=inner_iters, **ms)
        chains[f"inner_learned_model_exact_every_{every}"] = chain(surrogate=sur, inner_iters=inner_iters, **ms)
    # the exact force as the model's judge and fallback: the learned chain of
    # the largest E once more, judged at its exact kicks, under a policy that
    # hands trajectories to the exact force when the model errs or stalls
    every = max(every_list)
    policy = dict(window=8, min_acceptance=0.25, max_model_err=0.05, exact_trajectories=4)
    log(f"judged chain of {n_traj} trajectories: exact_every={every}, policy {policy}")
    lat.set_gauge(U_start)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = lat.chain(n_traj, beta, mass, tau, chain_steps, r_f, r_a, r_h, traj_index=10 ** 6, surrogate=sur,
                    inner_iters=inner_iters, exact_every=every, coarse_force=True, **policy, **kw)
    torch.cuda.synchronize()
    judged = summary(res, (time.perf_counter() - t1) / n_traj)
    errs = [r["model_force_err"] for r in res if r["used_model"]]
    judged.update(policy=policy, model_trajectories=len(errs), fallback_trajectories=n_traj - len(errs),
                  judged_model_force_err_mean=round(float(np.mean(errs)), 5) if errs else None,
                  judged_model_force_err_max=round(float(np.max(errs)), 5) if errs else None)
    chains[f"judged_learned_model_chain_exact_every_{every}"] = judged
    for k, v in chains.items():
        v["speedup_vs_exact"] = round(chains["exact"]["sec_per_traj"] / v["sec_per_traj"], 3)
    out["learned_force_rhmc"] = {
        "workload": f"the same RHMC with {chain_steps} leapfrog steps; two-time-scale leapfrog, exact force "
                    f"on the outer scale",
        "chain_steps": chain_steps, "inner_iters": inner_iters, "pairs": n_pairs, "recording_trajectories": len(rec),
        "recording_seconds": round(t_rec, 2),
        "recording_acceptance": round(float(np.mean([r["accepted"] for r in rec])), 3),
        "train_epochs": epochs, "train_seconds": round(t_train, 2),
        "train_loss_first_last": [losses[0], losses[-1]],
        "force_rel_error_model": [round(e, 4) for e in err_model],
        "force_rel_error_truncated_solve": [round(e, 4) for e in err_trunc],
        "force_rel_error_without_inner_force": 1.0,
        "chains": chains}
    return out


if __name__ == "__main__":
    main()
