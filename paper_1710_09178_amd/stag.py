"""Thin Python binding of libstag (include/stag.h) via ctypes.

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory (tensors) and the HIP stream.  If the
shared library has not been built this module raises instead of falling back
to anything else.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstag.so")

STAG_OK = 0
STAG_ERR_INVALID_ARG = -1
STAG_ERR_NO_GAUGE = -2
STAG_ERR_NOT_CONVERGED = -3
STAG_ERR_NONFINITE = -4
STAG_ERR_SPECTRUM = -5
STAG_ERR_HIP = -6
STAG_ERR_OOM = -7

FIELD_HALF_VEC, FIELD_MOM, FIELD_CANON_HALF_VEC, FIELD_CANON_GAUGE, FIELD_CANON_MOM = range(5)
LINKS_F64_18, LINKS_F64_12, LINKS_F32_18, LINKS_F16_12 = range(4)
MAX_POLES = 48


class StagError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stag error {code}: {msg}")
        self.code = code


class CRational(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("c0", ctypes.c_double),
                ("residue", ctypes.POINTER(ctypes.c_double)), ("pole", ctypes.POINTER(ctypes.c_double))]


class CSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("n", ctypes.c_int),
                ("true_resid", ctypes.POINTER(ctypes.c_double)),
                ("iters_per_pole", ctypes.POINTER(ctypes.c_int)), ("seconds", ctypes.c_double)]


class CMixedOpts(ctypes.Structure):
    _fields_ = [("sloppy", ctypes.c_int), ("tol_sloppy", ctypes.c_double), ("reliable_every", ctypes.c_int)]


class CHMCParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mass", ctypes.c_double), ("tau", ctypes.c_double),
                ("n_steps", ctypes.c_int), ("r_md", CRational), ("r_action", CRational),
                ("r_heatbath", CRational), ("tol_md", ctypes.c_double), ("tol_action", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("seed", ctypes.c_uint64), ("traj_index", ctypes.c_uint64),
                ("inject_mom", ctypes.c_void_p), ("inject_xi", ctypes.c_void_p),
                ("inject_u", ctypes.c_double), ("no_fermions", ctypes.c_int),
                ("surrogate", ctypes.c_void_p), ("exact_every", ctypes.c_int),
                ("coarse_force", ctypes.c_int), ("record_pairs", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("md_link_format", ctypes.c_int), ("spectrum_lo", ctypes.c_double),
                ("spectrum_hi", ctypes.c_double), ("judge_model", ctypes.c_int)]


class CTrajInfo(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("K_old", ctypes.c_double), ("Sg_old", ctypes.c_double),
                ("Sf_old", ctypes.c_double), ("K_new", ctypes.c_double), ("Sg_new", ctypes.c_double),
                ("Sf_new", ctypes.c_double), ("plaquette", ctypes.c_double), ("accepted", ctypes.c_int),
                ("cg_iters_total", ctypes.c_int), ("n_solves", ctypes.c_int), ("seconds", ctypes.c_double),
                ("model_force_err", ctypes.c_double), ("used_model", ctypes.c_int)]


class CChainPolicy(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int), ("min_acceptance", ctypes.c_double),
                ("max_model_err", ctypes.c_double), ("exact_trajectories", ctypes.c_int)]


class CBatchOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double), ("tol_sloppy", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("use_graph", ctypes.c_int)]


class CBatchInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("refine_iters", ctypes.c_int), ("seconds", ctypes.c_double),
                ("latency", ctypes.POINTER(ctypes.c_double)), ("true_resid", ctypes.POINTER(ctypes.c_double)),
                ("iters_sys", ctypes.POINTER(ctypes.c_int)), ("iters_per_pole", ctypes.POINTER(ctypes.c_int))]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libstag.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1710_09178_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    S = ctypes.c_int
    sig = {
        "stag_create": (S, [ctypes.POINTER(H), ctypes.POINTER(ctypes.c_int), P]),
        "stag_destroy": (S, [H]),
        "stag_last_error": (ctypes.c_char_p, [H]),
        "stag_field_bytes": (ctypes.c_size_t, [H, I]),
        "stag_set_gauge": (S, [H, P]),
        "stag_get_gauge": (S, [H, P]),
        "stag_vec_import": (S, [H, P, P, I]),
        "stag_vec_export": (S, [H, P, P, I]),
        "stag_mom_import": (S, [H, P, P]),
        "stag_mom_export": (S, [H, P, P]),
        "stag_dslash": (S, [H, P, P, I]),
        "stag_mdagm": (S, [H, P, P, D]),
        "stag_dslash_sloppy": (S, [H, P, P, I, I]),
        "stag_power_estimate": (S, [H, D, I, ctypes.c_uint64, ctypes.POINTER(D)]),
        "stag_check_spectrum": (S, [H, D, D, D, ctypes.POINTER(D)]),
        "stag_mdagm_sloppy": (S, [H, P, P, D, I]),
        "stag_multishift_solve": (S, [H, D, ctypes.POINTER(CRational), D, I, P, ctypes.POINTER(P), P,
                                      ctypes.POINTER(CSolveInfo)]),
        "stag_multishift_solve_mixed": (S, [H, D, ctypes.POINTER(CRational), D, I, P, ctypes.POINTER(P), P,
                                            ctypes.POINTER(CMixedOpts), ctypes.POINTER(CSolveInfo)]),
        "stag_set_link_format": (S, [H, I]),
        "stag_set_naik": (S, [H, D, D]),
        "stag_set_fused_iteration": (S, [H, I]),
        "stag_batch_autotune": (S, [H, I, ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "stag_set_link_streaming": (S, [H, I]),
        "stag_profile_samples": (S, [H, I, ctypes.POINTER(ctypes.c_float), I, ctypes.POINTER(I)]),
        "stag_mdagm_noalloc": (S, [H, P, P, D]),
        "stag_fermion_action": (S, [H, D, ctypes.POINTER(CRational), D, I, P, ctypes.POINTER(D),
                                    ctypes.POINTER(CSolveInfo)]),
        "stag_fermion_force": (S, [H, D, ctypes.POINTER(CRational), D, I, P, P, D, ctypes.POINTER(CSolveInfo)]),
        "stag_gauge_force": (S, [H, D, P, D]),
        "stag_gauge_action": (S, [H, D, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "stag_polyakov_loop": (S, [H, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "stag_chiral_condensate": (S, [H, D, D, I, I, ctypes.c_uint64, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "stag_kinetic_energy": (S, [H, P, ctypes.POINTER(D)]),
        "stag_link_update": (S, [H, P, D]),
        "stag_random_momentum": (S, [H, ctypes.c_uint64, ctypes.c_uint64, P]),
        "stag_random_source": (S, [H, ctypes.c_uint64, ctypes.c_uint64, P]),
        "stag_philox": (S, [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32), ctypes.c_size_t,
                            P, P]),
        "stag_md_trajectory": (S, [H, ctypes.POINTER(CHMCParams), ctypes.POINTER(CTrajInfo)]),
        "stag_md_chain": (S, [H, ctypes.POINTER(CHMCParams), ctypes.c_int, ctypes.POINTER(CChainPolicy),
                              ctypes.POINTER(CTrajInfo), ctypes.POINTER(ctypes.c_int)]),
        "stag_batch_create": (S, [ctypes.POINTER(H), I, ctypes.POINTER(ctypes.c_int), I, P]),
        "stag_batch_destroy": (S, [H]),
        "stag_batch_last_error": (ctypes.c_char_p, [H]),
        "stag_batch_vec_bytes": (ctypes.c_size_t, [H]),
        "stag_batch_set_gauge": (S, [H, I, P]),
        "stag_batch_solve": (S, [H, ctypes.POINTER(D), ctypes.POINTER(CRational), P, P, ctypes.POINTER(CBatchOpts),
                                 ctypes.POINTER(CBatchInfo)]),
        "stag_batch_tune": (S, [H, I, ctypes.POINTER(D)]),
        "stag_surrogate_create": (S, [ctypes.POINTER(H), H, I, ctypes.c_uint64]),
        "stag_surrogate_destroy": (S, [H]),
        "stag_surrogate_last_error": (ctypes.c_char_p, [H]),
        "stag_surrogate_param_count": (I, []),
        "stag_surrogate_pair_count": (I, [H]),
        "stag_surrogate_set_aux": (S, [H, P]),
        "stag_surrogate_capacity": (I, [H]),
        "stag_surrogate_params": (S, [H, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
        "stag_surrogate_add_pair": (S, [H, P]),
        "stag_surrogate_train": (S, [H, I, D, ctypes.POINTER(D)]),
        "stag_surrogate_eval": (S, [H, P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_float)]),
        "stag_surrogate_force": (S, [H, P, D]),
        "stag_set_shift_window": (S, [H, I]),
        "stag_set_graphs": (S, [H, I]),
        "stag_batch_set_shift_window": (S, [H, I]),
        "stag_batch_set_tps": (S, [H, I]),
        "stag_batch_set_link_format": (S, [H, I]),
        "stag_profile_enable": (S, [H, I]),
        "stag_profile_read": (S, [H, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_long)]),
        "stag_tune": (S, [H, I, I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_DOUBLE_TYPES = (torch.float64, torch.complex128)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _buf(t, nbytes: int, what: str, optional: bool = False) -> int | None:
    """Device pointer of a double-precision buffer of exactly nbytes bytes.

    The C ABI takes raw pointers, so a wrongly sized or typed tensor would make
    a kernel read or write outside it: every wrapper checks here first.
    """
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: a tensor is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if t.dtype not in _DOUBLE_TYPES:
        raise TypeError(f"{what}: expected float64 or complex128, got {t.dtype}")
    got = t.numel() * t.element_size()
    if got != nbytes:
        raise ValueError(f"{what}: expected {nbytes} bytes, got {got}")
    return _ptr(t)


def append_jsonl(log, record: dict) -> None:
    """Append record as one JSON line to log (a path, or an open text file):
    the per-trajectory log of a chain."""
    line = json.dumps(record, sort_keys=True) + "\n"
    if isinstance(log, (str, os.PathLike)):
        with open(log, "a") as f:
            f.write(line)
    else:
        log.write(line)
        log.flush()


class RationalArg:
    """Keeps the coefficient arrays of a CRational alive."""

    def __init__(self, rat):
        if isinstance(rat, dict):
            c0, res, pole = rat.get("c0", 0.0), rat["residue"], rat["pole"]
        else:
            c0, res, pole = rat
        self.res = np.ascontiguousarray(res, dtype=np.float64)
        self.pole = np.ascontiguousarray(pole, dtype=np.float64)
        self.c = CRational(len(self.pole), float(c0),
                           self.res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           self.pole.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


class Lattice:
    """One libstag handle: a lattice, its gauge field and solver workspace."""

    def __init__(self, dims: Sequence[int], stream: torch.cuda.Stream | None = None):
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.stream = stream or torch.cuda.current_stream()
        h = ctypes.c_void_p()
        arr = (ctypes.c_int * 4)(*self.dims)
        code = self.lib.stag_create(ctypes.byref(h), arr, ctypes.c_void_p(self.stream.cuda_stream))
        if code != STAG_OK:
            raise StagError(code, self.lib.stag_last_error(None).decode())
        self.h = h
        nx, ny, nz, nt = self.dims
        self.V = nx * ny * nz * nt
        self.Vh = self.V // 2
        # byte sizes of every field kind, checked before each call
        self._nb = {k: int(self.lib.stag_field_bytes(h, k)) for k in range(5)}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.stag_destroy(h)
            self.h = None

    def _check(self, code: int, allow=(STAG_OK,)):
        if code not in allow:
            raise StagError(code, self.lib.stag_last_error(self.h).decode())
        return code

    def _vec(self, t, what, optional=False):
        return _buf(t, self._nb[FIELD_HALF_VEC], what, optional)

    def _mom(self, t, what, optional=False):
        return _buf(t, self._nb[FIELD_MOM], what, optional)

    def _xs(self, xs, n):
        if xs is None:
            return None
        xs = list(xs)
        if len(xs) != n:
            raise ValueError(f"xs: expected {n} solution vectors (one per pole), got {len(xs)}")
        return (ctypes.c_void_p * n)(*[self._vec(x, f"xs[{k}]") for k, x in enumerate(xs)])

    # ---- allocation helpers (torch device memory)
    def field_bytes(self, kind: int) -> int:
        return int(self.lib.stag_field_bytes(self.h, kind))

    def new_vec(self) -> torch.Tensor:
        return torch.zeros(self.field_bytes(FIELD_HALF_VEC) // 8, dtype=torch.float64, device="cuda")

    def new_mom(self) -> torch.Tensor:
        return torch.zeros(self.field_bytes(FIELD_MOM) // 8, dtype=torch.float64, device="cuda")

    # ---- fields
    def set_gauge(self, U: torch.Tensor):
        self._check(self.lib.stag_set_gauge(self.h, _buf(U, self._nb[FIELD_CANON_GAUGE], "U")))

    def get_gauge(self) -> torch.Tensor:
        nx, ny, nz, nt = self.dims
        out = torch.empty((nt, nz, ny, nx, 4, 3, 3), dtype=torch.complex128, device="cuda")
        self._check(self.lib.stag_get_gauge(self.h, _ptr(out)))
        return out

    def vec_import(self, canon: torch.Tensor, parity: int = 0) -> torch.Tensor:
        out = self.new_vec()
        self._check(self.lib.stag_vec_import(self.h, _ptr(out), _buf(canon, self._nb[FIELD_CANON_HALF_VEC], "canon"),
                                             parity))
        return out

    def vec_export(self, internal: torch.Tensor, parity: int = 0) -> torch.Tensor:
        out = torch.empty((self.Vh, 3), dtype=torch.complex128, device="cuda")
        self._check(self.lib.stag_vec_export(self.h, _ptr(out), _buf(internal, self._nb[FIELD_HALF_VEC], "internal"),
                                             parity))
        return out

    def mom_import(self, canon: torch.Tensor) -> torch.Tensor:
        out = self.new_mom()
        self._check(self.lib.stag_mom_import(self.h, _ptr(out), _buf(canon, self._nb[FIELD_CANON_MOM], "canon")))
        return out

    def mom_export(self, internal: torch.Tensor) -> torch.Tensor:
        nx, ny, nz, nt = self.dims
        out = torch.empty((nt, nz, ny, nx, 4, 8), dtype=torch.float64, device="cuda")
        self._check(self.lib.stag_mom_export(self.h, _ptr(out), _buf(internal, self._nb[FIELD_MOM], "internal")))
        return out

    # ---- operators
    def dslash(self, out: torch.Tensor, inp: torch.Tensor, out_parity: int):
        self._check(self.lib.stag_dslash(self.h, self._vec(out, "out"), self._vec(inp, "inp"), out_parity))

    def mdagm(self, out: torch.Tensor, inp: torch.Tensor, mass: float):
        self._check(self.lib.stag_mdagm(self.h, self._vec(out, "out"), self._vec(inp, "inp"), float(mass)))

    def mdagm_noalloc(self, out: torch.Tensor, inp: torch.Tensor, mass: float):
        """stag_mdagm with its odd temporary in the library's static scratch array (no allocation)."""
        self._check(self.lib.stag_mdagm_noalloc(self.h, self._vec(out, "out"), self._vec(inp, "inp"), float(mass)))

    def dslash_sloppy(self, out: torch.Tensor, inp: torch.Tensor, out_parity: int, fmt: int):
        """The precision form's FP32 operator (links in fmt) on FP64 vectors."""
        self._check(self.lib.stag_dslash_sloppy(self.h, self._vec(out, "out"), self._vec(inp, "inp"), out_parity,
                                                int(fmt)))

    def mdagm_sloppy(self, out: torch.Tensor, inp: torch.Tensor, mass: float, fmt: int):
        self._check(self.lib.stag_mdagm_sloppy(self.h, self._vec(out, "out"), self._vec(inp, "inp"), float(mass),
                                               int(fmt)))

    def power_estimate(self, mass: float, iters: int, seed: int = 0) -> float:
        lam = ctypes.c_double()
        self._check(self.lib.stag_power_estimate(self.h, float(mass), int(iters), int(seed), ctypes.byref(lam)))
        return lam.value

    def check_spectrum(self, mass: float, xmin: float, xmax: float) -> float:
        """Raises StagError(STAG_ERR_SPECTRUM) if [xmin, xmax] misses the spectrum of A;
        returns the power estimate of its top (0 when the certain bound sufficed)."""
        lam = ctypes.c_double()
        self._check(self.lib.stag_check_spectrum(self.h, float(mass), float(xmin), float(xmax), ctypes.byref(lam)))
        return lam.value

    # ---- solver
    def multishift_solve(self, mass, rat, tol, maxiter, b, xs=None, sum_out=None, true_resid=True,
                         allow_not_converged=False):
        r = RationalArg(rat)
        n = r.c.n
        resid = (ctypes.c_double * n)()
        ipp = (ctypes.c_int * n)()
        info = CSolveInfo(0, 0, resid if true_resid else None, ipp, 0.0)
        xarr = self._xs(xs, n)
        code = self.lib.stag_multishift_solve(self.h, float(mass), ctypes.byref(r.c), float(tol), int(maxiter),
                                              self._vec(b, "b"), xarr, self._vec(sum_out, "sum_out", True),
                                              ctypes.byref(info))
        allow = (STAG_OK, STAG_ERR_NOT_CONVERGED) if allow_not_converged else (STAG_OK,)
        self._check(code, allow)
        return {"code": code, "iters": info.iters, "seconds": info.seconds,
                "true_resid": list(resid) if true_resid else None, "iters_per_pole": list(ipp)}

    def multishift_solve_mixed(self, mass, rat, tol, maxiter, b, xs=None, sum_out=None, sloppy=LINKS_F32_18,
                               tol_sloppy=1e-5, reliable_every=50, true_resid=True, allow_not_converged=False):
        r = RationalArg(rat)
        n = r.c.n
        resid = (ctypes.c_double * n)()
        ipp = (ctypes.c_int * n)()
        info = CSolveInfo(0, 0, resid if true_resid else None, ipp, 0.0)
        xarr = self._xs(xs, n)
        opts = CMixedOpts(int(sloppy), float(tol_sloppy), int(reliable_every))
        code = self.lib.stag_multishift_solve_mixed(self.h, float(mass), ctypes.byref(r.c), float(tol), int(maxiter),
                                                    self._vec(b, "b"), xarr, self._vec(sum_out, "sum_out", True),
                                                    ctypes.byref(opts), ctypes.byref(info))
        allow = (STAG_OK, STAG_ERR_NOT_CONVERGED) if allow_not_converged else (STAG_OK,)
        self._check(code, allow)
        return {"code": code, "iters": info.iters, "seconds": info.seconds,
                "true_resid": list(resid) if true_resid else None, "iters_per_pole": list(ipp)}

    def set_link_format(self, fmt: int):
        self._check(self.lib.stag_set_link_format(self.h, int(fmt)))

    def set_naik(self, c1: float = 9.0 / 8.0, c3: float = -1.0 / 24.0):
        """Naik-improved operator with weights (c1, c3); (1, 0) restores the one-hop operator."""
        self._check(self.lib.stag_set_naik(self.h, float(c1), float(c3)))

    def fermion_action(self, mass, rat, tol, maxiter, phi) -> float:
        r = RationalArg(rat)
        S = ctypes.c_double()
        info = CSolveInfo()
        self._check(self.lib.stag_fermion_action(self.h, float(mass), ctypes.byref(r.c), float(tol), int(maxiter),
                                                 self._vec(phi, "phi"), ctypes.byref(S), ctypes.byref(info)))
        return S.value

    def fermion_force(self, mass, rat, tol, maxiter, phi, mom, dt=0.0, allow_not_converged=False) -> dict:
        r = RationalArg(rat)
        info = CSolveInfo()
        code = self.lib.stag_fermion_force(self.h, float(mass), ctypes.byref(r.c), float(tol), int(maxiter),
                                           self._vec(phi, "phi"), self._mom(mom, "mom"), float(dt),
                                           ctypes.byref(info))
        self._check(code, (STAG_OK, STAG_ERR_NOT_CONVERGED) if allow_not_converged else (STAG_OK,))
        return {"code": code, "iters": info.iters, "seconds": info.seconds}

    def gauge_force(self, beta, mom, dt=0.0):
        self._check(self.lib.stag_gauge_force(self.h, float(beta), self._mom(mom, "mom"), float(dt)))

    def gauge_action(self, beta):
        S, plaq = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.stag_gauge_action(self.h, float(beta), ctypes.byref(S), ctypes.byref(plaq)))
        return S.value, plaq.value

    def polyakov_loop(self) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.stag_polyakov_loop(self.h, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def chiral_condensate(self, mass, tol, maxiter, n_noise, seed):
        mean, err = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.stag_chiral_condensate(self.h, float(mass), float(tol), int(maxiter), int(n_noise),
                                                    int(seed), ctypes.byref(mean), ctypes.byref(err)))
        return mean.value, err.value

    def kinetic_energy(self, mom) -> float:
        K = ctypes.c_double()
        self._check(self.lib.stag_kinetic_energy(self.h, self._mom(mom, "mom"), ctypes.byref(K)))
        return K.value

    def link_update(self, mom, dt):
        self._check(self.lib.stag_link_update(self.h, self._mom(mom, "mom"), float(dt)))

    def random_momentum(self, seed, traj) -> torch.Tensor:
        out = self.new_mom()
        self._check(self.lib.stag_random_momentum(self.h, int(seed), int(traj), _ptr(out)))
        return out

    def random_source(self, seed, traj) -> torch.Tensor:
        out = self.new_vec()
        self._check(self.lib.stag_random_source(self.h, int(seed), int(traj), _ptr(out)))
        return out

    def _hmc_params(self, args, beta, mass, tau, n_steps, r_md, r_action, r_heatbath, tol_md, tol_action,
                    maxiter, seed, traj_index, inject_mom, inject_xi, inject_u, no_fermions, surrogate,
                    exact_every, coarse_force, record_pairs, inner_iters, md_link_format, spectrum, judge_model):
        a, b, c = RationalArg(r_md), RationalArg(r_action), RationalArg(r_heatbath)
        args.extend((a, b, c))  # the coefficient arrays live as long as the caller's list
        return CHMCParams(beta, mass, tau, n_steps, a.c, b.c, c.c, tol_md, tol_action, maxiter, seed, traj_index,
                          self._mom(inject_mom, "inject_mom", True), self._vec(inject_xi, "inject_xi", True),
                          inject_u, int(no_fermions),
                          surrogate.h if surrogate is not None else None, int(exact_every),
                          int(coarse_force), int(record_pairs), int(inner_iters), int(md_link_format),
                          *(map(float, spectrum) if spectrum is not None else (0.0, 0.0)), int(judge_model))

    def trajectory(self, beta, mass, tau, n_steps, r_md, r_action, r_heatbath, tol_md=1e-10, tol_action=1e-10,
                   maxiter=100000, seed=0, traj_index=0, inject_mom=None, inject_xi=None, inject_u=-1.0,
                   no_fermions=False, surrogate=None, exact_every=1, coarse_force=False,
                   record_pairs=False, inner_iters=0, md_link_format=0, spectrum=None, judge_model=False,
                   log=None) -> dict:
        """One RHMC trajectory (stag_md_trajectory); returns the trajectory
        info as a dict.  log: a path or open text file that receives the info
        with the trajectory's parameters as one JSON line."""
        keep = []
        prm = self._hmc_params(keep, beta, mass, tau, n_steps, r_md, r_action, r_heatbath, tol_md, tol_action,
                               maxiter, seed, traj_index, inject_mom, inject_xi, inject_u, no_fermions, surrogate,
                               exact_every, coarse_force, record_pairs, inner_iters, md_link_format, spectrum,
                               judge_model)
        info = CTrajInfo()
        self._check(self.lib.stag_md_trajectory(self.h, ctypes.byref(prm), ctypes.byref(info)))
        out = {k: getattr(info, k) for k, _ in CTrajInfo._fields_}
        if log is not None:
            append_jsonl(log, dict(out, seed=int(seed), traj_index=int(traj_index), beta=float(beta),
                                   mass=float(mass), tau=float(tau), n_steps=int(n_steps),
                                   exact_every=int(exact_every), model=surrogate is not None,
                                   md_link_format=int(md_link_format)))
        return out

    def chain(self, n_traj, beta, mass, tau, n_steps, r_md, r_action, r_heatbath, window=4, min_acceptance=0.5,
              max_model_err=0.5, exact_trajectories=2, tol_md=1e-10, tol_action=1e-10, maxiter=100000, seed=0,
              traj_index=0, surrogate=None, exact_every=1, coarse_force=False, inner_iters=0, md_link_format=0,
              spectrum=None, log=None) -> list:
        """n_traj trajectories with the exact force judging the model and
        standing in for it (stag_md_chain); returns one info dict per
        trajectory.  log: as in trajectory(), one JSON line per trajectory."""
        keep = []
        prm = self._hmc_params(keep, beta, mass, tau, n_steps, r_md, r_action, r_heatbath, tol_md, tol_action,
                               maxiter, seed, traj_index, None, None, -1.0, False, surrogate, exact_every,
                               coarse_force, False, inner_iters, md_link_format, spectrum, True)
        pol = CChainPolicy(int(window), float(min_acceptance), float(max_model_err), int(exact_trajectories))
        infos = (CTrajInfo * max(int(n_traj), 1))()
        done = ctypes.c_int()
        code = self.lib.stag_md_chain(self.h, ctypes.byref(prm), int(n_traj), ctypes.byref(pol), infos,
                                      ctypes.byref(done))
        out = [{k: getattr(infos[t], k) for k, _ in CTrajInfo._fields_} for t in range(done.value)]
        if log is not None:
            for t, rec in enumerate(out):
                append_jsonl(log, dict(rec, seed=int(seed), traj_index=int(traj_index) + t, beta=float(beta),
                                       mass=float(mass), tau=float(tau), n_steps=int(n_steps),
                                       exact_every=int(exact_every) if rec["used_model"] else 1,
                                       model=bool(rec["used_model"]), md_link_format=int(md_link_format)))
        self._check(code)
        return out

    # ---- measurement / tuning
    def set_shift_window(self, lag: int):
        self._check(self.lib.stag_set_shift_window(self.h, int(lag)))

    def set_fused_iteration(self, mode):
        """0 / False: three-launch loop; 1 / True: fused on small grids (default); 2: fused at every size."""
        self._check(self.lib.stag_set_fused_iteration(self.h, int(mode)))

    def set_link_streaming(self, mode: int):
        """0 plain link loads, 1 non-temporal beyond the Infinity Cache (default), 2 always non-temporal."""
        self._check(self.lib.stag_set_link_streaming(self.h, int(mode)))

    def set_graphs(self, on: bool):
        self._check(self.lib.stag_set_graphs(self.h, int(bool(on))))

    def profile_enable(self, max_launches: int):
        self._check(self.lib.stag_profile_enable(self.h, int(max_launches)))

    def profile_read(self):
        ms = (ctypes.c_double * 3)()
        cnt = (ctypes.c_long * 3)()
        self._check(self.lib.stag_profile_read(self.h, ms, cnt))
        return list(ms), list(cnt)

    def profile_samples(self, kind: int) -> np.ndarray:
        """Recorded launch durations (microseconds) of one kind: 0 D_oe, 1 D_eo, 2 shift update."""
        n = ctypes.c_int()
        self._check(self.lib.stag_profile_samples(self.h, int(kind), None, 0, ctypes.byref(n)))
        buf = (ctypes.c_float * max(n.value, 1))()
        self._check(self.lib.stag_profile_samples(self.h, int(kind), buf, n.value, ctypes.byref(n)))
        return np.array(buf[:n.value], dtype=np.float64)

    def tune(self, tps: int, chunk: int):
        self._check(self.lib.stag_tune(self.h, int(tps), int(chunk)))


def philox(ctr, key, n: int) -> torch.Tensor:
    """Raw Philox4x32-10 words for counters ctr + (i,0,0,0), i < n (device tensor, int64 view of uint32)."""
    lib = load_library()
    out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    code = lib.stag_philox(c, k, n, _ptr(out), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if code != STAG_OK:
        raise StagError(code, lib.stag_last_error(None).decode())
    return out


class Batch:
    """A libstag batch: many lattices x right-hand sides, solved together."""

    def __init__(self, dims_list, nrhs: int, stream: torch.cuda.Stream | None = None):
        self.lib = load_library()
        self.dims = [tuple(int(v) for v in d) for d in dims_list]
        self.nrhs = int(nrhs)
        self.stream = stream or torch.cuda.current_stream()
        flat = (ctypes.c_int * (4 * len(self.dims)))(*[v for d in self.dims for v in d])
        h = ctypes.c_void_p()
        code = self.lib.stag_batch_create(ctypes.byref(h), len(self.dims), flat, self.nrhs,
                                          ctypes.c_void_p(self.stream.cuda_stream))
        if code != STAG_OK:
            raise StagError(code, self.lib.stag_batch_last_error(None).decode())
        self.h = h
        self.vh = [d[0] * d[1] * d[2] * d[3] // 2 for d in self.dims]

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.stag_batch_destroy(h)
            self.h = None

    def _check(self, code, allow=(STAG_OK,)):
        if code not in allow:
            raise StagError(code, self.lib.stag_batch_last_error(self.h).decode())
        return code

    def vec_len(self) -> int:
        """complex entries of one packed canonical batch vector"""
        return int(self.lib.stag_batch_vec_bytes(self.h)) // 16

    def set_gauge(self, inst: int, U: torch.Tensor):
        if not 0 <= int(inst) < len(self.dims):
            raise ValueError(f"inst: expected 0..{len(self.dims) - 1}, got {inst}")
        nb = 2 * self.vh[int(inst)] * 4 * 9 * 16
        self._check(self.lib.stag_batch_set_gauge(self.h, int(inst), _buf(U, nb, "U")))

    def solve(self, masses, rat, b: torch.Tensor, precision=0, tol=1e-10, tol_sloppy=1e-5, maxiter=100000,
              use_graph=True, true_resid=True, allow_not_converged=False):
        r = RationalArg(rat)
        n = r.c.n
        nsys = len(self.dims) * self.nrhs
        masses = [float(v) for v in masses]
        if len(masses) != len(self.dims):
            raise ValueError(f"masses: expected {len(self.dims)} values (one per lattice), got {len(masses)}")
        m = (ctypes.c_double * len(self.dims))(*masses)
        x = torch.empty(n * self.vec_len(), dtype=torch.complex128, device="cuda")
        lat = (ctypes.c_double * nsys)()
        res = (ctypes.c_double * (nsys * n))()
        its = (ctypes.c_int * nsys)()
        ipp = (ctypes.c_int * (nsys * n))()
        info = CBatchInfo(0, 0, 0.0, lat, res if true_resid else None, its, ipp)
        opts = CBatchOpts(int(precision), float(tol), float(tol_sloppy), int(maxiter), int(use_graph))
        code = self.lib.stag_batch_solve(self.h, m, ctypes.byref(r.c), _buf(b, 16 * self.vec_len(), "b"), _ptr(x),
                                         ctypes.byref(opts),
                                         ctypes.byref(info))
        allow = (STAG_OK, STAG_ERR_NOT_CONVERGED) if allow_not_converged else (STAG_OK,)
        self._check(code, allow)
        return x.view(n, -1), {"code": code, "iters": info.iters, "refine_iters": info.refine_iters,
                               "seconds": info.seconds, "latency": list(lat),
                               "true_resid": (np.array(list(res)).reshape(nsys, n) if true_resid else None),
                               "iters_sys": list(its), "iters_per_pole": np.array(list(ipp)).reshape(nsys, n)}

    def set_shift_window(self, lag: int):
        self._check(self.lib.stag_batch_set_shift_window(self.h, int(lag)))

    def set_tps(self, tps: int):
        self._check(self.lib.stag_batch_set_tps(self.h, int(tps)))

    def set_link_format(self, fmt: int):
        """LINKS_F64_18 (default) or LINKS_F64_12: the operators read rows 0-1 of each link."""
        self._check(self.lib.stag_batch_set_link_format(self.h, int(fmt)))

    def tune(self, precision=0):
        us = (ctypes.c_double * 4)()
        self._check(self.lib.stag_batch_tune(self.h, int(precision), us))
        return list(us)

    def autotune(self, precision=0, cache_path=None):
        """Threads per site x link loads, with an optional persisted cache; returns
        (microseconds per candidate, (tps, link_nt, from_cache))."""
        us = (ctypes.c_double * 7)()
        ch = (ctypes.c_int * 3)()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.stag_batch_autotune(self.h, int(precision), path, us, ch))
        return list(us), tuple(ch)


class Surrogate:
    """The learned force model of a Lattice (see include/stag.h)."""

    def __init__(self, lat: Lattice, capacity: int, seed: int = 0):
        self.lib = lat.lib
        self.lat = lat
        h = ctypes.c_void_p()
        code = self.lib.stag_surrogate_create(ctypes.byref(h), lat.h, int(capacity), int(seed))
        if code != STAG_OK:
            raise StagError(code, lat.lib.stag_last_error(lat.h).decode())
        self.h = h
        self.n_params = int(self.lib.stag_surrogate_param_count())

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.stag_surrogate_destroy(h)
            self.h = None

    def _check(self, code):
        if code != STAG_OK:
            raise StagError(code, self.lib.stag_surrogate_last_error(self.h).decode())

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.stag_surrogate_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), None))
        return out

    def set_params(self, p):
        arr = np.ascontiguousarray(p, dtype=np.float32)
        if arr.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {arr.size}")
        self._check(self.lib.stag_surrogate_params(self.h, None, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    @property
    def pairs(self) -> int:
        return int(self.lib.stag_surrogate_pair_count(self.h))

    @property
    def capacity(self) -> int:
        return int(self.lib.stag_surrogate_capacity(self.h))

    def set_aux(self, aux: torch.Tensor | None):
        self._check(self.lib.stag_surrogate_set_aux(self.h, self.lat._mom(aux, "aux", True)))

    def add_pair(self, force: torch.Tensor):
        self._check(self.lib.stag_surrogate_add_pair(self.h, self.lat._mom(force, "force")))

    def train(self, epochs: int, lr: float) -> float:
        loss = ctypes.c_double()
        self._check(self.lib.stag_surrogate_train(self.h, int(epochs), float(lr), ctypes.byref(loss)))
        return loss.value

    def eval(self, force: torch.Tensor, want_grad=False):
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None
        self._check(self.lib.stag_surrogate_eval(self.h, self.lat._mom(force, "force"), ctypes.byref(loss), gp))
        return loss.value, g

    def force(self, mom: torch.Tensor, dt: float = 0.0):
        self._check(self.lib.stag_surrogate_force(self.h, self.lat._mom(mom, "mom"), float(dt)))


def surrogate_params_to_flat(params: dict) -> np.ndarray:
    """Flatten a parameter dict (W1, b1, W2, b2, W3, b3) in the library's order."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
