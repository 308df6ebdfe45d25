"""Helpers for the GPU parity tests (device transfers and logging)."""
import sys

import numpy as np
import torch

from paper_1710_09178_amd.stag import Lattice


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def lattice(dims, U=None) -> Lattice:
    lat = Lattice(dims)
    if U is not None:
        lat.set_gauge(dev(U))
    return lat


def rel_err(got, exp) -> float:
    return float(np.abs(got - exp).max() / max(np.abs(exp).max(), 1e-300))
