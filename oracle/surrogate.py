"""Reference for the learned force model (not in the paper).

The model stands in for the pseudofermion force on intermediate MD steps.  It
is gauge covariant by construction:

* channels: for link (x, mu) and each nu != mu the upper and lower staples
      S_up = U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
      S_dn = U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
  in the order nu = the three directions other than mu ascending, up then down
  (6 channels; U_mu(x) S_j is a closed loop through the link);
* an optional seventh channel: an auxiliary force field G(x, mu) supplied by
  the caller (8 components per link, transforming like a force), used as is;
* invariant inputs: Re and Im tr(U_mu(x) S_j) for the 6 channels, the site
  parity (+-1), the staggered sign of the link (+-1), and the cosine of the
  angle between G and the sum of the six staple forces (0 without G), padded
  with zeros to F_IN = 16;
* MLP: h1 = silu(W1 f + b1), h2 = silu(W2 h1 + b2), c = W3 h2 + b3, widths
  16 -> 64 -> 64 -> 8 (the first 7 outputs are used);
* force: F_a(x, mu) = sum_{j<6} c_j Im tr(T_a U_mu(x) S_j) + c_6 G_a(x, mu):
  a learned, link-dependent combination of covariant force fields.

Loss: L = (1/N) sum over links and a of (F_s - F_target)^2, N = number of
links.  Gradients are written out by hand (the reference for the GPU's
backward kernels) and checked against finite differences.  A "bf16" mode
rounds the weights and the inputs of every matrix product to bfloat16
(round to nearest even) where the GPU's matrix-core kernels do: the inputs
of every forward product (features, h1, h2 and the weights) and of every
backward product (dL/dc, dL/dz2, dL/dz1 with the weights and activations);
biases, pre-activations, the loss and all accumulations stay wide.
"""
from __future__ import annotations

import numpy as np

from . import lattice as L
from .su3 import T

F_IN, HID, N_OUT, N_CH = 16, 64, 8, 7
N_STAPLE = 6


def channels(U: np.ndarray, dims) -> np.ndarray:
    """Staple channels, shape (Nt,Nz,Ny,Nx,4,6,3,3)."""
    nx, ny, nz, nt = dims
    out = np.zeros((nt, nz, ny, nx, 4, N_STAPLE, 3, 3), dtype=np.complex128)
    dag = lambda m: np.swapaxes(m, -1, -2).conj()
    mm = lambda a, b: np.einsum("...ij,...jk->...ik", a, b)
    for mu in range(4):
        u_mu = U[..., mu, :, :]
        j = 0
        for nu in range(4):
            if nu == mu:
                continue
            u_nu = U[..., nu, :, :]
            out[..., mu, 2 * j, :, :] = mm(mm(L.fwd(u_nu, mu), dag(L.fwd(u_mu, nu))), dag(u_nu))
            low = mm(mm(dag(L.fwd(u_nu, mu)), dag(u_mu)), u_nu)
            out[..., mu, 2 * j + 1, :, :] = L.bwd(low, nu)
            j += 1
    return out


def features(U: np.ndarray, dims, aux=None):
    """Per-link inputs (N_links, F_IN) in canonical link order (site, mu), and
    the loops U S_j (N_links, 6, 3, 3).  aux: optional auxiliary force field
    (Nt,Nz,Ny,Nx,4,8)."""
    S = channels(U, dims)
    loops = np.einsum("...ij,...cjk->...cik", U, S)
    tr = np.trace(loops, axis1=-2, axis2=-1)
    V = L.volume(dims)
    f = np.zeros((V, 4, F_IN))
    f[..., 0:12:2] = tr.real.reshape(V, 4, N_STAPLE)
    f[..., 1:12:2] = tr.imag.reshape(V, 4, N_STAPLE)
    par = L.parity(dims).reshape(V)
    f[..., 12] = np.where(par == 0, 1.0, -1.0)[:, None]
    for mu in range(4):
        f[:, mu, 13] = L.staggered_sign(dims, mu).reshape(V)
    f = f.reshape(4 * V, F_IN)
    loops = loops.reshape(4 * V, N_STAPLE, 3, 3)
    if aux is not None:
        g = np.asarray(aux, dtype=np.float64).reshape(4 * V, 8)
        gs = basis(loops)[:, :N_STAPLE, :].sum(1)
        f[:, 14] = np.einsum("na,na->n", g, gs) / (np.linalg.norm(g, axis=1) * np.linalg.norm(gs, axis=1) + 1e-30)
    return f, loops


def basis(loops: np.ndarray, aux=None) -> np.ndarray:
    """B[l, j, a]: Im tr(T_a loop_j) (the force of staple channel j) for j < 6
    and the auxiliary force for j = 6 (zero without one), shape (N, 7, 8)."""
    B = np.zeros((loops.shape[0], N_CH, 8))
    B[:, :N_STAPLE, :] = np.einsum("aij,ncji->nca", T, loops).imag
    if aux is not None:
        B[:, N_STAPLE, :] = np.asarray(aux, dtype=np.float64).reshape(-1, 8)
    return B


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(rng: np.random.Generator) -> dict:
    """He-style initialisation; the last layer starts at zero force."""
    return {"W1": rng.standard_normal((HID, F_IN)) * np.sqrt(2.0 / F_IN), "b1": np.zeros(HID),
            "W2": rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID), "b2": np.zeros(HID),
            "W3": rng.standard_normal((N_OUT, HID)) * 0.01, "b3": np.zeros(N_OUT)}


def forward(params, f, B, mode="fp64"):
    """Returns (force (N,8), cache).  mode 'bf16' rounds weights and layer
    inputs to bfloat16 before each product (FP32/FP64 accumulation)."""
    r = bf16 if mode == "bf16" else (lambda a: a)
    W1, W2, W3 = r(params["W1"]), r(params["W2"]), r(params["W3"])
    z1 = r(f) @ W1.T + params["b1"]
    h1 = silu(z1)
    z2 = r(h1) @ W2.T + params["b2"]
    h2 = silu(z2)
    c = r(h2) @ W3.T + params["b3"]
    F = np.einsum("nj,nja->na", c[:, :N_CH], B)
    return F, {"f": f, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "c": c, "B": B, "W": (W1, W2, W3), "r": r}


def loss_and_grad(params, f, B, target, mode="fp64"):
    """L = mean over links of |F - target|^2 (summed over a) and dL/dparams."""
    F, k = forward(params, f, B, mode)
    N = f.shape[0]
    diff = F - target
    L_ = float(np.sum(diff * diff) / N)
    r = k["r"]
    W1, W2, W3 = k["W"]
    dF = 2.0 * diff / N                                   # (N, 8)
    dc = np.zeros((N, N_OUT))
    dc[:, :N_CH] = np.einsum("na,nja->nj", dF, k["B"])    # (N, 8)
    g = {"W3": r(dc).T @ r(k["h2"]), "b3": dc.sum(0)}
    dh2 = r(dc) @ W3
    dz2 = dh2 * dsilu(k["z2"])
    g["W2"] = r(dz2).T @ r(k["h1"])
    g["b2"] = dz2.sum(0)
    dh1 = r(dz2) @ W2
    dz1 = dh1 * dsilu(k["z1"])
    g["W1"] = r(dz1).T @ r(k["f"])
    g["b1"] = dz1.sum(0)
    return L_, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for key in params:
        m = state.setdefault("m_" + key, np.zeros_like(params[key]))
        v = state.setdefault("v_" + key, np.zeros_like(params[key]))
        m[...] = beta1 * m + (1 - beta1) * grads[key]
        v[...] = beta2 * v + (1 - beta2) * grads[key] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[key] -= lr * mh / (np.sqrt(vh) + eps)


def surrogate_force(params, U, dims, mode="fp64", aux=None) -> np.ndarray:
    """The model's force field, shape (Nt,Nz,Ny,Nx,4,8)."""
    f, loops = features(U, dims, aux)
    F, _ = forward(params, f, basis(loops, aux), mode)
    nx, ny, nz, nt = dims
    return F.reshape(nt, nz, ny, nx, 4, 8)
