"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) and Box-Muller
Gaussians, for the random fields of an HMC trajectory (paper Sec. 3.1 step 1;
Sec. 4, "generation of large arrays of random numbers").

One Philox round maps (c0,c1,c2,c3) with key (k0,k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is advanced by the Weyl constants
(0x9E3779B9, 0xBB67AE85) before every round after the first; 10 rounds.

Counter layout of this project (both sides use it):
    c0 = low 32 bits of the draw index,  c1 = field | (high bits of index) << 8,
    c2, c3 = low / high 32 bits of the trajectory number,  key = seed (lo, hi).
Fields: 0 momenta, 1 heat-bath source, 2 Metropolis uniform, 3 estimator
noise (c2, c3 then hold the noise vector's number).
Each draw gives two 53-bit uniforms u = ((w0 << 32 | w1) >> 11 + 1/2) 2^-53
in (0,1) and, by Box-Muller, two Gaussians
    g0 = sqrt(-2 ln u1) cos(2 pi u2),   g1 = sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF

FIELD_MOMENTUM = 0
FIELD_SOURCE = 1
FIELD_UNIFORM = 2
FIELD_NOISE = 3


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """ctr: (N, 4) integers < 2^32; key: (k0, k1).  Returns (N, 4) uint64 words."""
    c = [np.asarray(ctr[:, i], dtype=np.uint64) for i in range(4)]
    k0 = np.uint64(key[0] & MASK)
    k1 = np.uint64(key[1] & MASK)
    m = np.uint64(MASK)
    for rnd in range(10):
        if rnd:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & m, p1 & m,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & m, p0 & m]
    return np.stack(c, axis=1)


def _counters(index: np.ndarray, field: int, traj: int) -> np.ndarray:
    index = np.asarray(index, dtype=np.uint64)
    n = index.shape[0]
    ctr = np.empty((n, 4), dtype=np.uint64)
    ctr[:, 0] = index & np.uint64(MASK)
    ctr[:, 1] = np.uint64(field) | ((index >> np.uint64(32)) << np.uint64(8))
    ctr[:, 2] = np.uint64(traj & MASK)
    ctr[:, 3] = np.uint64((traj >> 32) & MASK)
    return ctr


def uniforms(index, field, seed, traj):
    """Two uniforms in (0,1) per draw index: (N, 2) float64."""
    w = philox4x32_10(_counters(index, field, traj), (seed & MASK, (seed >> 32) & MASK))
    a = ((w[:, 0] << np.uint64(32)) | w[:, 1]) >> np.uint64(11)
    b = ((w[:, 2] << np.uint64(32)) | w[:, 3]) >> np.uint64(11)
    scale = 2.0 ** -53
    return np.stack([(a.astype(np.float64) + 0.5) * scale, (b.astype(np.float64) + 0.5) * scale], axis=1)


def gaussians(index, field, seed, traj):
    """Two N(0,1) numbers per draw index: (N, 2) float64."""
    u = uniforms(index, field, seed, traj)
    rad = np.sqrt(-2.0 * np.log(u[:, 0]))
    ang = 2.0 * np.pi * u[:, 1]
    return np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)


def momentum(dims, seed: int, traj: int) -> np.ndarray:
    """Gaussian momenta P[t,z,y,x,mu,a] ~ N(0,1); link j = 4*l + mu uses draws
    4j..4j+3, draw q giving components 2q and 2q+1."""
    nx, ny, nz, nt = dims
    nlink = 4 * nx * ny * nz * nt
    g = gaussians(np.arange(4 * nlink, dtype=np.uint64), FIELD_MOMENTUM, seed, traj)
    return g.reshape(nt, nz, ny, nx, 4, 8)


def source(dims, seed: int, traj: int) -> np.ndarray:
    """Half vector xi (V/2, 3) with density exp(-xi^dag xi): site k, colour q
    uses draw 3k+q, real and imaginary parts N(0, 1/2)."""
    vh = nx_ny_nz_nt(dims) // 2
    g = gaussians(np.arange(3 * vh, dtype=np.uint64), FIELD_SOURCE, seed, traj)
    return (g[:, 0] + 1j * g[:, 1]).reshape(vh, 3) * np.sqrt(0.5)


def noise(dims, seed: int, k: int) -> np.ndarray:
    """Noise vector number k of the stochastic estimators: the same
    distribution as `source`, from its own field of the counter, so that it is
    independent of every heat-bath source of a chain with the same seed."""
    vh = nx_ny_nz_nt(dims) // 2
    g = gaussians(np.arange(3 * vh, dtype=np.uint64), FIELD_NOISE, seed, k)
    return (g[:, 0] + 1j * g[:, 1]).reshape(vh, 3) * np.sqrt(0.5)


def uniform(seed: int, traj: int) -> float:
    """The Metropolis uniform of a trajectory: first number of draw 0."""
    return float(uniforms(np.zeros(1, dtype=np.uint64), FIELD_UNIFORM, seed, traj)[0, 0])


def nx_ny_nz_nt(dims) -> int:
    nx, ny, nz, nt = dims
    return nx * ny * nz * nt
