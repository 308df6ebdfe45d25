// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) and Box-Muller
// Gaussians for the random fields of a trajectory (Sec. 3.1 step 1).
// Counter words: (draw index low, field | draw index high << 8, traj low,
// traj high); key = (seed low, seed high).  Fields: 0 momenta, 1 heat-bath
// source, 2 Metropolis uniform, 3 estimator noise.
#include "common.h"

namespace stag {

namespace {

struct U4 {
    uint32_t w[4];
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(M0, c.w[0]), lo0 = M0 * c.w[0];
        const uint32_t hi1 = __umulhi(M1, c.w[2]), lo1 = M1 * c.w[2];
        U4 n;
        n.w[0] = hi1 ^ c.w[1] ^ k0;
        n.w[1] = lo1;
        n.w[2] = hi0 ^ c.w[3] ^ k1;
        n.w[3] = lo0;
        c = n;
    }
    return c;
}

__device__ __forceinline__ void gauss_pair(uint64_t index, uint32_t field, uint64_t seed, uint64_t traj,
                                           double& g0, double& g1) {
    U4 c;
    c.w[0] = (uint32_t)index;
    c.w[1] = field | ((uint32_t)(index >> 32) << 8);
    c.w[2] = (uint32_t)traj;
    c.w[3] = (uint32_t)(traj >> 32);
    const U4 o = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = (((uint64_t)o.w[0] << 32) | o.w[1]) >> 11;
    const uint64_t b = (((uint64_t)o.w[2] << 32) | o.w[3]) >> 11;
    const double u1 = ((double)a + 0.5) * 0x1.0p-53;
    const double u2 = ((double)b + 0.5) * 0x1.0p-53;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * 3.14159265358979323846 * u2;
    double sn, cs;
    sincos(ang, &sn, &cs);
    g0 = rad * cs;
    g1 = rad * sn;
}

__global__ __launch_bounds__(kBlock) void k_random_momentum(Geom g, uint64_t seed, uint64_t traj,
                                                            double* __restrict__ mom) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    int x, y, z, t;
    cb_coords(g, par, cb, x, y, z, t);
    const uint64_t l = (uint64_t)x + (uint64_t)g.nx * (y + (uint64_t)g.ny * (z + (uint64_t)g.nz * t));
    const uint64_t link = 4 * l + mu;
    double* m = mom + mom_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double g0, g1;
        gauss_pair(4 * link + q, 0u, seed, traj, g0, g1);
        m[(size_t)(2 * q) * g.vh] = g0;
        m[(size_t)(2 * q + 1) * g.vh] = g1;
    }
}

__global__ __launch_bounds__(kBlock) void k_random_source(Geom g, uint64_t seed, uint64_t traj, uint32_t field,
                                                          double2* __restrict__ xi) {
    const int cb = blockIdx.x * kBlock + threadIdx.x;
    if (cb >= g.vh) return;
    const double s = 0.70710678118654752440;  // sqrt(1/2)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double g0, g1;
        gauss_pair(3 * (uint64_t)cb + q, field, seed, traj, g0, g1);
        xi[(size_t)q * g.vh + cb] = make_double2(s * g0, s * g1);
    }
}

__global__ void k_philox(U4 base, uint32_t k0, uint32_t k1, size_t n, uint32_t* __restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    U4 c = base;
    c.w[0] = base.w[0] + (uint32_t)i;
    const U4 o = philox10(c, k0, k1);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * i + k] = o.w[k];
}

__global__ void k_uniform(uint64_t seed, uint64_t traj, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    U4 c;
    c.w[0] = 0u;
    c.w[1] = 2u;
    c.w[2] = (uint32_t)traj;
    c.w[3] = (uint32_t)(traj >> 32);
    const U4 o = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = (((uint64_t)o.w[0] << 32) | o.w[1]) >> 11;
    out[0] = ((double)a + 0.5) * 0x1.0p-53;
}

}  // namespace

void launch_uniform(uint64_t seed, uint64_t traj, double* out, hipStream_t s) {
    k_uniform<<<1, 64, 0, s>>>(seed, traj, out);
}

void launch_random_momentum(const Geom& g, uint64_t seed, uint64_t traj, double* mom, hipStream_t s) {
    const int grid = (8 * g.vh + kBlock - 1) / kBlock;
    k_random_momentum<<<grid, kBlock, 0, s>>>(g, seed, traj, mom);
}

// field 1: the heat-bath source of trajectory traj; field 3: noise vector
// number traj of the stochastic estimators (an independent stream, so that a
// measurement with the chain's seed never reuses a heat-bath source)
void launch_random_source(const Geom& g, uint64_t seed, uint64_t traj, double2* xi, hipStream_t s, uint32_t field) {
    const int grid = (g.vh + kBlock - 1) / kBlock;
    k_random_source<<<grid, kBlock, 0, s>>>(g, seed, traj, field, xi);
}

void launch_philox(const uint32_t ctr[4], const uint32_t key[2], size_t n, uint32_t* out, hipStream_t s) {
    U4 base;
    for (int k = 0; k < 4; ++k) base.w[k] = ctr[k];
    const int grid = (int)((n + 255) / 256);
    k_philox<<<grid, 256, 0, s>>>(base, key[0], key[1], n, out);
}

}  // namespace stag
