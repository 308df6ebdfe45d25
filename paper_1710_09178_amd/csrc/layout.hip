// Conversions between the canonical boundary formats and the internal
// structure-of-arrays layouts, plus fill/copy kernels.
#include <hip/hip_fp16.h>

#include "common.h"
#include "dslash.h"

namespace stag {

namespace {

__global__ void k_gauge_to_internal(Geom g, const double2* __restrict__ canon, double2* __restrict__ links) {
    // one thread per (site, mu); canonical is [l][mu][9]
    const int V = 2 * g.vh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int l = i >> 2, mu = i & 3;
    const int x = l % g.nx, r = l / g.nx;
    const int y = r % g.ny, r2 = r / g.ny;
    const int z = r2 % g.nz, t = r2 / g.nz;
    const int par = (x + y + z + t) & 1;
    const int cb = l >> 1;
#pragma unroll
    for (int e = 0; e < 9; ++e) links[link_off(g, par, mu, e) + cb] = canon[(size_t)i * 9 + e];
}

__global__ void k_gauge_to_canon(Geom g, const double2* __restrict__ links, double2* __restrict__ canon) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int l = i >> 2, mu = i & 3;
    const int x = l % g.nx, r = l / g.nx;
    const int y = r % g.ny, r2 = r / g.ny;
    const int z = r2 % g.nz, t = r2 / g.nz;
    const int par = (x + y + z + t) & 1;
    const int cb = l >> 1;
#pragma unroll
    for (int e = 0; e < 9; ++e) canon[(size_t)i * 9 + e] = links[link_off(g, par, mu, e) + cb];
}

__global__ void k_vec_to_internal(int vh, const double2* __restrict__ canon, double2* __restrict__ vec) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= vh) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) vec[(size_t)c * vh + k] = canon[(size_t)k * 3 + c];
}

__global__ void k_vec_to_canon(int vh, const double2* __restrict__ vec, double2* __restrict__ canon) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= vh) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) canon[(size_t)k * 3 + c] = vec[(size_t)c * vh + k];
}

__global__ void k_mom_to_internal(Geom g, const double* __restrict__ canon, double* __restrict__ mom) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int l = i >> 2, mu = i & 3;
    const int x = l % g.nx, r = l / g.nx;
    const int y = r % g.ny, r2 = r / g.ny;
    const int z = r2 % g.nz, t = r2 / g.nz;
    const int par = (x + y + z + t) & 1;
    const int cb = l >> 1;
#pragma unroll
    for (int a = 0; a < 8; ++a) mom[mom_off(g, par, mu, a) + cb] = canon[(size_t)i * 8 + a];
}

__global__ void k_mom_to_canon(Geom g, const double* __restrict__ mom, double* __restrict__ canon) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int l = i >> 2, mu = i & 3;
    const int x = l % g.nx, r = l / g.nx;
    const int y = r % g.ny, r2 = r / g.ny;
    const int z = r2 % g.nz, t = r2 / g.nz;
    const int par = (x + y + z + t) & 1;
    const int cb = l >> 1;
#pragma unroll
    for (int a = 0; a < 8; ++a) canon[(size_t)i * 8 + a] = mom[mom_off(g, par, mu, a) + cb];
}

__global__ void k_fill_zero(uint4* __restrict__ p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_copy(uint4* __restrict__ d, const uint4* __restrict__ s, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// derived link copies: one thread per (parity, mu, site)
__global__ void k_links_to_d12(Geom g, const double2* __restrict__ d18, double2* __restrict__ d12) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * g.vh) return;
    const int pm = i / g.vh, cb = i % g.vh;
    const int par = pm >> 2, mu = pm & 3;
#pragma unroll
    for (int e = 0; e < 6; ++e) d12[link12_off(g, par, mu, e) + cb] = d18[link_off(g, par, mu, e) + cb];
}

__global__ void k_links_to_s18(Geom g, const double2* __restrict__ d18, float2* __restrict__ s18) {
    const size_t n = (size_t)72 * g.vh;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 v = d18[i];
        s18[i] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_links_to_h12(Geom g, const double2* __restrict__ d18, __half2* __restrict__ h12) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * g.vh) return;
    const int pm = i / g.vh, cb = i % g.vh;
    const int par = pm >> 2, mu = pm & 3;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double2 v = d18[link_off(g, par, mu, e) + cb];
        h12[link12_off(g, par, mu, e) + cb] = __floats2half2_rn((float)v.x, (float)v.y);
    }
}

// Long links: one thread per (parity, mu, site); the three factors sit on
// parities par, 1 - par, par.
__global__ void k_long_links(Geom g, const double2* __restrict__ d18, double2* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * g.vh) return;
    const int pm = i / g.vh, cb = i % g.vh;
    const int par = pm >> 2, mu = pm & 3;
    int c[4];
    cb_coords(g, par, cb, c[0], c[1], c[2], c[3]);
    const int n[4] = {g.nx, g.ny, g.nz, g.nt};
    M3 acc, u;
#pragma unroll
    for (int e = 0; e < 9; ++e) acc.e[e] = d18[link_off(g, par, mu, e) + cb];
#pragma unroll
    for (int k = 1; k <= 2; ++k) {
        c[mu] = (c[mu] + 1 == n[mu]) ? 0 : c[mu] + 1;
        const int cbk = cb_index(g, c[0], c[1], c[2], c[3]);
        const int pk = par ^ (k & 1);
#pragma unroll
        for (int e = 0; e < 9; ++e) u.e[e] = d18[link_off(g, pk, mu, e) + cbk];
        acc = m3_mul(acc, u);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) out[link_off(g, par, mu, e) + cb] = acc.e[e];
}

__global__ void k_axpy_real(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

// FP64 <-> FP32 copies of internal half vectors (the sloppy operator's input
// rounding and output widening)
__global__ void k_vec_narrow(size_t n, const double2* __restrict__ in, float2* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ void k_vec_widen(size_t n, const float2* __restrict__ in, double2* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

inline int blocks_for(size_t n, int bs = 256) { return (int)((n + bs - 1) / bs); }

}  // namespace

void launch_gauge_to_internal(const Geom& g, const double2* canon, double2* links, hipStream_t s) {
    const size_t n = (size_t)8 * g.vh;
    k_gauge_to_internal<<<blocks_for(n), 256, 0, s>>>(g, canon, links);
}
void launch_gauge_to_canon(const Geom& g, const double2* links, double2* canon, hipStream_t s) {
    const size_t n = (size_t)8 * g.vh;
    k_gauge_to_canon<<<blocks_for(n), 256, 0, s>>>(g, links, canon);
}
void launch_vec_to_internal(const Geom& g, const double2* canon, double2* vec, hipStream_t s) {
    k_vec_to_internal<<<blocks_for(g.vh), 256, 0, s>>>(g.vh, canon, vec);
}
void launch_vec_to_canon(const Geom& g, const double2* vec, double2* canon, hipStream_t s) {
    k_vec_to_canon<<<blocks_for(g.vh), 256, 0, s>>>(g.vh, vec, canon);
}
void launch_mom_to_internal(const Geom& g, const double* canon, double* mom, int, hipStream_t s) {
    const size_t n = (size_t)8 * g.vh;
    k_mom_to_internal<<<blocks_for(n), 256, 0, s>>>(g, canon, mom);
}
void launch_mom_to_canon(const Geom& g, const double* mom, double* canon, hipStream_t s) {
    const size_t n = (size_t)8 * g.vh;
    k_mom_to_canon<<<blocks_for(n), 256, 0, s>>>(g, mom, canon);
}
void launch_long_links(const Geom& g, const double2* d18, double2* long18, hipStream_t s) {
    k_long_links<<<blocks_for((size_t)8 * g.vh), 256, 0, s>>>(g, d18, long18);
}
void launch_links_to_d12(const Geom& g, const double2* d18, double2* d12, hipStream_t s) {
    k_links_to_d12<<<blocks_for((size_t)8 * g.vh), 256, 0, s>>>(g, d18, d12);
}
void launch_links_to_s18(const Geom& g, const double2* d18, float2* s18, hipStream_t s) {
    int nb = blocks_for((size_t)72 * g.vh);
    if (nb > 8192) nb = 8192;
    k_links_to_s18<<<nb, 256, 0, s>>>(g, d18, s18);
}
void launch_links_to_h12(const Geom& g, const double2* d18, void* h12, hipStream_t s) {
    k_links_to_h12<<<blocks_for((size_t)8 * g.vh), 256, 0, s>>>(g, d18, (__half2*)h12);
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    // every internal buffer is a multiple of 16 bytes
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    int nb = blocks_for(n16);
    if (nb > 8192) nb = 8192;
    k_fill_zero<<<nb, 256, 0, s>>>((uint4*)p, n16);
}
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    int nb = blocks_for(n16);
    if (nb > 8192) nb = 8192;
    k_copy<<<nb, 256, 0, s>>>((uint4*)dst, (const uint4*)src, n16);
}

void launch_vec_narrow(const Geom& g, const double2* in, float2* out, hipStream_t s) {
    const size_t n = (size_t)3 * g.vh;
    int nb = blocks_for(n);
    if (nb > 8192) nb = 8192;
    k_vec_narrow<<<nb, 256, 0, s>>>(n, in, out);
}
void launch_vec_widen(const Geom& g, const float2* in, double2* out, hipStream_t s) {
    const size_t n = (size_t)3 * g.vh;
    int nb = blocks_for(n);
    if (nb > 8192) nb = 8192;
    k_vec_widen<<<nb, 256, 0, s>>>(n, in, out);
}

void launch_axpy_real(size_t n, double a, const double* x, double* y, hipStream_t s) {
    if (n == 0) return;
    int nb = blocks_for(n);
    if (nb > 8192) nb = 8192;
    k_axpy_real<<<nb, 256, 0, s>>>(n, a, x, y);
}

}  // namespace stag
