// Even-odd staggered hopping operator (Sec. 3.2):
//   (D psi)(x) = sum_mu s_mu(x) U_mu(x) psi(x+mu) - s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu)
// for output sites of one parity, with fused epilogues for the multi-shift CG.
//
// Work decomposition: a 256-thread block owns SB = 256/TPS consecutive output
// sites (after the XCD-aware tile remap).  Each 64-lane wave takes one "slice"
// of 4/TPS directions for 64 sites, so every link load of a wave is one
// contiguous 1 KB stream of the structure-of-arrays layout.  The TPS partial
// colour vectors of a site meet in LDS; the epilogue then walks (colour, site)
// items so that all vector loads and stores are contiguous too.
#include "common.h"

namespace stag {

namespace {

__device__ __forceinline__ void hop_geometry(const Geom& g, int mu, int x, int y, int z, int t, int& cbf,
                                             int& cbb, double& sf, double& sb) {
    if (mu == 0) {
        const int xp = (x + 1 == g.nx) ? 0 : x + 1;
        const int xm = (x == 0) ? g.nx - 1 : x - 1;
        cbf = cb_index(g, xp, y, z, t);
        cbb = cb_index(g, xm, y, z, t);
        sf = sb = 1.0;
    } else if (mu == 1) {
        const int yp = (y + 1 == g.ny) ? 0 : y + 1;
        const int ym = (y == 0) ? g.ny - 1 : y - 1;
        cbf = cb_index(g, x, yp, z, t);
        cbb = cb_index(g, x, ym, z, t);
        sf = sb = (x & 1) ? -1.0 : 1.0;
    } else if (mu == 2) {
        const int zp = (z + 1 == g.nz) ? 0 : z + 1;
        const int zm = (z == 0) ? g.nz - 1 : z - 1;
        cbf = cb_index(g, x, y, zp, t);
        cbb = cb_index(g, x, y, zm, t);
        sf = sb = ((x + y) & 1) ? -1.0 : 1.0;
    } else {
        const int tp = (t + 1 == g.nt) ? 0 : t + 1;
        const int tm = (t == 0) ? g.nt - 1 : t - 1;
        cbf = cb_index(g, x, y, z, tp);
        cbb = cb_index(g, x, y, z, tm);
        const double eta = ((x + y + z) & 1) ? -1.0 : 1.0;
        sf = (t == g.nt - 1) ? -eta : eta;   // antiperiodic time boundary
        sb = (t == 0) ? -eta : eta;
    }
}

// acc += sf * U psi_f - sb * U'^dag psi_b for one direction
__device__ __forceinline__ void hop(const Geom& g, const double2* __restrict__ links, const double2* __restrict__ in,
                                    int out_par, int mu, int cb, int x, int y, int z, int t, double2 (&acc)[3]) {
    int cbf, cbb;
    double sf, sb;
    hop_geometry(g, mu, x, y, z, t, cbf, cbb, sf, sb);
    const double2* uf = links + link_off(g, out_par, mu, 0) + cb;
    const double2* ub = links + link_off(g, 1 - out_par, mu, 0) + cbb;
    double2 U[9], W[9], pf[3], pb[3];
#pragma unroll
    for (int e = 0; e < 9; ++e) U[e] = uf[(size_t)e * g.vh];
#pragma unroll
    for (int c = 0; c < 3; ++c) pf[c] = in[(size_t)c * g.vh + cbf];
#pragma unroll
    for (int e = 0; e < 9; ++e) W[e] = ub[(size_t)e * g.vh];
#pragma unroll
    for (int c = 0; c < 3; ++c) pb[c] = in[(size_t)c * g.vh + cbb];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double2 f = cmul(U[3 * a], pf[0]);
        f = cadd(f, cmul(U[3 * a + 1], pf[1]));
        f = cadd(f, cmul(U[3 * a + 2], pf[2]));
        double2 b = cmulc(W[a], pb[0]);
        b = cadd(b, cmulc(W[3 + a], pb[1]));
        b = cadd(b, cmulc(W[6 + a], pb[2]));
        acc[a].x += sf * f.x - sb * b.x;
        acc[a].y += sf * f.y - sb * b.y;
    }
}

// ---- epilogues: called once per (colour, site) item with the hopping sum v
struct EpiStore {
    static constexpr int K = 0;
    double2* out;
    int vh;
    __device__ void item(int site, int c, double2 v, double*) const { out[(size_t)c * vh + site] = v; }
    __device__ void finish(double*) const {}
};

// out = coef * in - v   (A = 4m^2 - D_eo D_oe when v = D_eo D_oe in)
struct EpiAxpy {
    static constexpr int K = 0;
    double2* out;
    const double2* in;
    double coef;
    int vh;
    __device__ void item(int site, int c, double2 v, double*) const {
        const size_t i = (size_t)c * vh + site;
        const double2 a = in[i];
        out[i] = make_double2(coef * a.x - v.x, coef * a.y - v.y);
    }
    __device__ void finish(double*) const {}
};

// Ap = mt p - v with the block partials of <p,Ap>, <r,Ap>, <Ap,Ap>; the
// multi-shift step kernel turns them into the iteration's scalars.
struct EpiCG {
    static constexpr int K = 3;
    double2* Ap;
    const double2* p;
    const double2* r;
    double* part;
    double mt;  // 4m^2 + sigma_0
    int vh;
    __device__ void item(int site, int c, double2 v, double* acc) const {
        const size_t i = (size_t)c * vh + site;
        const double2 pv = p[i], rv = r[i];
        const double2 a = make_double2(mt * pv.x - v.x, mt * pv.y - v.y);
        Ap[i] = a;
        acc[0] += pv.x * a.x + pv.y * a.y;
        acc[1] += rv.x * a.x + rv.y * a.y;
        acc[2] += a.x * a.x + a.y * a.y;
    }
    __device__ void finish(double* acc) const {
        double v[3] = {acc[0], acc[1], acc[2]};
        block_partial<3>(v, part);
    }
};

// block partials of |b - (coef x - v)|^2
struct EpiResid {
    static constexpr int K = 1;
    const double2* x;
    const double2* b;
    double* part;
    double coef;
    int vh;
    __device__ void item(int site, int c, double2 v, double* acc) const {
        const size_t i = (size_t)c * vh + site;
        const double2 xv = x[i], bv = b[i];
        const double rx = bv.x - (coef * xv.x - v.x), ry = bv.y - (coef * xv.y - v.y);
        acc[0] += rx * rx + ry * ry;
    }
    __device__ void finish(double* acc) const {
        double v[1] = {acc[0]};
        block_partial<1>(v, part);
    }
};

template <int TPS, class Epi>
__global__ __launch_bounds__(kBlock) void k_dslash(Geom g, const double2* __restrict__ links,
                                                   const double2* __restrict__ in, int out_par, Epi epi,
                                                   const MsState* __restrict__ gate) {
    constexpr int SB = kBlock / TPS;
    constexpr int DPT = 4 / TPS;
    if (gate && gate->done) return;  // converged solve: the whole grid skips
    __shared__ double2 part[TPS * 3 * SB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slice = wave % TPS, sgrp = wave / TPS;
    const int j = sgrp * 64 + lane;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int cb = tile * SB + j;
    double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    if (cb < g.vh) {
        int x, y, z, t;
        cb_coords(g, out_par, cb, x, y, z, t);
#pragma unroll
        for (int d = 0; d < DPT; ++d) hop(g, links, in, out_par, slice * DPT + d, cb, x, y, z, t, acc);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) part[(slice * 3 + c) * SB + j] = acc[c];
    __syncthreads();
    double racc[Epi::K > 0 ? Epi::K : 1];
#pragma unroll
    for (int k = 0; k < (Epi::K > 0 ? Epi::K : 1); ++k) racc[k] = 0.0;
    for (int it = threadIdx.x; it < 3 * SB; it += kBlock) {
        const int c = it / SB, jj = it % SB;
        const int site = tile * SB + jj;
        if (site >= g.vh) continue;
        double2 v = part[c * SB + jj];
#pragma unroll
        for (int s = 1; s < TPS; ++s) v = cadd(v, part[(s * 3 + c) * SB + jj]);
        epi.item(site, c, v, racc);
    }
    epi.finish(racc);
}

template <class Epi>
void launch_tps(const Geom& g, const double2* links, const double2* in, int out_par, const Epi& epi, int tps,
                const MsState* gate, hipStream_t s) {
    const int grid = dslash_grid(g, tps);
    switch (tps) {
        case 1: k_dslash<1, Epi><<<grid, kBlock, 0, s>>>(g, links, in, out_par, epi, gate); break;
        case 2: k_dslash<2, Epi><<<grid, kBlock, 0, s>>>(g, links, in, out_par, epi, gate); break;
        default: k_dslash<4, Epi><<<grid, kBlock, 0, s>>>(g, links, in, out_par, epi, gate); break;
    }
}

}  // namespace

int dslash_grid(const Geom& g, int tps) {
    const int sb = kBlock / (tps == 1 ? 1 : (tps == 2 ? 2 : 4));
    return (g.vh + sb - 1) / sb;
}

void launch_dslash(const Geom& g, const double2* links, const double2* in, double2* out, int out_par, int tps,
                   hipStream_t s) {
    launch_tps(g, links, in, out_par, EpiStore{out, g.vh}, tps, nullptr, s);
}

void launch_dslash_gated(const Geom& g, const double2* links, const double2* in, double2* out, int out_par,
                         int tps, const MsState* gate, hipStream_t s) {
    launch_tps(g, links, in, out_par, EpiStore{out, g.vh}, tps, gate, s);
}

void launch_dslash_axpy(const Geom& g, const double2* links, const double2* w_o, const double2* in, double c,
                        double2* out, int tps, hipStream_t s) {
    launch_tps(g, links, w_o, 0, EpiAxpy{out, in, c, g.vh}, tps, nullptr, s);
}

void launch_dslash_cg(const Geom& g, const double2* links, const double2* w_o, const double2* p, const double2* r,
                      double2* Ap, const MsState* gate, double* dpart, int tps, hipStream_t s, double mass_term) {
    launch_tps(g, links, w_o, 0, EpiCG{Ap, p, r, dpart, mass_term, g.vh}, tps, gate, s);
}

void launch_dslash_resid(const Geom& g, const double2* links, const double2* w_o, const double2* x,
                         const double2* b, double c, double* part, int tps, hipStream_t s) {
    launch_tps(g, links, w_o, 0, EpiResid{x, b, part, c, g.vh}, tps, nullptr, s);
}

}  // namespace stag
