// Even-odd staggered hopping operator (Sec. 3.2):
//   (D psi)(x) = sum_mu s_mu(x) U_mu(x) psi(x+mu) - s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu)
// for output sites of one parity, with fused epilogues for the solvers.
// The Naik-improved operator (the "improved" quarks of the Summary, Sec. 8)
// weights that sum by c1 and adds c3 times the same stencil at distance 3,
// with the three-link products L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu)
// ("long links", built once per gauge field) in place of U.
//
// Work decomposition: a 256-thread block owns SB = 256/TPS consecutive output
// sites (after the XCD-aware tile remap).  Each 64-lane wave takes one "slice"
// of 4/TPS directions for 64 sites, so every link load of a wave is one
// contiguous stream of the structure-of-arrays layout.  The TPS partial colour
// vectors of a site meet in LDS; the epilogue then walks (colour, site) items
// so that all vector loads and stores are contiguous too.
//
// Link storage formats (template parameter):
//   LinkD18  FP64, 9 complex entries            (144 B/link)
//   LinkD12  FP64, rows 0-1, row 2 rebuilt       (96 B/link)
//   LinkS18  FP32, 9 complex entries             (72 B/link)
//   LinkH12  FP16, rows 0-1, row 2 rebuilt       (24 B/link)
// For an SU(3) matrix row 2 = conj(row 0 x row 1); the staggered signs are
// applied outside the matrix, so stored links stay in SU(3).
// FP64 links go with FP64 vectors, the others with FP32 vectors.
#include <hip/hip_fp16.h>

#include "common.h"
#include "dslash.h"

namespace stag {

namespace {

template <class C>
__device__ __forceinline__ void rebuild_row2(C (&m)[9]) {
    m[6] = cconj(csub(cmul(m[1], m[5]), cmul(m[2], m[4])));
    m[7] = cconj(csub(cmul(m[2], m[3]), cmul(m[0], m[5])));
    m[8] = cconj(csub(cmul(m[0], m[4]), cmul(m[1], m[3])));
}

struct LinkD18 {
    using C = double2;
    using R = double;
    const double2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const double2* p = u + link_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = p[(size_t)e * g.vh];
    }
};

struct LinkD12 {
    using C = double2;
    using R = double;
    const double2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const double2* p = u + link12_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 6; ++e) m[e] = p[(size_t)e * g.vh];
        rebuild_row2(m);
    }
};

struct LinkS18 {
    using C = float2;
    using R = float;
    const float2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const float2* p = u + link_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = p[(size_t)e * g.vh];
    }
};

struct LinkH12 {
    using C = float2;
    using R = float;
    const __half2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const __half2* p = u + link12_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 6; ++e) m[e] = __half22float2(p[(size_t)e * g.vh]);
        rebuild_row2(m);
    }
};

__device__ __forceinline__ void hop_geometry(const Geom& g, int mu, int x, int y, int z, int t, int& cbf,
                                             int& cbb, bool& nf, bool& nb) {
    // nf / nb: the forward / backward term carries a minus sign
    if (mu == 0) {
        const int xp = (x + 1 == g.nx) ? 0 : x + 1;
        const int xm = (x == 0) ? g.nx - 1 : x - 1;
        cbf = cb_index(g, xp, y, z, t);
        cbb = cb_index(g, xm, y, z, t);
        nf = nb = false;
    } else if (mu == 1) {
        const int yp = (y + 1 == g.ny) ? 0 : y + 1;
        const int ym = (y == 0) ? g.ny - 1 : y - 1;
        cbf = cb_index(g, x, yp, z, t);
        cbb = cb_index(g, x, ym, z, t);
        nf = nb = (x & 1);
    } else if (mu == 2) {
        const int zp = (z + 1 == g.nz) ? 0 : z + 1;
        const int zm = (z == 0) ? g.nz - 1 : z - 1;
        cbf = cb_index(g, x, y, zp, t);
        cbb = cb_index(g, x, y, zm, t);
        nf = nb = ((x + y) & 1);
    } else {
        const int tp = (t + 1 == g.nt) ? 0 : t + 1;
        const int tm = (t == 0) ? g.nt - 1 : t - 1;
        cbf = cb_index(g, x, y, z, tp);
        cbb = cb_index(g, x, y, z, tm);
        const bool eta = ((x + y + z) & 1);
        nf = eta ^ (t == g.nt - 1);  // antiperiodic time boundary
        nb = eta ^ (t == 0);
    }
}

// Neighbours at distance 3 and the signs of the three-link paths to them.
// eta_mu does not depend on x_mu, so a path carries eta_mu(x) once; each of
// its links that leaves the last time slice adds a factor -1: the forward
// path from t crosses floor((t+3)/Nt) times, the backward path (from t-3 to
// t) 3 - floor((t-3+3Nt)/Nt) times, for any even Nt >= 2.
__device__ __forceinline__ int wrap_p3(int v, int n) {
    v += 3;
    v -= (v >= n) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}
__device__ __forceinline__ int wrap_m3(int v, int n) {
    v -= 3;
    v += (v < 0) ? n : 0;
    v += (v < 0) ? n : 0;
    return v;
}
__device__ __forceinline__ void hop3_geometry(const Geom& g, int mu, int x, int y, int z, int t, int& cbf,
                                              int& cbb, bool& nf, bool& nb) {
    if (mu == 0) {
        cbf = cb_index(g, wrap_p3(x, g.nx), y, z, t);
        cbb = cb_index(g, wrap_m3(x, g.nx), y, z, t);
        nf = nb = false;
    } else if (mu == 1) {
        cbf = cb_index(g, x, wrap_p3(y, g.ny), z, t);
        cbb = cb_index(g, x, wrap_m3(y, g.ny), z, t);
        nf = nb = (x & 1);
    } else if (mu == 2) {
        cbf = cb_index(g, x, y, wrap_p3(z, g.nz), t);
        cbb = cb_index(g, x, y, wrap_m3(z, g.nz), t);
        nf = nb = ((x + y) & 1);
    } else {
        cbf = cb_index(g, x, y, z, wrap_p3(t, g.nt));
        cbb = cb_index(g, x, y, z, wrap_m3(t, g.nt));
        const bool eta = ((x + y + z) & 1);
        nf = eta ^ (((t + 3) / g.nt) & 1);
        nb = eta ^ ((3 - (t - 3 + 3 * g.nt) / g.nt) & 1);
    }
}

// acc += wf * U psi_f - wb * U'^dag psi_b for one direction: U is the link
// (or long link) leaving the output site (parity out_par, index cb), U' the
// one arriving from the backward neighbour cbb (which also indexes psi_b).
template <class Link>
__device__ __forceinline__ void hop_w(const Geom& g, const Link& L, const typename Link::C* __restrict__ in,
                                      int out_par, int mu, int cb, int cbf, int cbb, typename Link::R wf,
                                      typename Link::R wb, typename Link::C (&acc)[3]) {
    using C = typename Link::C;
    C U[9], W[9], pf[3], pb[3];
    L.load(g, out_par, mu, cb, U);
#pragma unroll
    for (int c = 0; c < 3; ++c) pf[c] = in[(size_t)c * g.vh + cbf];
    L.load(g, 1 - out_par, mu, cbb, W);
#pragma unroll
    for (int c = 0; c < 3; ++c) pb[c] = in[(size_t)c * g.vh + cbb];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C f = cmul(U[3 * a], pf[0]);
        f = cadd(f, cmul(U[3 * a + 1], pf[1]));
        f = cadd(f, cmul(U[3 * a + 2], pf[2]));
        C b = cmulc(W[a], pb[0]);
        b = cadd(b, cmulc(W[3 + a], pb[1]));
        b = cadd(b, cmulc(W[6 + a], pb[2]));
        acc[a].x += wf * f.x - wb * b.x;
        acc[a].y += wf * f.y - wb * b.y;
    }
}

// The improved operator: one-hop links and long links in the same storage
// format, and the weights of the two stencils.
template <class Link>
struct NaikOp {
    using C = typename Link::C;
    using R = typename Link::R;
    Link one, three;
    double c1, c3;
};

// acc += sf * U psi_f - sb * U'^dag psi_b for one direction
template <class Link>
__device__ __forceinline__ void hop(const Geom& g, const Link& L, const typename Link::C* __restrict__ in, int out_par,
                                    int mu, int cb, int x, int y, int z, int t, typename Link::C (&acc)[3]) {
    using C = typename Link::C;
    using R = typename Link::R;
    int cbf, cbb;
    bool nf, nb;
    hop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
    C U[9], W[9], pf[3], pb[3];
    L.load(g, out_par, mu, cb, U);
#pragma unroll
    for (int c = 0; c < 3; ++c) pf[c] = in[(size_t)c * g.vh + cbf];
    L.load(g, 1 - out_par, mu, cbb, W);
#pragma unroll
    for (int c = 0; c < 3; ++c) pb[c] = in[(size_t)c * g.vh + cbb];
    const R sf = nf ? R(-1) : R(1);  // sign of the forward link
    const R sb = nb ? R(-1) : R(1);  // sign of the backward link (its term is subtracted)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C f = cmul(U[3 * a], pf[0]);
        f = cadd(f, cmul(U[3 * a + 1], pf[1]));
        f = cadd(f, cmul(U[3 * a + 2], pf[2]));
        C b = cmulc(W[a], pb[0]);
        b = cadd(b, cmulc(W[3 + a], pb[1]));
        b = cadd(b, cmulc(W[6 + a], pb[2]));
        acc[a].x += sf * f.x - sb * b.x;
        acc[a].y += sf * f.y - sb * b.y;
    }
}

template <class Link>
__device__ __forceinline__ void hop(const Geom& g, const NaikOp<Link>& op, const typename Link::C* __restrict__ in,
                                    int out_par, int mu, int cb, int x, int y, int z, int t,
                                    typename Link::C (&acc)[3]) {
    using R = typename Link::R;
    int cbf, cbb;
    bool nf, nb;
    hop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
    const R c1 = (R)op.c1, c3 = (R)op.c3;
    hop_w(g, op.one, in, out_par, mu, cb, cbf, cbb, nf ? -c1 : c1, nb ? -c1 : c1, acc);
    hop3_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
    hop_w(g, op.three, in, out_par, mu, cb, cbf, cbb, nf ? -c3 : c3, nb ? -c3 : c3, acc);
}

// ---- epilogues: called once per (colour, site) item with the hopping sum v
template <class C>
struct EpiStore {
    static constexpr int K = 0;
    C* out;
    int vh;
    __device__ void item(int site, int c, C v, double*) const { out[(size_t)c * vh + site] = v; }
    __device__ void finish(double*) const {}
};

// out = coef * in - v   (A = 4m^2 - D_eo D_oe when v = D_eo D_oe in)
template <class C>
struct EpiAxpy {
    static constexpr int K = 0;
    C* out;
    const C* in;
    double coef;
    int vh;
    __device__ void item(int site, int c, C v, double*) const {
        const size_t i = (size_t)c * vh + site;
        const C a = in[i];
        out[i] = C{(decltype(a.x))(coef * a.x - v.x), (decltype(a.y))(coef * a.y - v.y)};
    }
    __device__ void finish(double*) const {}
};

// Ap = mt p - v with the block partials of <p,Ap>, <r,Ap>, <Ap,Ap> in FP64;
// the multi-shift step kernel turns them into the iteration's scalars.
template <class C>
struct EpiCG {
    static constexpr int K = 3;
    C* Ap;
    const C* p;
    const C* r;
    double* part;
    double mt;  // 4m^2 + sigma_0
    int vh;
    __device__ void item(int site, int c, C v, double* acc) const {
        const size_t i = (size_t)c * vh + site;
        const C pv = p[i], rv = r[i];
        using R = decltype(pv.x);
        const R m = (R)mt;
        const C a = C{m * pv.x - v.x, m * pv.y - v.y};
        Ap[i] = a;
        const double2 pd = to_d2(pv), rd = to_d2(rv), ad = to_d2(a);
        acc[0] += pd.x * ad.x + pd.y * ad.y;
        acc[1] += rd.x * ad.x + rd.y * ad.y;
        acc[2] += ad.x * ad.x + ad.y * ad.y;
    }
    __device__ void finish(double* acc) const {
        double v[3] = {acc[0], acc[1], acc[2]};
        block_partial<3>(v, part);
    }
};

// FP64 residual res = b - (coef x - v): block partials of |res|^2, and
// optionally res itself stored in precision Out (reliable updates).
template <class Out>
struct EpiResid {
    static constexpr int K = 1;
    const double2* x;
    const double2* b;
    Out* rout;
    double* part;
    double coef;
    int vh;
    __device__ void item(int site, int c, double2 v, double* acc) const {
        const size_t i = (size_t)c * vh + site;
        const double2 xv = x[i], bv = b[i];
        const double rx = bv.x - (coef * xv.x - v.x), ry = bv.y - (coef * xv.y - v.y);
        if (rout) rout[i] = from_d2<Out>(make_double2(rx, ry));
        acc[0] += rx * rx + ry * ry;
    }
    __device__ void finish(double* acc) const {
        double v[1] = {acc[0]};
        block_partial<1>(v, part);
    }
};

template <int TPS, class Link, class Epi>
__global__ __launch_bounds__(kBlock) void k_dslash(Geom g, Link L, const typename Link::C* __restrict__ in,
                                                   int out_par, Epi epi, const int* __restrict__ gate) {
    using C = typename Link::C;
    constexpr int SB = kBlock / TPS;
    constexpr int DPT = 4 / TPS;
    if (gate && *gate) return;  // converged solve: the whole grid skips
    __shared__ C part[TPS * 3 * SB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slice = wave % TPS, sgrp = wave / TPS;
    const int j = sgrp * 64 + lane;
    const int tile = xcd_tile_slab(blockIdx.x, gridDim.x, g, SB);
    const int cb = tile * SB + j;
    C acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = C{0, 0};
    if (cb < g.vh) {
        int x, y, z, t;
        cb_coords(g, out_par, cb, x, y, z, t);
#pragma unroll
        for (int d = 0; d < DPT; ++d) hop(g, L, in, out_par, slice * DPT + d, cb, x, y, z, t, acc);
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
        C v = part[c * SB + jj];
#pragma unroll
        for (int s = 1; s < TPS; ++s) v = cadd(v, part[(s * 3 + c) * SB + jj]);
        epi.item(site, c, v, racc);
    }
    epi.finish(racc);
}

template <class Link, class Epi>
void launch_tps(const Geom& g, const Link& L, const typename Link::C* in, int out_par, const Epi& epi, int tps,
                const int* gate, hipStream_t s) {
    const int grid = dslash_grid(g, tps);
    switch (tps) {
        case 1: timed_launch(k_dslash<1, Link, Epi>, dim3(grid), dim3(kBlock), s, g, L, in, out_par, epi, gate); break;
        case 2: timed_launch(k_dslash<2, Link, Epi>, dim3(grid), dim3(kBlock), s, g, L, in, out_par, epi, gate); break;
        default: timed_launch(k_dslash<4, Link, Epi>, dim3(grid), dim3(kBlock), s, g, L, in, out_par, epi, gate); break;
    }
}

// dispatch on the storage format of the operator and on the improvement
template <class Fn>
void with_link64(const LinkSet& ls, Fn fn) {
    if (ls.naik) {
        if (ls.fmt64 == STAG_LINKS_F64_12)
            fn(NaikOp<LinkD12>{LinkD12{ls.d12}, LinkD12{ls.ld12}, ls.c1, ls.c3});
        else
            fn(NaikOp<LinkD18>{LinkD18{ls.d18}, LinkD18{ls.ld18}, ls.c1, ls.c3});
    } else if (ls.fmt64 == STAG_LINKS_F64_12) {
        fn(LinkD12{ls.d12});
    } else {
        fn(LinkD18{ls.d18});
    }
}
template <class Fn>
void with_link32(const LinkSet& ls, Fn fn) {
    if (ls.naik) {
        if (ls.fmt32 == STAG_LINKS_F16_12)
            fn(NaikOp<LinkH12>{LinkH12{(const __half2*)ls.h12}, LinkH12{(const __half2*)ls.lh12}, ls.c1, ls.c3});
        else
            fn(NaikOp<LinkS18>{LinkS18{ls.s18}, LinkS18{ls.ls18}, ls.c1, ls.c3});
    } else if (ls.fmt32 == STAG_LINKS_F16_12) {
        fn(LinkH12{(const __half2*)ls.h12});
    } else {
        fn(LinkS18{ls.s18});
    }
}

}  // namespace

int dslash_grid(const Geom& g, int tps) {
    const int sb = kBlock / (tps == 1 ? 1 : (tps == 2 ? 2 : 4));
    return (g.vh + sb - 1) / sb;
}

// ---- FP64 operator
void launch_dslash(const Geom& g, const LinkSet& ls, const double2* in, double2* out, int out_par, int tps,
                   const int* gate, hipStream_t s) {
    with_link64(ls, [&](auto L) { launch_tps(g, L, in, out_par, EpiStore<double2>{out, g.vh}, tps, gate, s); });
}

void launch_dslash_axpy(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* in, double c,
                        double2* out, int tps, hipStream_t s) {
    with_link64(ls, [&](auto L) { launch_tps(g, L, w_o, 0, EpiAxpy<double2>{out, in, c, g.vh}, tps, nullptr, s); });
}

void launch_dslash_cg(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* p, const double2* r,
                      double2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mass_term) {
    with_link64(ls, [&](auto L) {
        launch_tps(g, L, w_o, 0, EpiCG<double2>{Ap, p, r, dpart, mass_term, g.vh}, tps, gate, s);
    });
}

void launch_dslash_resid(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* x, const double2* b,
                         double c, double* part, int tps, hipStream_t s, float2* r32_out) {
    with_link64(ls, [&](auto L) {
        if (r32_out)
            launch_tps(g, L, w_o, 0, EpiResid<float2>{x, b, r32_out, part, c, g.vh}, tps, nullptr, s);
        else
            launch_tps(g, L, w_o, 0, EpiResid<double2>{x, b, nullptr, part, c, g.vh}, tps, nullptr, s);
    });
}

// ---- FP32 (sloppy) operator
void launch_dslash32(const Geom& g, const LinkSet& ls, const float2* in, float2* out, int out_par, int tps,
                     const int* gate, hipStream_t s) {
    with_link32(ls, [&](auto L) { launch_tps(g, L, in, out_par, EpiStore<float2>{out, g.vh}, tps, gate, s); });
}

void launch_dslash32_cg(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* p, const float2* r,
                        float2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mass_term) {
    with_link32(ls, [&](auto L) {
        launch_tps(g, L, w_o, 0, EpiCG<float2>{Ap, p, r, dpart, mass_term, g.vh}, tps, gate, s);
    });
}

void launch_dslash32_axpy(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* in, double c,
                          float2* out, int tps, hipStream_t s) {
    with_link32(ls, [&](auto L) { launch_tps(g, L, w_o, 0, EpiAxpy<float2>{out, in, c, g.vh}, tps, nullptr, s); });
}

}  // namespace stag
