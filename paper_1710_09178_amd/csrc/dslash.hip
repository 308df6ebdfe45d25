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
#include "msfused.h"

namespace stag {

namespace {

template <class C>
__device__ __forceinline__ void rebuild_row2(C (&m)[9]) {
    m[6] = cconj(csub(cmul(m[1], m[5]), cmul(m[2], m[4])));
    m[7] = cconj(csub(cmul(m[2], m[3]), cmul(m[0], m[5])));
    m[8] = cconj(csub(cmul(m[0], m[4]), cmul(m[1], m[3])));
}

// FP64 link entry; NT: a non-temporal load, for link fields larger than the
// Infinity Cache, which every Dslash streams once from HBM: they then do not
// evict the vectors the neighbours share.
template <bool NT>
__device__ __forceinline__ double2 link_entry(const double2* p) {
    if constexpr (NT) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v t = __builtin_nontemporal_load((const d2v*)p);
        return make_double2(t.x, t.y);
    } else {
        return *p;
    }
}

template <bool NT>
struct LinkD18T {
    using C = double2;
    using R = double;
    const double2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const double2* p = u + link_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = link_entry<NT>(p + (size_t)e * g.vh);
    }
};
using LinkD18 = LinkD18T<false>;

template <bool NT>
struct LinkD12T {
    using C = double2;
    using R = double;
    const double2* __restrict__ u;
    __device__ __forceinline__ void load(const Geom& g, int par, int mu, int cb, C (&m)[9]) const {
        const double2* p = u + link12_off(g, par, mu, 0) + cb;
#pragma unroll
        for (int e = 0; e < 6; ++e) m[e] = link_entry<NT>(p + (size_t)e * g.vh);
        rebuild_row2(m);
    }
};
using LinkD12 = LinkD12T<false>;

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
// `in` is the input vector: a pointer, or an accessor that forms each element
// where it is read (the fused multi-shift iteration).
template <class Link, class In>
__device__ __forceinline__ void hop_w(const Geom& g, const Link& L, In in, int out_par, int mu, int cb, int cbf,
                                      int cbb, typename Link::R wf, typename Link::R wb,
                                      typename Link::C (&acc)[3]) {
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
template <class Link, class In>
__device__ __forceinline__ void hop(const Geom& g, const Link& L, In in, int out_par, int mu, int cb, int x, int y,
                                    int z, int t, typename Link::C (&acc)[3]) {
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

template <class Link, class In>
__device__ __forceinline__ void hop(const Geom& g, const NaikOp<Link>& op, In in, int out_par, int mu, int cb, int x,
                                    int y, int z, int t, typename Link::C (&acc)[3]) {
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

// p_j = (r_{j-1} - alpha Ap_{j-1}) + beta p_{j-1}, formed where it is read
template <class V>
struct InUpd {
    const V* __restrict__ r;
    const V* __restrict__ a;
    const V* __restrict__ p;
    double alpha, beta;
    __device__ __forceinline__ V operator[](size_t i) const {
        return cg_p_next(cg_r_next(r[i], a[i], alpha), p[i], beta);
    }
};

// Iteration j of the fused multi-shift CG: w = D_oe p_j for the odd
// sites of this block's tile, after
//   * summing the partials of |r_{j-1}|^2 and of the three D_eo(j-1) dots in
//     block order (every block, bitwise alike) and evaluating step j-1's
//     scalars (fused_step_scalars; block 0 writes the state),
//   * forming p_j at every neighbour from r_{j-1}, Ap_{j-1}, p_{j-1};
// then the even sites with the tile's indices get r_j (ring slot j % L),
// p_j (the other p buffer), x_base += alpha p_{j-1}, and the block partial of
// |r_j|^2.  FIRST (j = 0): D_oe p_0 and the partials of |r_0|^2 only.  A
// stopped solve (flag done[par]) skips the launch and carries the flag.
//
// The loop serves lattices whose grid is a few hundred blocks, where an
// iteration is a chain of dependent memory round trips rather than a
// bandwidth budget.  So one wave per direction (4 threads per site), and
// every load that does not depend on the step's scalars -- the partials, the
// state, both links, the neighbours' r, Ap, p and the owned site's r, Ap, p,
// x_base -- is issued before the scalars are formed: one round trip before
// the arithmetic instead of four.  (The improved operator's 16 links take the
// plain order: scalars first, operands after.)
template <class Link>
struct is_naik_op {
    static constexpr bool value = false;
};
template <class Link>
struct is_naik_op<NaikOp<Link>> {
    static constexpr bool value = true;
};

template <class Link, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_dslash_fused(Geom g, Link L, FusedIterT<typename Link::C> f,
                                                         typename Link::C* __restrict__ w_out) {
    // C: the Krylov vectors' precision, that of the operator's format (FP64
    // links with FP64 vectors, FP32 or FP16 links with FP32 vectors); the
    // scalars, the update arithmetic, x_base and the partial sums are FP64
    using C = typename Link::C;
    using R = typename Link::R;
    constexpr int TPS = 4, SB = kBlock / TPS;
    MsState* st = f.st;
    // the stop flag is tested once this launch's other loads are in flight
    // (a stopped solve's queued launches pay one round trip for them)
    const int stopped = FIRST ? 0 : st->done[f.par];
    __shared__ C part[TPS * 3 * SB];
    __shared__ double lds[16];
    const C* r_prev = f.ring + (size_t)f.slot_prev * 3 * g.vh;
    const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
    const int tile = xcd_tile_slab(blockIdx.x, gridDim.x, g, SB);
    const int cb = tile * SB + lane;
    const bool site_ok = cb < g.vh;
    int x = 0, y = 0, z = 0, t = 0, cbf = 0, cbb = 0;
    bool nf = false, nb = false;
    if (site_ok) {
        cb_coords(g, 1, cb, x, y, z, t);
        hop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
    }
    // the owned even site (colour c, index site) of this thread: 3 SB = 192 of the 256 threads
    const int oc = threadIdx.x / SB, osite = tile * SB + (threadIdx.x % SB);
    const bool own = threadIdx.x < 3 * SB && osite < g.vh;
    const size_t oi = (size_t)oc * g.vh + osite;
    C acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = C{0, 0};
    double alpha = 0.0, beta = 0.0;
    int base_on = 0;
    C o_r = {0, 0}, o_a = {0, 0}, o_p = {0, 0};
    double2 o_x = {0, 0};
    if (FIRST) {
        if (site_ok) hop(g, L, f.p_prev, 1, mu, cb, x, y, z, t, acc);
        if (own) o_r = r_prev[oi];
    } else {
        // the fused loop runs on grids of at most 512 blocks, whose partials
        // two loads per thread and array cover (a larger grid adds the rest
        // in the loop below); more unconditional loads would only repeat the
        // clamped last index
        constexpr int kU = 2;
        const int nb2 = f.nb2;
        double tq[kU], t1[kU], t2[kU], t3[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int b = min((int)threadIdx.x + u * kBlock, nb2 - 1);
            tq[u] = f.qin[b];
            t1[u] = f.dpart[b];
            t2[u] = f.dpart[nb2 + b];
            t3[u] = f.dpart[2 * nb2 + b];
        }
        const LaneState lst = load_lane_state(f);
        if (own) {
            o_r = r_prev[oi];
            o_a = f.Ap[oi];
            o_p = f.p_prev[oi];
            o_x = f.x_base[oi];
        }
        // hop operands (plain links): both links and the neighbours' r, Ap, p
        C U[9], W[9], fr[3], fa[3], fp[3], br[3], ba[3], bp[3];
        if constexpr (!is_naik_op<Link>::value) {
            if (site_ok) {
                L.load(g, 1, mu, cb, U);
                L.load(g, 0, mu, cbb, W);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const size_t jf = (size_t)c * g.vh + cbf, jb = (size_t)c * g.vh + cbb;
                    fr[c] = r_prev[jf];
                    fa[c] = f.Ap[jf];
                    fp[c] = f.p_prev[jf];
                    br[c] = r_prev[jb];
                    ba[c] = f.Ap[jb];
                    bp[c] = f.p_prev[jb];
                }
            }
        }
        if (stopped) {
            if (blockIdx.x == 0 && threadIdx.x == 0) st->done[f.par ^ 1] = 1;
            return;
        }
        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if ((int)threadIdx.x + u * kBlock < nb2) {
                v[0] += tq[u];
                v[1] += t1[u];
                v[2] += t2[u];
                v[3] += t3[u];
            }
        for (int b = threadIdx.x + kU * kBlock; b < nb2; b += kBlock) {
            v[0] += f.qin[b];
            v[1] += f.dpart[b];
            v[2] += f.dpart[nb2 + b];
            v[3] += f.dpart[2 * nb2 + b];
        }
        block_sum<4>(v, lds);
        const StepOut so = fused_step_scalars(f, v, lst);
        if (so.stop) return;
        alpha = so.alpha;
        beta = so.beta;
        base_on = so.base_on;
        if (site_ok) {
            if constexpr (is_naik_op<Link>::value) {
                const InUpd<C> in{r_prev, f.Ap, f.p_prev, alpha, beta};
                hop(g, L, in, 1, mu, cb, x, y, z, t, acc);
            } else {
                C pf[3], pb[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pf[c] = cg_p_next(cg_r_next(fr[c], fa[c], alpha), fp[c], beta);
                    pb[c] = cg_p_next(cg_r_next(br[c], ba[c], alpha), bp[c], beta);
                }
                const R sf = nf ? R(-1) : R(1), sb = nb ? R(-1) : R(1);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    C fv = cmul(U[3 * a], pf[0]);
                    fv = cadd(fv, cmul(U[3 * a + 1], pf[1]));
                    fv = cadd(fv, cmul(U[3 * a + 2], pf[2]));
                    C bv = cmulc(W[a], pb[0]);
                    bv = cadd(bv, cmulc(W[3 + a], pb[1]));
                    bv = cadd(bv, cmulc(W[6 + a], pb[2]));
                    acc[a].x += sf * fv.x - sb * bv.x;
                    acc[a].y += sf * fv.y - sb * bv.y;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) part[(mu * 3 + c) * SB + lane] = acc[c];
    __syncthreads();
    double racc[1] = {0.0};
    if (own) {
        const int jj = threadIdx.x % SB;
        C v = part[oc * SB + jj];
#pragma unroll
        for (int sl = 1; sl < TPS; ++sl) v = cadd(v, part[(sl * 3 + oc) * SB + jj]);
        w_out[oi] = v;
        if (FIRST) {
            const double2 rd = to_d2(o_r);
            racc[0] = rd.x * rd.x + rd.y * rd.y;
        } else {
            const C rn = cg_r_next(o_r, o_a, alpha);
            f.ring[(size_t)f.slot_new * 3 * g.vh + oi] = rn;
            const double2 rd = to_d2(rn), pd = to_d2(o_p);
            racc[0] = rd.x * rd.x + rd.y * rd.y;
            if (base_on) f.x_base[oi] = make_double2(fma(alpha, pd.x, o_x.x), fma(alpha, pd.y, o_x.y));
            f.p_new[oi] = cg_p_next(rn, o_p, beta);
        }
    }
    block_partial<1>(racc, f.qout);
}

// D_eo launch of the fused loop: Ap = mt p - D_eo w and the block partials of
// <p,Ap>, <r,Ap>, <Ap,Ap> (the arithmetic of the EpiCG epilogue), with 4
// threads per site and every load -- links, the neighbours' w, the owned
// site's p and r -- issued before the stop flag is tested.
template <class Link>
__global__ __launch_bounds__(kBlock) void k_dslash_cg_fused(Geom g, Link L, const typename Link::C* __restrict__ w,
                                                            const typename Link::C* __restrict__ p,
                                                            const typename Link::C* __restrict__ r,
                                                            typename Link::C* __restrict__ Ap,
                                                            double* __restrict__ part, double mt,
                                                            const int* __restrict__ gate) {
    using C = typename Link::C;
    using R = typename Link::R;
    constexpr int TPS = 4, SB = kBlock / TPS;
    const int stopped = *gate;
    __shared__ C lpart[TPS * 3 * SB];
    const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
    const int tile = xcd_tile_slab(blockIdx.x, gridDim.x, g, SB);
    const int cb = tile * SB + lane;
    const bool site_ok = cb < g.vh;
    int x = 0, y = 0, z = 0, t = 0, cbf = 0, cbb = 0;
    bool nf = false, nb = false;
    if (site_ok) {
        cb_coords(g, 0, cb, x, y, z, t);
        hop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
    }
    const int oc = threadIdx.x / SB, osite = tile * SB + (threadIdx.x % SB);
    const bool own = threadIdx.x < 3 * SB && osite < g.vh;
    const size_t oi = (size_t)oc * g.vh + osite;
    C o_p = {0, 0}, o_r = {0, 0};
    if (own) {
        o_p = p[oi];
        o_r = r[oi];
    }
    C acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = C{0, 0};
    if constexpr (is_naik_op<Link>::value) {
        if (stopped) return;
        if (site_ok) hop(g, L, w, 0, mu, cb, x, y, z, t, acc);
    } else {
        C U[9], W[9], pf[3], pb[3];
        if (site_ok) {
            L.load(g, 0, mu, cb, U);
            L.load(g, 1, mu, cbb, W);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pf[c] = w[(size_t)c * g.vh + cbf];
                pb[c] = w[(size_t)c * g.vh + cbb];
            }
        }
        if (stopped) return;
        if (site_ok) {
            const R sf = nf ? R(-1) : R(1), sb = nb ? R(-1) : R(1);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                C fv = cmul(U[3 * a], pf[0]);
                fv = cadd(fv, cmul(U[3 * a + 1], pf[1]));
                fv = cadd(fv, cmul(U[3 * a + 2], pf[2]));
                C bv = cmulc(W[a], pb[0]);
                bv = cadd(bv, cmulc(W[3 + a], pb[1]));
                bv = cadd(bv, cmulc(W[6 + a], pb[2]));
                acc[a].x += sf * fv.x - sb * bv.x;
                acc[a].y += sf * fv.y - sb * bv.y;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) lpart[(mu * 3 + c) * SB + lane] = acc[c];
    __syncthreads();
    double dots[3] = {0.0, 0.0, 0.0};
    if (own) {
        const int jj = threadIdx.x % SB;
        C v = lpart[oc * SB + jj];
#pragma unroll
        for (int sl = 1; sl < TPS; ++sl) v = cadd(v, lpart[(sl * 3 + oc) * SB + jj]);
        // (the arithmetic of the EpiCG epilogue, in the vectors' precision)
        const R m = (R)mt;
        const C a = C{m * o_p.x - v.x, m * o_p.y - v.y};
        Ap[oi] = a;
        const double2 pd = to_d2(o_p), rd = to_d2(o_r), ad = to_d2(a);
        dots[0] = pd.x * ad.x + pd.y * ad.y;
        dots[1] = rd.x * ad.x + rd.y * ad.y;
        dots[2] = ad.x * ad.x + ad.y * ad.y;
    }
    block_partial<3>(dots, part);
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
template <bool NT, class Fn>
void with_link64_nt(const LinkSet& ls, Fn fn) {
    using D18 = LinkD18T<NT>;
    using D12 = LinkD12T<NT>;
    if (ls.naik) {
        if (ls.fmt64 == STAG_LINKS_F64_12)
            fn(NaikOp<D12>{D12{ls.d12}, D12{ls.ld12}, ls.c1, ls.c3});
        else
            fn(NaikOp<D18>{D18{ls.d18}, D18{ls.ld18}, ls.c1, ls.c3});
    } else if (ls.fmt64 == STAG_LINKS_F64_12) {
        fn(D12{ls.d12});
    } else {
        fn(D18{ls.d18});
    }
}
template <class Fn>
void with_link64(const LinkSet& ls, Fn fn) {
    if (ls.nt)
        with_link64_nt<true>(ls, fn);
    else
        with_link64_nt<false>(ls, fn);
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

// ---- fused multi-shift iteration, 4 threads per site: FP64 (format fmt64)
// or FP32 Krylov vectors (format fmt32)
int dslash_fused_grid(const Geom& g) { return dslash_grid(g, 4); }

namespace {
template <class V, class Disp>
void cg_fused_any(const Geom& g, const LinkSet& ls, Disp disp, const V* w_o, const V* p, const V* r, V* Ap,
                  const int* gate, double* dpart, hipStream_t s, double mass_term) {
    const int grid = dslash_fused_grid(g);
    disp(ls, [&](auto L) {
        timed_launch(k_dslash_cg_fused<decltype(L)>, dim3(grid), dim3(kBlock), s, g, L, w_o, p, r, Ap, dpart,
                     mass_term, gate);
    });
}
template <class V, class Disp>
void fused_any(const Geom& g, const LinkSet& ls, Disp disp, const FusedIterT<V>& f, V* w_out, bool first,
               hipStream_t s) {
    const int grid = dslash_fused_grid(g);
    disp(ls, [&](auto L) {
        using LT = decltype(L);
        if (first)
            k_dslash_fused<LT, true><<<grid, kBlock, 0, s>>>(g, L, f, w_out);
        else
            timed_launch(k_dslash_fused<LT, false>, dim3(grid), dim3(kBlock), s, g, L, f, w_out);
    });
}
struct Disp64 {
    template <class Fn>
    void operator()(const LinkSet& ls, Fn fn) const { with_link64(ls, fn); }
};
struct Disp32 {
    template <class Fn>
    void operator()(const LinkSet& ls, Fn fn) const { with_link32(ls, fn); }
};
}  // namespace

void launch_dslash_cg_fused(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* p, const double2* r,
                            double2* Ap, const int* gate, double* dpart, hipStream_t s, double mass_term) {
    cg_fused_any(g, ls, Disp64{}, w_o, p, r, Ap, gate, dpart, s, mass_term);
}
void launch_dslash_cg_fused(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* p, const float2* r,
                            float2* Ap, const int* gate, double* dpart, hipStream_t s, double mass_term) {
    cg_fused_any(g, ls, Disp32{}, w_o, p, r, Ap, gate, dpart, s, mass_term);
}
void launch_dslash_fused(const Geom& g, const LinkSet& ls, const FusedIterT<double2>& f, double2* w_out, bool first,
                         hipStream_t s) {
    fused_any(g, ls, Disp64{}, f, w_out, first, s);
}
void launch_dslash_fused(const Geom& g, const LinkSet& ls, const FusedIterT<float2>& f, float2* w_out, bool first,
                         hipStream_t s) {
    fused_any(g, ls, Disp32{}, f, w_out, first, s);
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
