// Batched multi-shift CG kernels: every launch covers all tiles of all
// lattices of the batch, and each Dslash thread applies the links it loads to
// every right-hand side of its lattice (links read once per nrhs vectors).
// Scalars are per system (lattice, right-hand side); reductions are per tile
// and are summed over the lattice's tiles by the consuming kernel.
#include <type_traits>

#include "batch.h"

namespace stag {

namespace {

template <class V>
struct BPrec;
template <>
struct BPrec<double2> {
    using R = double;
};
template <>
struct BPrec<float2> {
    using R = float;
};

// a link entry; NT: non-temporal (link fields larger than the Infinity Cache)
template <bool NT>
__device__ __forceinline__ double2 bload(const double2* p) {
    if constexpr (NT) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v t = __builtin_nontemporal_load((const d2v*)p);
        return make_double2(t.x, t.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ float2 bload(const float2* p) {
    if constexpr (NT) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        const f2v t = __builtin_nontemporal_load((const f2v*)p);
        return make_float2(t.x, t.y);
    } else {
        return *p;
    }
}

// An SU(3) matrix's row 2 from rows 0 and 1: conj(row 0 x row 1).  With it
// the operators read 12 of a link's 18 reals (rows 0-1; the storage keeps
// all 9 entries as separate planes, so row 2's planes are simply not read).
template <class V>
__device__ __forceinline__ void brebuild_row2(V (&m)[9]) {
    m[6] = cconj(csub(cmul(m[1], m[5]), cmul(m[2], m[4])));
    m[7] = cconj(csub(cmul(m[2], m[3]), cmul(m[0], m[5])));
    m[8] = cconj(csub(cmul(m[0], m[4]), cmul(m[1], m[3])));
}

__device__ __forceinline__ void bhop_geometry(const Geom& g, int mu, int x, int y, int z, int t, int& cbf, int& cbb,
                                              bool& nf, bool& nb) {
    if (mu == 0) {
        cbf = cb_index(g, (x + 1 == g.nx) ? 0 : x + 1, y, z, t);
        cbb = cb_index(g, (x == 0) ? g.nx - 1 : x - 1, y, z, t);
        nf = nb = false;
    } else if (mu == 1) {
        cbf = cb_index(g, x, (y + 1 == g.ny) ? 0 : y + 1, z, t);
        cbb = cb_index(g, x, (y == 0) ? g.ny - 1 : y - 1, z, t);
        nf = nb = (x & 1);
    } else if (mu == 2) {
        cbf = cb_index(g, x, y, (z + 1 == g.nz) ? 0 : z + 1, t);
        cbb = cb_index(g, x, y, (z == 0) ? g.nz - 1 : z - 1, t);
        nf = nb = ((x + y) & 1);
    } else {
        cbf = cb_index(g, x, y, z, (t + 1 == g.nt) ? 0 : t + 1);
        cbb = cb_index(g, x, y, z, (t == 0) ? g.nt - 1 : t - 1);
        const bool eta = ((x + y + z) & 1);
        nf = eta ^ (t == g.nt - 1);
        nb = eta ^ (t == 0);
    }
}

// ---- epilogues over (rhs, colour, site) items of one tile
template <class V>
struct BEpiStore {
    static constexpr int K = 1;
    V* out;
    __device__ __forceinline__ void item(const BInst& I, int, int R, int rh, int site, int c, V v,
                                         double (&)[K]) const {
        out[bvec_off(I, R, rh, c) + site] = v;
    }
    __device__ __forceinline__ void finish(int, double (&)[K]) const {}
};

// Ap = (4 m_i^2 + sigma_0) p - v and per-rhs partials of <p,Ap>, <r,Ap>, <Ap,Ap>
template <class V>
struct BEpiCG {
    static constexpr int K = 3 * kMaxRhs;
    V* Ap;
    const V* p;
    const V* r;
    const double* sigma0_term;  // [inst] 4 m_i^2 + sigma_0
    double* part;  // [tile][kMaxRhs][3]
    __device__ __forceinline__ void item(const BInst& I, int inst, int R, int rh, int site, int c, V v,
                                         double (&acc)[K]) const {
        const size_t i = bvec_off(I, R, rh, c) + site;
        const V pv = p[i], rv = r[i];
        using Rl = typename BPrec<V>::R;
        const Rl m = (Rl)sigma0_term[inst];
        const V a = V{m * pv.x - v.x, m * pv.y - v.y};
        Ap[i] = a;
        const double2 pd = to_d2(pv), rd = to_d2(rv), ad = to_d2(a);
        const double d0 = pd.x * ad.x + pd.y * ad.y, d1 = rd.x * ad.x + rd.y * ad.y, d2 = ad.x * ad.x + ad.y * ad.y;
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q) {  // selects: no dynamic register indexing
            acc[3 * q + 0] += (q == rh) ? d0 : 0.0;
            acc[3 * q + 1] += (q == rh) ? d1 : 0.0;
            acc[3 * q + 2] += (q == rh) ? d2 : 0.0;
        }
    }
    __device__ __forceinline__ void finish(int tile, double (&acc)[K]) const {
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = acc[k];
        __shared__ double lds[4 * K];
        block_sum<K>(v, lds);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) part[(size_t)tile * K + k] = v[k];
    }
};

// FP64 residual b - ((4 m_i^2 + pole) x - v): per-rhs partials of |res|^2
struct BEpiResid {
    static constexpr int K = kMaxRhs;
    const double2* x;
    const double2* b;
    double2* rout;
    double pole;
    double* part;  // [tile][kMaxRhs]
    __device__ __forceinline__ void item(const BInst& I, int, int R, int rh, int site, int c, double2 v,
                                         double (&acc)[K]) const {
        const size_t i = bvec_off(I, R, rh, c) + site;
        const double coef = I.four_m2 + pole;
        const double2 xv = x[i], bv = b[i];
        const double rx = bv.x - (coef * xv.x - v.x), ry = bv.y - (coef * xv.y - v.y);
        if (rout) rout[i] = make_double2(rx, ry);
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (q == rh) acc[q] += rx * rx + ry * ry;
    }
    __device__ __forceinline__ void finish(int tile, double (&acc)[K]) const {
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = acc[k];
        __shared__ double lds[4 * K];
        block_sum<K>(v, lds);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) part[(size_t)tile * K + k] = v[k];
    }
};

// One block per tile: TPS threads per site split the 4 directions; every
// thread applies its links to all right-hand sides of the lattice.
template <int TPS, class V, class Epi, bool NT, bool L12>
__global__ __launch_bounds__(kBlock) void k_bdslash(BatchDev bd, const V* __restrict__ links, const V* __restrict__ in,
                                                    int out_par, Epi epi, const int* __restrict__ inst_done) {
    constexpr int SB = kBlock / TPS;
    constexpr int DPT = 4 / TPS;
    using Rl = typename BPrec<V>::R;
    const BTile tl = bd.tiles[blockIdx.x];
    if (inst_done && inst_done[tl.inst]) return;
    const BInst I = bd.inst[tl.inst];
    const Geom& g = I.g;
    const int R = bd.nrhs;
    __shared__ V part[TPS * kMaxRhs * 3 * SB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slice = wave % TPS, sgrp = wave / TPS;
    const int j = sgrp * 64 + lane;
    const int cb = tl.cb0 + j;
    V acc[kMaxRhs][3];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][c] = V{0, 0};
    const V* lk = links + blink_base(I);
    if (cb < g.vh) {
        int x, y, z, t;
        cb_coords(g, out_par, cb, x, y, z, t);
#pragma unroll
        for (int d = 0; d < DPT; ++d) {
            const int mu = slice * DPT + d;
            int cbf, cbb;
            bool nf, nb;
            bhop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
            V U[9], W[9];
            const V* uf = lk + link_off(g, out_par, mu, 0) + cb;
            const V* ub = lk + link_off(g, 1 - out_par, mu, 0) + cbb;
            constexpr int NE = L12 ? 6 : 9;
#pragma unroll
            for (int e = 0; e < NE; ++e) U[e] = bload<NT>(uf + (size_t)e * g.vh);
#pragma unroll
            for (int e = 0; e < NE; ++e) W[e] = bload<NT>(ub + (size_t)e * g.vh);
            if constexpr (L12) {
                brebuild_row2(U);
                brebuild_row2(W);
            }
            const Rl sf = nf ? Rl(-1) : Rl(1);
            const Rl sb = nb ? Rl(-1) : Rl(1);
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r) {
                if (r >= R) break;
                V pf[3], pb[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pf[c] = in[bvec_off(I, R, r, c) + cbf];
                    pb[c] = in[bvec_off(I, R, r, c) + cbb];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    V f = cmul(U[3 * a], pf[0]);
                    f = cadd(f, cmul(U[3 * a + 1], pf[1]));
                    f = cadd(f, cmul(U[3 * a + 2], pf[2]));
                    V bb = cmulc(W[a], pb[0]);
                    bb = cadd(bb, cmulc(W[3 + a], pb[1]));
                    bb = cadd(bb, cmulc(W[6 + a], pb[2]));
                    acc[r][a].x += sf * f.x - sb * bb.x;
                    acc[r][a].y += sf * f.y - sb * bb.y;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (r < R) part[((slice * kMaxRhs + r) * 3 + c) * SB + j] = acc[r][c];
    __syncthreads();
    double racc[Epi::K];
#pragma unroll
    for (int k = 0; k < Epi::K; ++k) racc[k] = 0.0;
    for (int it = threadIdx.x; it < R * 3 * SB; it += kBlock) {
        const int rh = it / (3 * SB), c = (it / SB) % 3, jj = it % SB;
        const int site = tl.cb0 + jj;
        if (site >= g.vh) continue;
        V v = part[((0 * kMaxRhs + rh) * 3 + c) * SB + jj];
#pragma unroll
        for (int s = 1; s < TPS; ++s) v = cadd(v, part[((s * kMaxRhs + rh) * 3 + c) * SB + jj]);
        epi.item(I, tl.inst, R, rh, site, c, v, racc);
    }
    epi.finish(blockIdx.x, racc);
}

// Eight lanes per output site, one hop each: lane h takes direction h / 2,
// the forward hop U_mu(x) p(x+mu) for even h and the backward hop
// U_mu(x-mu)^dag p(x-mu) for odd h (its matrix is loaded transposed and
// conjugated, so both kinds run the same arithmetic).  Each lane holds one
// link matrix, the eight partial colour vectors of a site meet by lane
// exchanges (no LDS), and every right-hand side is finished right after its
// exchange: its three (rhs, colour) outputs go to lanes (3 rhs + colour) mod 8.
template <class V, class Epi>
__global__ __launch_bounds__(kBlock) void k_bdslash8(BatchDev bd, const V* __restrict__ links,
                                                     const V* __restrict__ in, int out_par, Epi epi,
                                                     const int* __restrict__ inst_done) {
    using Rl = typename BPrec<V>::R;
    const BTile tl = bd.tiles[blockIdx.x];
    if (inst_done && inst_done[tl.inst]) return;
    const BInst I = bd.inst[tl.inst];
    const Geom& g = I.g;
    const int R = bd.nrhs;
    const int h = threadIdx.x & 7, mu = h >> 1;
    const bool bwd = h & 1;
    const int cb = tl.cb0 + (int)(threadIdx.x >> 3);
    const bool on = cb < g.vh;
    V U[9];
    int nbr = 0;
    Rl sg = 0;
    if (on) {
        int x, y, z, t;
        cb_coords(g, out_par, cb, x, y, z, t);
        int cbf, cbb;
        bool nf, nb;
        bhop_geometry(g, mu, x, y, z, t, cbf, cbb, nf, nb);
        const V* lk = links + blink_base(I);
        const V* u = bwd ? lk + link_off(g, 1 - out_par, mu, 0) + cbb : lk + link_off(g, out_par, mu, 0) + cb;
        const Rl cj = bwd ? Rl(-1) : Rl(1);
        V M[9];
        if (bd.link12) {
#pragma unroll
            for (int e = 0; e < 6; ++e) M[e] = u[(size_t)e * g.vh];
            brebuild_row2(M);
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) M[e] = u[(size_t)e * g.vh];
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const int src = bwd ? 3 * (e % 3) + e / 3 : e;
            U[e] = V{M[src].x, cj * M[src].y};
        }
        nbr = bwd ? cbb : cbf;
        sg = bwd ? (nb ? Rl(1) : Rl(-1)) : (nf ? Rl(-1) : Rl(1));
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) U[e] = V{0, 0};
    }
    double racc[Epi::K];
#pragma unroll
    for (int k = 0; k < Epi::K; ++k) racc[k] = 0.0;
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) {
        if (r >= R) break;
        V pv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) pv[c] = on ? in[bvec_off(I, R, r, c) + nbr] : V{0, 0};
        V a[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            V f = cmul(U[3 * c], pv[0]);
            f = cadd(f, cmul(U[3 * c + 1], pv[1]));
            f = cadd(f, cmul(U[3 * c + 2], pv[2]));
            a[c] = V{sg * f.x, sg * f.y};
        }
#pragma unroll
        for (int m = 1; m < 8; m <<= 1)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[c].x += __shfl_xor(a[c].x, m, 64);
                a[c].y += __shfl_xor(a[c].y, m, 64);
            }
        if (on)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((3 * r + c) % 8 == h) epi.item(I, tl.inst, R, r, cb, c, a[c], racc);
    }
    epi.finish(blockIdx.x, racc);
}

template <class V, class Epi>
void bdslash_tps(const BatchDev& bd, int tps, const V* links, const V* in, int out_par, const Epi& epi,
                 const int* inst_done, hipStream_t s) {
    if (tps == 8) {
        k_bdslash8<V, Epi><<<bd.ntiles, kBlock, 0, s>>>(bd, links, in, out_par, epi, inst_done);
        return;
    }
    auto go = [&](auto nt, auto l12) {
        constexpr bool NT = decltype(nt)::value, L12 = decltype(l12)::value;
        switch (tps) {
            case 1:
                k_bdslash<1, V, Epi, NT, L12><<<bd.ntiles, kBlock, 0, s>>>(bd, links, in, out_par, epi, inst_done);
                break;
            case 2:
                k_bdslash<2, V, Epi, NT, L12><<<bd.ntiles, kBlock, 0, s>>>(bd, links, in, out_par, epi, inst_done);
                break;
            default:
                k_bdslash<4, V, Epi, NT, L12><<<bd.ntiles, kBlock, 0, s>>>(bd, links, in, out_par, epi, inst_done);
                break;
        }
    };
    if (bd.link_nt) {
        if (bd.link12)
            go(std::true_type{}, std::true_type{});
        else
            go(std::true_type{}, std::false_type{});
    } else {
        if (bd.link12)
            go(std::false_type{}, std::true_type{});
        else
            go(std::false_type{}, std::false_type{});
    }
}

// r = p = p_k = b, x_k = 0, per-rhs partials of |b|^2
template <class V>
__global__ __launch_bounds__(kBlock) void k_bms_init(BatchDev bd, const double2* __restrict__ b, V* __restrict__ r,
                                                     V* __restrict__ p, VecPtrs x, VecPtrs ps,
                                                     BState st, double* __restrict__ qout) {
    const BTile tl = bd.tiles[blockIdx.x];
    const BInst I = bd.inst[tl.inst];
    const int R = bd.nrhs, SB = bd.tile_sites;
    const int n = st.n, base = st.base;
    double acc[kMaxRhs] = {0.0, 0.0, 0.0, 0.0};
    for (int it = threadIdx.x; it < R * 3 * SB; it += kBlock) {
        const int rh = it / (3 * SB), c = (it / SB) % 3, jj = it % SB;
        const int site = tl.cb0 + jj;
        if (site >= I.g.vh) continue;
        const size_t i = bvec_off(I, R, rh, c) + site;
        const double2 bv = b[i];
        const V bl = from_d2<V>(bv);
        r[i] = bl;
        p[i] = bl;
        for (int k = 0; k < n; ++k) {
            x.at<double2>(k)[i] = make_double2(0.0, 0.0);
            if (k != base) ps.at<V>(k)[i] = bl;
        }
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (q == rh) acc[q] += bv.x * bv.x + bv.y * bv.y;
    }
    __shared__ double lds[4 * kMaxRhs];
    block_sum<kMaxRhs>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kMaxRhs; ++q) qout[(size_t)blockIdx.x * kMaxRhs + q] = acc[q];
}

// Scalars of system s from this iteration's sums (one thread per system).
// The shifted updates are deferred over windows of st.lag iterations as in
// the single-lattice solver: the scalars of each iteration go to the
// system's history, and the window's last iteration (or the stopping one)
// applies them in order.  w_*: this system's [lag][n] window tables.  Also
// writes the system's state for the next iteration (or the final one).
__device__ void bsystem_scalars(BState& st, int s, int par, double rr, double pAp, double rAp, double ApAp,
                                BScal& o, double* w_as, double* w_bs, double* w_zn, int* w_act) {
    const int n = st.n, base = st.base, L = st.lag;
    const MsIter& S = st.it[par][s];
    const int iter = S.iter;
    const int slot = iter % L;
    const double bb = (iter == 0 && !st.bb_given) ? rr : S.bb;
    int nonfinite = !isfinite(rr);
    int any = 0;
    for (int k = 0; k < n; ++k) {
        const int a = S.active[k] && !(S.zeta[k] * S.zeta[k] * rr <= st.tol2 * bb);
        w_act[slot * n + k] = a;
        any |= a;
    }
    int stop = nonfinite || !any || iter >= st.maxiter;
    double alpha = 0.0, beta = 0.0;
    if (!stop) {
        alpha = rr / pAp;
        double rr1 = rr - 2.0 * alpha * rAp + alpha * alpha * ApAp;
        if (rr1 < 0.0) rr1 = 0.0;
        beta = rr1 / rr;
        if (!isfinite(alpha) || !isfinite(beta)) {
            nonfinite = 1;
            stop = 1;
        }
    }
    const double a_old = S.alpha_old, b_old = S.beta_old;
    for (int k = 0; k < n; ++k) {
        const double z = S.zeta[k], zo = S.zeta_old[k];
        double zn = z, as = 0.0, bs = 0.0;
        if (!stop) {
            if (k == base) {
                zn = 1.0;
                as = alpha;
                bs = beta;
            } else if (w_act[slot * n + k]) {
                zn = z * zo * a_old / (alpha * b_old * (zo - z) + zo * a_old * (1.0 + st.shift[k] * alpha));
                const double q = zn / z;
                as = alpha * q;
                bs = beta * q * q;
            }
        }
        w_as[slot * n + k] = as;
        w_bs[slot * n + k] = bs;
        w_zn[slot * n + k] = zn;
    }
    const int npend = stop ? slot : slot + 1;
    const int flush = npend > 0 && (stop || slot == L - 1);
    if (flush)
        for (int t = 0; t < slot; ++t)
            for (int k = 0; k < n; ++k) {
                const MsHist& h = st.hist[(size_t)s * kLagMax + t];
                w_as[t * n + k] = h.as[k];
                w_bs[t * n + k] = h.bs[k];
                w_zn[t * n + k] = h.zn[k];
                w_act[t * n + k] = h.act[k];
            }
    o.alpha = alpha;
    o.beta = beta;
    o.stop = stop;
    o.flush = flush;
    o.npend = npend;
    o.slot = slot;
    o.base_on = !stop && w_act[slot * n + base];
    int m = 0;
    if (flush)
        for (int k = 0; k < n; ++k)
            if (k != base && w_act[k]) o.list[m++] = k;  // active at the window's first iteration
    o.nact = m;
    {
        MsIter& N = stop ? st.fin[s] : st.it[par ^ 1][s];
        for (int k = 0; k < n; ++k) {
            const int a = stop ? 0 : w_act[slot * n + k];
            N.active[k] = w_act[slot * n + k];
            N.iters_per_pole[k] = (a && !stop) ? iter + 1 : (S.active[k] ? iter : S.iters_per_pole[k]);
            N.zeta[k] = stop ? S.zeta[k] : w_zn[slot * n + k];
            N.zeta_old[k] = stop ? S.zeta_old[k] : S.zeta[k];
            if (!stop && !flush) {
                MsHist& h = st.hist[(size_t)s * kLagMax + slot];
                h.as[k] = w_as[slot * n + k];
                h.bs[k] = w_bs[slot * n + k];
                h.zn[k] = w_zn[slot * n + k];
                h.act[k] = w_act[slot * n + k];
            }
        }
        N.alpha_old = stop ? S.alpha_old : alpha;
        N.beta_old = stop ? S.beta_old : beta;
        N.bb = bb;
        N.rr = rr;
        N.iter = stop ? iter : iter + 1;
        N.nonfinite = nonfinite;
        if (stop) {
            st.sys_done[(size_t)(par ^ 1) * st.n_inst * st.nrhs + s] = 1;
            st.t_done[s] = wall_clock64();
        }
    }
}

// One block per instance: the sums over the instance's tiles (in tile
// order) and the scalars of its systems, evaluated once per iteration instead
// of in every tile of the step.  Reads the stop flags of parity par and
// writes those of par ^ 1.
__global__ __launch_bounds__(kBlock) void k_bms_scalars(BatchDev bd, BState st, const double* __restrict__ dpart,
                                                        const double* __restrict__ qin, int par) {
    const int inst = blockIdx.x;
    const int* done_in = st.inst_done + par * st.n_inst;
    int* done_out = st.inst_done + (par ^ 1) * st.n_inst;
    if (done_in[inst]) {
        if (threadIdx.x == 0) done_out[inst] = 1;
        return;
    }
    const BInst I = bd.inst[inst];
    const int R = bd.nrhs;
    __shared__ double lds[4 * 4 * kMaxRhs];
    __shared__ int sh_stop[kMaxRhs];
    // sums over the lattice's tiles: [rhs] rr, [rhs][3] dots
    double v[4 * kMaxRhs];
#pragma unroll
    for (int k = 0; k < 4 * kMaxRhs; ++k) v[k] = 0.0;
    for (int t = I.tile0 + threadIdx.x; t < I.tile0 + I.ntiles; t += kBlock) {
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q) {
            v[4 * q + 0] += qin[(size_t)t * kMaxRhs + q];
            v[4 * q + 1] += dpart[(size_t)t * 3 * kMaxRhs + 3 * q + 0];
            v[4 * q + 2] += dpart[(size_t)t * 3 * kMaxRhs + 3 * q + 1];
            v[4 * q + 3] += dpart[(size_t)t * 3 * kMaxRhs + 3 * q + 2];
        }
    }
    block_sum<4 * kMaxRhs>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4 * kMaxRhs; ++k) lds[k] = v[k];
    }
    __syncthreads();
    // stopped before this launch; a stop in this launch is written to the other parity
    const int* sys_in = st.sys_done + (size_t)par * st.n_inst * R;
    int* sys_out = st.sys_done + (size_t)(par ^ 1) * st.n_inst * R;
    if (threadIdx.x < R) {
        const int q = threadIdx.x;
        const int s = inst * R + q;
        BScal& o = st.scal[s];
        if (sys_in[s]) {
            sys_out[s] = 1;
            o.stop = 1;
            o.flush = 0;
            o.nact = 0;
            o.base_on = 0;
            sh_stop[q] = 1;
        } else {
            double* wt = st.w_tab + (size_t)s * 3 * kWinTab;
            bsystem_scalars(st, s, par, lds[4 * q], lds[4 * q + 1], lds[4 * q + 2], lds[4 * q + 3], o, wt,
                            wt + kWinTab, wt + 2 * kWinTab, st.w_act + (size_t)s * kWinTab);
            sh_stop[q] = o.stop;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int all = 1;
        for (int q = 0; q < R; ++q) all &= sh_stop[q];
        if (all) done_out[inst] = 1;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_bms_step(BatchDev bd, V* __restrict__ ring, const V* __restrict__ Ap,
                                                     V* __restrict__ p, VecPtrs x, VecPtrs ps, BState st,
                                                     double* __restrict__ qout, int par) {
    const BTile tl = bd.tiles[blockIdx.x];
    if (st.inst_done[par * st.n_inst + tl.inst]) return;
    const BInst I = bd.inst[tl.inst];
    const int R = bd.nrhs, SB = bd.tile_sites, n = st.n, L = st.lag;
    __shared__ BScal sc[kMaxRhs];
    __shared__ double lds[4 * kMaxRhs];
    // window tables [rhs][lag][n]: as, bs, zn (double) then act (int)
    extern __shared__ double wdyn[];
    const int wsz = L * n;
    double* w_as = wdyn;
    double* w_bs = w_as + kMaxRhs * wsz;
    double* w_zn = w_bs + kMaxRhs * wsz;
    int* w_act = (int*)(w_zn + kMaxRhs * wsz);
    {
        constexpr int words = (int)(sizeof(BScal) / sizeof(int));
        const int* src = (const int*)(st.scal + (size_t)tl.inst * R);
        int* dst = (int*)sc;
        for (int w = threadIdx.x; w < R * words; w += kBlock) dst[w] = src[w];
    }
    __syncthreads();
    int anyflush = 0;
    for (int q = 0; q < R; ++q) anyflush |= sc[q].flush;
    if (anyflush) {
        for (int e = threadIdx.x; e < R * wsz; e += kBlock) {
            const int q = e / wsz, j = e % wsz;
            const size_t sy = (size_t)tl.inst * R + q;
            const double* wt = st.w_tab + sy * 3 * kWinTab;
            w_as[e] = wt[j];
            w_bs[e] = wt[kWinTab + j];
            w_zn[e] = wt[2 * kWinTab + j];
            w_act[e] = st.w_act[sy * kWinTab + j];
        }
        __syncthreads();
    }
    double acc[kMaxRhs] = {0.0, 0.0, 0.0, 0.0};
    const int base = st.base;
    for (int it = threadIdx.x; it < R * 3 * SB; it += kBlock) {
        const int rh = it / (3 * SB), c = (it / SB) % 3, jj = it % SB;
        const int site = tl.cb0 + jj;
        if (site >= I.g.vh) continue;
        const BScal& S = sc[rh];
        if (S.stop && !S.flush) continue;
        const size_t i = bvec_off(I, R, rh, c) + site;
        const int slot = S.slot;
        const double2 r0 = to_d2(ring[(size_t)slot * st.ring_stride + i]);
        double2 rv = r0;
        if (!S.stop) {
            const double alpha = S.alpha, beta = S.beta;
            const double2 a = to_d2(Ap[i]);
            const double2 pv = to_d2(p[i]);
            rv.x -= alpha * a.x;
            rv.y -= alpha * a.y;
            const V rl = from_d2<V>(rv);
            ring[(size_t)((slot + 1) % L) * st.ring_stride + i] = rl;
            rv = to_d2(rl);
#pragma unroll
            for (int q = 0; q < kMaxRhs; ++q)
                if (q == rh) acc[q] += rv.x * rv.x + rv.y * rv.y;
            if (S.base_on) {
                double2* xb = x.at<double2>(base);
                const double2 xv = xb[i];
                xb[i] = make_double2(xv.x + alpha * pv.x, xv.y + alpha * pv.y);
            }
            p[i] = from_d2<V>(make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y));
        }
        if (!S.flush) continue;
        const int npend = S.npend;
        const int iter0 = S.slot;  // position of the current iteration in its window
        double2 rw[kLagMax];
#pragma unroll
        for (int t = 0; t < kLagMax; ++t) {
            if (t >= npend) break;
            const int pos_next = t + 1;  // window position of r_{i+1}
            if (pos_next == iter0 + 1)
                rw[t] = rv;
            else if (pos_next == iter0)
                rw[t] = r0;
            else
                rw[t] = to_d2(ring[(size_t)(pos_next % L) * st.ring_stride + i]);
        }
        const double* was = w_as + rh * wsz;
        const double* wbs = w_bs + rh * wsz;
        const double* wzn = w_zn + rh * wsz;
        const int* wact = w_act + rh * wsz;
        constexpr int G = 4;
        for (int g0 = 0; g0 < S.nact; g0 += G) {
            double2 pk[G], xk[G];
#pragma unroll
            for (int jq = 0; jq < G; ++jq)
                if (g0 + jq < S.nact) {
                    const int k = S.list[g0 + jq];
                    pk[jq] = to_d2(ps.at<V>(k)[i]);
                    xk[jq] = x.at<double2>(k)[i];
                }
#pragma unroll
            for (int t = 0; t < kLagMax; ++t) {
                if (t >= npend) break;
#pragma unroll
                for (int jq = 0; jq < G; ++jq)
                    if (g0 + jq < S.nact) {
                        const int k = S.list[g0 + jq];
                        if (wact[t * n + k]) {
                            const double aq = was[t * n + k], bq = wbs[t * n + k], zq = wzn[t * n + k];
                            xk[jq] = make_double2(xk[jq].x + aq * pk[jq].x, xk[jq].y + aq * pk[jq].y);
                            pk[jq] = to_d2(from_d2<V>(make_double2(zq * rw[t].x + bq * pk[jq].x,
                                                                   zq * rw[t].y + bq * pk[jq].y)));
                        }
                    }
            }
#pragma unroll
            for (int jq = 0; jq < G; ++jq)
                if (g0 + jq < S.nact) {
                    const int k = S.list[g0 + jq];
                    x.at<double2>(k)[i] = xk[jq];
                    ps.at<V>(k)[i] = from_d2<V>(pk[jq]);
                }
        }
    }
    block_sum<kMaxRhs>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kMaxRhs; ++q) qout[(size_t)blockIdx.x * kMaxRhs + q] = acc[q];
}

// one block per system: its (tile, rhs) partials over the instance's tiles
__global__ __launch_bounds__(kBlock) void k_bsys_sum(BatchDev bd, const double* __restrict__ part,
                                                     double* __restrict__ out) {
    const int s = blockIdx.x;
    const int R = bd.nrhs;
    const BInst I = bd.inst[s / R];
    const int q = s % R;
    double t[1] = {0.0};
    for (int k = threadIdx.x; k < I.ntiles; k += kBlock) t[0] += part[(size_t)(I.tile0 + k) * kMaxRhs + q];
    __shared__ double lds[4];
    block_sum<1>(t, lds);
    if (threadIdx.x == 0) out[s] = t[0];
}

// canonical packed [inst][rhs][site][colour] <-> internal [inst][rhs][colour][site]
__global__ void k_bvec_import(BatchDev bd, const double2* __restrict__ canon, double2* __restrict__ vec) {
    const BTile tl = bd.tiles[blockIdx.x];
    const BInst I = bd.inst[tl.inst];
    const int R = bd.nrhs, SB = bd.tile_sites;
    for (int it = threadIdx.x; it < R * SB; it += blockDim.x) {
        const int rh = it / SB, site = tl.cb0 + it % SB;
        if (site >= I.g.vh) continue;
        const size_t cbase = (size_t)3 * ((size_t)R * I.off + (size_t)rh * I.g.vh + site);
#pragma unroll
        for (int c = 0; c < 3; ++c) vec[bvec_off(I, R, rh, c) + site] = canon[cbase + c];
    }
}

__global__ void k_bvec_export(BatchDev bd, const double2* __restrict__ vec, double2* __restrict__ canon) {
    const BTile tl = bd.tiles[blockIdx.x];
    const BInst I = bd.inst[tl.inst];
    const int R = bd.nrhs, SB = bd.tile_sites;
    for (int it = threadIdx.x; it < R * SB; it += blockDim.x) {
        const int rh = it / SB, site = tl.cb0 + it % SB;
        if (site >= I.g.vh) continue;
        const size_t cbase = (size_t)3 * ((size_t)R * I.off + (size_t)rh * I.g.vh + site);
#pragma unroll
        for (int c = 0; c < 3; ++c) canon[cbase + c] = vec[bvec_off(I, R, rh, c) + site];
    }
}

__global__ void k_blinks_to_f32(const double2* __restrict__ d, float2* __restrict__ f, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 v = d[i];
        f[i] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_bstate_init(BState st, int from_fin) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int nsys = st.n_inst * st.nrhs;
    if (s >= nsys) return;
    MsIter& S = st.it[0][s];
    for (int k = 0; k < st.n; ++k) {
        S.zeta[k] = S.zeta_old[k] = 1.0;
        S.active[k] = 1;
        S.iters_per_pole[k] = 0;
    }
    S.alpha_old = 1.0;
    S.beta_old = 0.0;
    S.bb = from_fin ? st.fin[s].bb : 0.0;
    S.rr = 0.0;
    S.iter = 0;
    S.nonfinite = 0;
    st.sys_done[s] = 0;
    st.sys_done[nsys + s] = 0;
    st.t_done[s] = 0;
    if (s % st.nrhs == 0) {
        st.inst_done[s / st.nrhs] = 0;
        st.inst_done[st.n_inst + s / st.nrhs] = 0;
    }
}

__global__ void k_baxpy(size_t n, double2* __restrict__ x, const double2* __restrict__ e) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 a = x[i], b = e[i];
        x[i] = make_double2(a.x + b.x, a.y + b.y);
    }
}

__global__ void k_timestamp(unsigned long long* t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] = wall_clock64();
}

}  // namespace

template <class V>
void launch_bdslash(const BatchDev& bd, int tps, const void* links, const V* in, V* out, int out_par,
                    const int* inst_done, hipStream_t s) {
    bdslash_tps<V>(bd, tps, (const V*)links, in, out_par, BEpiStore<V>{out}, inst_done, s);
}
template void launch_bdslash<double2>(const BatchDev&, int, const void*, const double2*, double2*, int, const int*,
                                      hipStream_t);
template void launch_bdslash<float2>(const BatchDev&, int, const void*, const float2*, float2*, int, const int*,
                                     hipStream_t);

template <class V>
void launch_bdslash_cg(const BatchDev& bd, int tps, const void* links, const V* w_o, const V* p, const V* r, V* Ap,
                       BState st, const int* inst_done, double* dpart, hipStream_t s) {
    bdslash_tps<V>(bd, tps, (const V*)links, w_o, 0, BEpiCG<V>{Ap, p, r, st.sigma0_term, dpart}, inst_done, s);
}
template void launch_bdslash_cg<double2>(const BatchDev&, int, const void*, const double2*, const double2*,
                                         const double2*, double2*, BState, const int*, double*, hipStream_t);
template void launch_bdslash_cg<float2>(const BatchDev&, int, const void*, const float2*, const float2*, const float2*,
                                        float2*, BState, const int*, double*, hipStream_t);

void launch_bdslash_resid(const BatchDev& bd, int tps, const double2* links, const double2* w_o, const double2* x,
                          const double2* b, double pole, double* part, double2* rout, hipStream_t s) {
    bdslash_tps<double2>(bd, tps, links, w_o, 0, BEpiResid{x, b, rout, pole, part}, nullptr, s);
}

template <class V>
void launch_bms_init(const BatchDev& bd, const double2* b, V* r, V* p, VecPtrs x, VecPtrs ps, BState st,
                     double* qout, hipStream_t s) {
    k_bms_init<V><<<bd.ntiles, kBlock, 0, s>>>(bd, b, r, p, x, ps, st, qout);
}
template void launch_bms_init<double2>(const BatchDev&, const double2*, double2*, double2*, VecPtrs, VecPtrs,
                                       BState, double*, hipStream_t);
template void launch_bms_init<float2>(const BatchDev&, const double2*, float2*, float2*, VecPtrs, VecPtrs,
                                      BState, double*, hipStream_t);

template <class V>
void launch_bms_step(const BatchDev& bd, V* r, const V* Ap, V* p, VecPtrs x, VecPtrs ps, BState st,
                     const double* dpart, const double* qin, double* qout, int par, hipStream_t s) {
    (void)dpart;
    (void)qin;
    const size_t lds = (size_t)kMaxRhs * st.lag * st.n * (3 * sizeof(double) + sizeof(int));
    k_bms_step<V><<<bd.ntiles, kBlock, lds, s>>>(bd, r, Ap, p, x, ps, st, qout, par);
}
template void launch_bms_step<double2>(const BatchDev&, double2*, const double2*, double2*, VecPtrs, VecPtrs, BState,
                                       const double*, const double*, double*, int, hipStream_t);
template void launch_bms_step<float2>(const BatchDev&, float2*, const float2*, float2*, VecPtrs, VecPtrs, BState,
                                      const double*, const double*, double*, int, hipStream_t);

void launch_bms_scalars(const BatchDev& bd, BState st, const double* dpart, const double* qin, int par,
                        hipStream_t s) {
    k_bms_scalars<<<st.n_inst, kBlock, 0, s>>>(bd, st, dpart, qin, par);
}

void launch_bsys_sum(const BatchDev& bd, int n_inst, const double* part, double* out, hipStream_t s) {
    const int n = n_inst * bd.nrhs;
    k_bsys_sum<<<n, kBlock, 0, s>>>(bd, part, out);
}

void launch_bvec_import(const BatchDev& bd, const double2* canon, double2* vec, hipStream_t s) {
    k_bvec_import<<<bd.ntiles, kBlock, 0, s>>>(bd, canon, vec);
}
void launch_bvec_export(const BatchDev& bd, const double2* vec, double2* canon, hipStream_t s) {
    k_bvec_export<<<bd.ntiles, kBlock, 0, s>>>(bd, vec, canon);
}
void launch_blinks_to_f32(const double2* d, float2* f, size_t n, hipStream_t s) {
    int nb = (int)((n + 255) / 256);
    if (nb > 8192) nb = 8192;
    k_blinks_to_f32<<<nb, 256, 0, s>>>(d, f, n);
}
void launch_b_timestamp(unsigned long long* t, hipStream_t s) { k_timestamp<<<1, 64, 0, s>>>(t); }

void launch_bstate_init(BState st, int from_fin, hipStream_t s) {
    const int n = st.n_inst * st.nrhs;
    k_bstate_init<<<(n + 255) / 256, 256, 0, s>>>(st, from_fin);
}

void launch_baxpy(size_t n, double2* x, const double2* e, hipStream_t s) {
    int nb = (int)((n + 255) / 256);
    if (nb > 8192) nb = 8192;
    k_baxpy<<<nb, 256, 0, s>>>(n, x, e);
}

}  // namespace stag
