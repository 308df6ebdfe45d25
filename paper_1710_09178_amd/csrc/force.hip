// Molecular-dynamics kernels of the HMC trajectory (Sec. 3.1):
// pseudofermion force, Wilson gauge force, link update exp(i dt p) U with
// reunitarisation, and the plaquette / kinetic-energy reductions.
#include "common.h"

namespace stag {

namespace {

__device__ __forceinline__ M3 load_link(const double2* __restrict__ links, const Geom& g, int par, int cb, int mu) {
    M3 m;
    const double2* u = links + link_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = u[(size_t)e * g.vh];
    return m;
}

__device__ __forceinline__ M3 load_link_at(const double2* __restrict__ links, const Geom& g, int x, int y, int z,
                                           int t, int mu) {
    const int par = (x + y + z + t) & 1;
    return load_link(links, g, par, cb_index(g, x, y, z, t), mu);
}

__device__ __forceinline__ void store_force(double* __restrict__ mom, const Geom& g, int par, int mu, int cb,
                                            const double f[8], double dt) {
    double* m = mom + mom_off(g, par, mu, 0) + cb;
    if (dt == 0.0) {
#pragma unroll
        for (int a = 0; a < 8; ++a) m[(size_t)a * g.vh] = f[a];
    } else {
#pragma unroll
        for (int a = 0; a < 8; ++a) m[(size_t)a * g.vh] += dt * f[a];
    }
}

// F_a(x,mu) = 2 Im tr(T_a s U_mu(x) W),  W = eps(x) sum_k c_k chi_k(x+mu) chi_k(x)^dag,
// chi_k = X_k on even sites and Y_k = D_oe X_k on odd sites, eps = +1 (even) / -1 (odd).
// (w1: the weight of the one-hop term, c1 for the improved operator, else 1)
// One thread per link (mu, parity, site): consecutive threads take consecutive
// sites of one (mu, parity) plane, so every stream is contiguous.
__global__ __launch_bounds__(kBlock) void k_fermion_force(Geom g, const double2* __restrict__ links,
                                                          VecPtrs X, VecPtrs Y, const double* __restrict__ coef,
                                                          int n, double* __restrict__ mom, double dt, double w1) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 8 * g.vh) return;
    const int mu = i / (2 * g.vh), rem = i % (2 * g.vh);
    const int par = rem / g.vh, cb = rem % g.vh;
    int x, y, z, t;
    cb_coords(g, par, cb, x, y, z, t);
    const double eps = par == 0 ? 1.0 : -1.0;
    int xn = x, yn = y, zn = z, tn = t;
    double s;
    if (mu == 0) {
        xn = (x + 1 == g.nx) ? 0 : x + 1;
        s = 1.0;
    } else if (mu == 1) {
        yn = (y + 1 == g.ny) ? 0 : y + 1;
        s = (x & 1) ? -1.0 : 1.0;
    } else if (mu == 2) {
        zn = (z + 1 == g.nz) ? 0 : z + 1;
        s = ((x + y) & 1) ? -1.0 : 1.0;
    } else {
        tn = (t + 1 == g.nt) ? 0 : t + 1;
        s = ((x + y + z) & 1) ? -1.0 : 1.0;
        if (t == g.nt - 1) s = -s;
    }
    const int cbn = cb_index(g, xn, yn, zn, tn);
    M3 W;
#pragma unroll
    for (int e = 0; e < 9; ++e) W.e[e] = make_double2(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
        const double2* here = (par == 0 ? X.at<double2>(k) : Y.at<double2>(k));
        const double2* there = (par == 0 ? Y.at<double2>(k) : X.at<double2>(k));
        double2 a[3], b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[c] = there[(size_t)c * g.vh + cbn];
            b[c] = here[(size_t)c * g.vh + cb];
        }
        const double ck = coef[k];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double2 v = cmul(a[r], cconj(b[j]));
                W.e[3 * r + j].x += ck * v.x;
                W.e[3 * r + j].y += ck * v.y;
            }
    }
    M3 U = load_link(links, g, par, cb, mu);
    M3 M = m3_mul(U, W);
    double f[8];
    im_tr_ta(M, f);
    const double fac = 2.0 * s * eps * w1;
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a] *= fac;
    store_force(mom, g, par, mu, cb, f, dt);
}

// ---- three-hop part of the force of the improved operator (the "improved"
// quarks of the Summary, Sec. 8, read as the Naik stencil): S_f of Sec. 3.1
// differentiated through every three-link path a link lies on, at path
// positions 0, 1 and 2 (paths starting at z, z-mu and z-2mu).
__device__ __forceinline__ int step_mod(int v, int d, int n) {
    v += d;
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// W3(x, mu) = s3(x) eps(x) sum_k c_k chi_k(x+3mu) chi_k(x)^dag, one thread per
// (mu, parity, site); s3 is the path's sign (eta_mu(x) once, -1 per link that
// leaves the last time slice).
__global__ __launch_bounds__(kBlock) void k_naik_w3(Geom g, VecPtrs X, VecPtrs Y, const double* __restrict__ coef,
                                                    int n, double2* __restrict__ w3) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 8 * g.vh) return;
    const int mu = i / (2 * g.vh), rem = i % (2 * g.vh);
    const int par = rem / g.vh, cb = rem % g.vh;
    int c[4];
    cb_coords(g, par, cb, c[0], c[1], c[2], c[3]);
    const int nn[4] = {g.nx, g.ny, g.nz, g.nt};
    const double eps = par == 0 ? 1.0 : -1.0;
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = step_mod(c[mu], 3, nn[mu]);
    const int cb3 = cb_index(g, d[0], d[1], d[2], d[3]);
    double s = 1.0;
    if (mu == 1) s = (c[0] & 1) ? -1.0 : 1.0;
    if (mu == 2) s = ((c[0] + c[1]) & 1) ? -1.0 : 1.0;
    if (mu == 3) {
        s = ((c[0] + c[1] + c[2]) & 1) ? -1.0 : 1.0;
        if (((c[3] + 3) / g.nt) & 1) s = -s;
    }
    M3 W;
#pragma unroll
    for (int e = 0; e < 9; ++e) W.e[e] = make_double2(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
        const double2* here = (par == 0 ? X.at<double2>(k) : Y.at<double2>(k));
        const double2* there = (par == 0 ? Y.at<double2>(k) : X.at<double2>(k));
        double2 a[3], b[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            a[cc] = there[(size_t)cc * g.vh + cb3];
            b[cc] = here[(size_t)cc * g.vh + cb];
        }
        const double ck = coef[k];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double2 v = cmul(a[r], cconj(b[j]));
                W.e[3 * r + j].x += ck * v.x;
                W.e[3 * r + j].y += ck * v.y;
            }
    }
    const double fac = s * eps;
    double2* out = w3 + link_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int e = 0; e < 9; ++e) out[(size_t)e * g.vh] = make_double2(fac * W.e[e].x, fac * W.e[e].y);
}

// F_a(z, mu) += 2 c3 Im tr(T_a U(z) [U(z+mu) U(z+2mu) W3(z) + U(z+mu) W3(z-mu) U(z-mu)
//                                    + W3(z-2mu) U(z-2mu) U(z-mu)])
// (plain links: every path's sign is in its W3).  One thread per link; added
// to mom with factor dt, or 1 when dt == 0 (the one-hop kernel wrote F first).
__global__ __launch_bounds__(kBlock) void k_naik_force3(Geom g, const double2* __restrict__ links,
                                                        const double2* __restrict__ w3, double c3,
                                                        double* __restrict__ mom, double dt) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    int c[4];
    cb_coords(g, par, cb, c[0], c[1], c[2], c[3]);
    const int nn[4] = {g.nx, g.ny, g.nz, g.nt};
    auto at = [&](int d) {  // cb index and parity of z + d mu
        int e[4] = {c[0], c[1], c[2], c[3]};
        e[mu] = step_mod(c[mu], d, nn[mu]);
        return cb_index(g, e[0], e[1], e[2], e[3]);
    };
    const int p1 = par ^ 1;
    const int cp1 = at(1), cp2 = at(2), cm1 = at(-1), cm2 = at(-2);
    // M = U(z+mu) [U(z+2mu) W3(z) + W3(z-mu) U(z-mu)] + W3(z-2mu) U(z-2mu) U(z-mu),
    // built in an order that keeps few matrices live
    M3 P = m3_mul(load_link(links, g, par, cp2, mu), load_link(w3, g, par, cb, mu));
    const M3 Um1 = load_link(links, g, p1, cm1, mu);
    P = m3_add(P, m3_mul(load_link(w3, g, p1, cm1, mu), Um1));
    M3 M = m3_mul(load_link(links, g, p1, cp1, mu), P);
    P = m3_mul(load_link(w3, g, par, cm2, mu), load_link(links, g, par, cm2, mu));
    M = m3_add(M, m3_mul(P, Um1));
    double f[8];
    im_tr_ta(m3_mul(load_link(links, g, par, cb, mu), M), f);
    const double fac = 2.0 * c3 * (dt == 0.0 ? 1.0 : dt);
    double* m = mom + mom_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int a = 0; a < 8; ++a) m[(size_t)a * g.vh] += fac * f[a];
}

// F_a = -(beta/3) Im tr(T_a U_mu(x) A_mu(x)), A = sum of the six staples.
__global__ __launch_bounds__(kBlock) void k_gauge_force(Geom g, const double2* __restrict__ links, double beta,
                                                        double* __restrict__ mom, double dt) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    int x, y, z, t;
    cb_coords(g, par, cb, x, y, z, t);
    const int n[4] = {g.nx, g.ny, g.nz, g.nt};
    int c[4] = {x, y, z, t};
    M3 A;
#pragma unroll
    for (int e = 0; e < 9; ++e) A.e[e] = make_double2(0.0, 0.0);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int cp[4] = {c[0], c[1], c[2], c[3]};  // x + mu
        cp[mu] = (c[mu] + 1 == n[mu]) ? 0 : c[mu] + 1;
        int cn[4] = {c[0], c[1], c[2], c[3]};  // x + nu
        cn[nu] = (c[nu] + 1 == n[nu]) ? 0 : c[nu] + 1;
        int cm[4] = {c[0], c[1], c[2], c[3]};  // x - nu
        cm[nu] = (c[nu] == 0) ? n[nu] - 1 : c[nu] - 1;
        int cpm[4] = {cp[0], cp[1], cp[2], cp[3]};  // x + mu - nu
        cpm[nu] = cm[nu];
        // upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        const M3 a1 = load_link_at(links, g, cp[0], cp[1], cp[2], cp[3], nu);
        const M3 a2 = load_link_at(links, g, cn[0], cn[1], cn[2], cn[3], mu);
        const M3 a3 = load_link_at(links, g, c[0], c[1], c[2], c[3], nu);
        A = m3_add(A, m3_mul(m3_mul(a1, m3_dag(a2)), m3_dag(a3)));
        // lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        const M3 b1 = load_link_at(links, g, cpm[0], cpm[1], cpm[2], cpm[3], nu);
        const M3 b2 = load_link_at(links, g, cm[0], cm[1], cm[2], cm[3], mu);
        const M3 b3 = load_link_at(links, g, cm[0], cm[1], cm[2], cm[3], nu);
        A = m3_add(A, m3_mul(m3_mul(m3_dag(b1), m3_dag(b2)), b3));
    }
    const M3 U = load_link(links, g, par, cb, mu);
    double f[8];
    im_tr_ta(m3_mul(U, A), f);
    const double fac = -beta / 3.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a] *= fac;
    store_force(mom, g, par, mu, cb, f, dt);
}

// exp(i X) for Hermitian X: scaling and squaring with a degree-12 Taylor
// polynomial (Moler & Van Loan, SIAM Review 45 (2003) 3): after scaling
// |X|/2^s <= 1/4 the truncation error is below 3e-18.
__device__ M3 expi_herm(const M3& X) {
    double nrm2 = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) nrm2 += X.e[e].x * X.e[e].x + X.e[e].y * X.e[e].y;
    const double nrm = sqrt(nrm2);
    int s = 0;
    double scale = 1.0;
    while (nrm * scale > 0.25 && s < 60) {
        scale *= 0.5;
        ++s;
    }
    M3 Z;  // Z = i X scale
#pragma unroll
    for (int e = 0; e < 9; ++e) Z.e[e] = make_double2(-X.e[e].y * scale, X.e[e].x * scale);
    // Horner: E = I + Z (I + Z/2 (I + Z/3 (... (I + Z/12))))
    M3 E;
#pragma unroll
    for (int e = 0; e < 9; ++e) E.e[e] = make_double2(0.0, 0.0);
    for (int k = 12; k >= 1; --k) {
        M3 T = m3_mul(Z, E);
        const double inv = 1.0 / (double)k;
#pragma unroll
        for (int e = 0; e < 9; ++e) E.e[e] = cscale(inv, T.e[e]);
        E.e[0].x += 1.0;
        E.e[4].x += 1.0;
        E.e[8].x += 1.0;
    }
    for (int k = 0; k < s; ++k) E = m3_mul(E, E);
    return E;
}

// Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1).
__device__ M3 reunitarise(const M3& u) {
    M3 r;
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += u.e[j].x * u.e[j].x + u.e[j].y * u.e[j].y;
    const double i0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[j] = cscale(i0, u.e[j]);
    double2 d = make_double2(0.0, 0.0);  // <r0, u1>
#pragma unroll
    for (int j = 0; j < 3; ++j) d = cadd(d, cmulc(r.e[j], u.e[3 + j]));
    double n1 = 0.0;
    double2 v[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        v[j] = csub(u.e[3 + j], cmul(d, r.e[j]));
        n1 += v[j].x * v[j].x + v[j].y * v[j].y;
    }
    const double i1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 + j] = cscale(i1, v[j]);
    r.e[6] = cconj(csub(cmul(r.e[1], r.e[5]), cmul(r.e[2], r.e[4])));
    r.e[7] = cconj(csub(cmul(r.e[2], r.e[3]), cmul(r.e[0], r.e[5])));
    r.e[8] = cconj(csub(cmul(r.e[0], r.e[4]), cmul(r.e[1], r.e[3])));
    return r;
}

// sum_a p_a T_a as a 3x3 Hermitian matrix, T_a = lambda_a / 2
__device__ __forceinline__ M3 algebra_matrix(const double p[8], double scale) {
    const double h = 0.5 * scale;
    const double r3 = 0.57735026918962576451;
    M3 X;
    X.e[0] = make_double2(h * (p[2] + r3 * p[7]), 0.0);
    X.e[4] = make_double2(h * (-p[2] + r3 * p[7]), 0.0);
    X.e[8] = make_double2(h * (-2.0 * r3 * p[7]), 0.0);
    X.e[1] = make_double2(h * p[0], -h * p[1]);
    X.e[3] = make_double2(h * p[0], h * p[1]);
    X.e[2] = make_double2(h * p[3], -h * p[4]);
    X.e[6] = make_double2(h * p[3], h * p[4]);
    X.e[5] = make_double2(h * p[5], -h * p[6]);
    X.e[7] = make_double2(h * p[5], h * p[6]);
    return X;
}

__global__ __launch_bounds__(kBlock) void k_link_update(Geom g, double2* __restrict__ links,
                                                        const double* __restrict__ mom, double dt) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    double p[8];
    const double* m = mom + mom_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int a = 0; a < 8; ++a) p[a] = m[(size_t)a * g.vh];
    const M3 E = expi_herm(algebra_matrix(p, dt));
    const M3 U = load_link(links, g, par, cb, mu);
    const M3 R = reunitarise(m3_mul(E, U));
    double2* u = links + link_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int e = 0; e < 9; ++e) u[(size_t)e * g.vh] = R.e[e];
}

// sum over sites and mu<nu of Re tr P_{mu nu}(x)
__global__ __launch_bounds__(kBlock) void k_plaquette(Geom g, const double2* __restrict__ links,
                                                      double* __restrict__ part) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double acc[1] = {0.0};
    if (i < V) {
        const int par = i / g.vh, cb = i % g.vh;
        int c[4];
        cb_coords(g, par, cb, c[0], c[1], c[2], c[3]);
        const int n[4] = {g.nx, g.ny, g.nz, g.nt};
        for (int mu = 0; mu < 4; ++mu) {
            int cp[4] = {c[0], c[1], c[2], c[3]};
            cp[mu] = (c[mu] + 1 == n[mu]) ? 0 : c[mu] + 1;
            const M3 umu = load_link(links, g, par, cb, mu);
            for (int nu = mu + 1; nu < 4; ++nu) {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cn[nu] = (c[nu] + 1 == n[nu]) ? 0 : c[nu] + 1;
                const M3 a = load_link_at(links, g, cp[0], cp[1], cp[2], cp[3], nu);
                const M3 b = load_link_at(links, g, cn[0], cn[1], cn[2], cn[3], mu);
                const M3 d = load_link(links, g, par, cb, nu);
                const M3 P = m3_mul(m3_mul(umu, a), m3_dag(m3_mul(d, b)));
                acc[0] += P.e[0].x + P.e[4].x + P.e[8].x;
            }
        }
    }
    block_partial<1>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_sumsq(size_t n, const double* __restrict__ v, double* __restrict__ part) {
    double acc[1] = {0.0};
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const double a = v[i];
        acc[0] += a * a;
    }
    block_partial<1>(acc, part);
}

}  // namespace

// block partials of |a - b|^2 and |b|^2 over n reals, then their totals into out2[0..1]
__global__ __launch_bounds__(kBlock) void k_diff_norm2(size_t n, const double* __restrict__ a,
                                                       const double* __restrict__ b, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const double bi = b[i], d = a[i] - bi;
        v[0] += d * d;
        v[1] += bi * bi;
    }
    block_partial<2>(v, part);
}

void launch_fermion_force(const Geom& g, const double2* links, VecPtrs X, VecPtrs Y, const double* coef, int n,
                          double* mom, double dt, hipStream_t s, double w1) {
    const int grid = (8 * g.vh + kBlock - 1) / kBlock;
    k_fermion_force<<<grid, kBlock, 0, s>>>(g, links, X, Y, coef, n, mom, dt, w1);
}

// part: >= 2 * 1024 doubles
void launch_diff_norm2(size_t n, const double* a, const double* b, double* part, double* out2, hipStream_t s) {
    constexpr int nb = 1024;
    k_diff_norm2<<<nb, kBlock, 0, s>>>(n, a, b, part);
    launch_finalize(part, nb, 2, out2, s);
}

void launch_naik_force3(const Geom& g, const double2* links, VecPtrs X, VecPtrs Y, const double* coef, int n,
                        double2* w3, double c3, double* mom, double dt, hipStream_t s) {
    const int grid = (8 * g.vh + kBlock - 1) / kBlock;
    k_naik_w3<<<grid, kBlock, 0, s>>>(g, X, Y, coef, n, w3);
    k_naik_force3<<<grid, kBlock, 0, s>>>(g, links, w3, c3, mom, dt);
}

void launch_gauge_force(const Geom& g, const double2* links, double beta, double* mom, double dt, hipStream_t s) {
    const int grid = (8 * g.vh + kBlock - 1) / kBlock;
    k_gauge_force<<<grid, kBlock, 0, s>>>(g, links, beta, mom, dt);
}

void launch_link_update(const Geom& g, double2* links, const double* mom, double dt, hipStream_t s) {
    const int grid = (8 * g.vh + kBlock - 1) / kBlock;
    k_link_update<<<grid, kBlock, 0, s>>>(g, links, mom, dt);
}

int launch_plaquette(const Geom& g, const double2* links, double* part, hipStream_t s) {
    const int grid = (2 * g.vh + kBlock - 1) / kBlock;
    k_plaquette<<<grid, kBlock, 0, s>>>(g, links, part);
    return grid;
}

int launch_kinetic(const Geom& g, const double* mom, double* part, hipStream_t s) {
    const size_t n = (size_t)64 * g.vh;
    int grid = (int)((n + kBlock - 1) / kBlock);
    if (grid > 4096) grid = 4096;
    k_sumsq<<<grid, kBlock, 0, s>>>(n, mom, part);
    return grid;
}

}  // namespace stag
