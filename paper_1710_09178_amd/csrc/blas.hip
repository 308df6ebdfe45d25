// Vector kernels of the multi-shift CG (Sec. 4): initialisation, the fused
// per-iteration step (scalar recurrences + update of r, p and every active
// shift), the rational sum c0 b + sum_k c_k x_k, a real dot product and the
// one-block finaliser for partial sums.  One thread per complex element of a
// half vector ([3][Vh] double2); all accesses are contiguous.
//
// Reductions never synchronise blocks inside a kernel: each block writes its
// partial sum, and whoever needs the total adds the partials in block order
// after the kernel boundary.  The step kernel does this redundantly in every
// block (a few thousand doubles, L2 resident), so each block derives the same
// bitwise scalars without a grid-wide barrier.
#include "common.h"

namespace stag {

namespace {

__global__ __launch_bounds__(kBlock) void k_ms_init(int n3, const double2* __restrict__ b, double2* __restrict__ r,
                                                    double2* __restrict__ p, VecPtrs x, VecPtrs ps,
                                                    const MsState* __restrict__ st, double* __restrict__ qout) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int n = st->n, base = st->base;
    double acc[1] = {0.0};
    if (i < n3) {
        const double2 bv = b[i];
        r[i] = bv;
        p[i] = bv;
        for (int k = 0; k < n; ++k) {
            x.p[k][i] = make_double2(0.0, 0.0);
            if (k != base) ps.p[k][i] = bv;
        }
        acc[0] = bv.x * bv.x + bv.y * bv.y;
    }
    block_partial<1>(acc, qout);
}

// Iteration k (parity par):
//   rr_k   = sum of the <r,r> partials of the previous step (or of init)
//   freeze every shift with zeta_k^2 rr_k <= tol^2 <b,b>; stop if none is left
//   alpha  = rr_k / <p,Ap>,   rr_{k+1} = rr_k - 2 alpha <r,Ap> + alpha^2 <Ap,Ap>
//   beta   = rr_{k+1} / rr_k, zeta', alpha_s, beta_s from the shifted-CG recurrences
//   r -= alpha Ap; x_base += alpha p; p = r + beta p;
//   x_s += alpha_s p_s; p_s = zeta_s' r + beta_s p_s      (active shifts)
__global__ __launch_bounds__(kBlock) void k_ms_step(int n3, double2* __restrict__ r, const double2* __restrict__ Ap,
                                                    double2* __restrict__ p, VecPtrs x, VecPtrs ps,
                                                    MsState* __restrict__ st, const double* __restrict__ dpart,
                                                    int nb2, const double* __restrict__ qin, double* __restrict__ qout,
                                                    int par) {
    if (st->done) return;
    __shared__ double lds[16];
    __shared__ double sh_as[kMaxPoles], sh_bs[kMaxPoles], sh_zn[kMaxPoles];
    __shared__ int sh_act[kMaxPoles];
    __shared__ double sh_alpha, sh_beta;
    __shared__ int sh_stop;
    const int n = st->n, base = st->base;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int nbq = gridDim.x;  // init and step kernels use the same grid
    for (int b = threadIdx.x; b < nbq; b += kBlock) v[0] += qin[b];
    for (int b = threadIdx.x; b < nb2; b += kBlock) {
        v[1] += dpart[b];
        v[2] += dpart[nb2 + b];
        v[3] += dpart[2 * nb2 + b];
    }
    block_sum<4>(v, lds);
    if (threadIdx.x == 0) {
        const MsIter& s = st->it[par];
        const double rr = v[0], pAp = v[1], rAp = v[2], ApAp = v[3];
        const int iter = s.iter;
        const double bb = (iter == 0) ? rr : s.bb;
        int nonfinite = !isfinite(rr);
        int any = 0;
        int act[kMaxPoles];
        for (int k = 0; k < n; ++k) {
            act[k] = s.active[k];
            if (act[k] && s.zeta[k] * s.zeta[k] * rr <= st->tol2 * bb) act[k] = 0;
            any |= act[k];
        }
        int stop = nonfinite || !any || iter >= st->maxiter;
        double alpha = 0.0, beta = 0.0;
        double zn[kMaxPoles];
        if (!stop) {
            alpha = rr / pAp;
            double rr1 = rr - 2.0 * alpha * rAp + alpha * alpha * ApAp;
            if (rr1 < 0.0) rr1 = 0.0;
            beta = rr1 / rr;
            const double a_old = s.alpha_old, b_old = s.beta_old;
            for (int k = 0; k < n; ++k) {
                if (k == base) {
                    zn[k] = 1.0;
                    sh_as[k] = alpha;
                    sh_bs[k] = beta;
                    continue;
                }
                const double z = s.zeta[k], zo = s.zeta_old[k];
                if (!act[k]) {
                    zn[k] = z;
                    sh_as[k] = sh_bs[k] = 0.0;
                    continue;
                }
                const double znk = z * zo * a_old / (alpha * b_old * (zo - z) + zo * a_old * (1.0 + st->shift[k] * alpha));
                const double q = znk / z;
                zn[k] = znk;
                sh_as[k] = alpha * q;
                sh_bs[k] = beta * q * q;
            }
            if (!isfinite(alpha) || !isfinite(beta)) {
                nonfinite = 1;
                stop = 1;
            }
        }
        for (int k = 0; k < n; ++k) {
            sh_act[k] = act[k];
            sh_zn[k] = zn[k];
        }
        sh_alpha = alpha;
        sh_beta = beta;
        sh_stop = stop;
        if (blockIdx.x == 0) {
            MsIter& o = stop ? st->fin : st->it[par ^ 1];
            for (int k = 0; k < n; ++k) {
                o.active[k] = act[k];
                o.iters_per_pole[k] = (act[k] && !stop) ? iter + 1 : (s.active[k] ? iter : s.iters_per_pole[k]);
                o.zeta[k] = stop ? s.zeta[k] : zn[k];
                o.zeta_old[k] = stop ? s.zeta_old[k] : s.zeta[k];
            }
            o.alpha_old = stop ? s.alpha_old : alpha;
            o.beta_old = stop ? s.beta_old : beta;
            o.bb = bb;
            o.rr = rr;
            o.iter = stop ? iter : iter + 1;
            o.nonfinite = nonfinite;
            if (stop) st->done = 1;
        }
    }
    __syncthreads();
    if (sh_stop) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double alpha = sh_alpha, beta = sh_beta;
    double acc[1] = {0.0};
    if (i < n3) {
        const double2 a = Ap[i];
        double2 rv = r[i];
        rv.x -= alpha * a.x;
        rv.y -= alpha * a.y;
        r[i] = rv;
        acc[0] = rv.x * rv.x + rv.y * rv.y;
        const double2 pv = p[i];
        if (sh_act[base]) {
            double2 xv = x.p[base][i];
            xv.x += alpha * pv.x;
            xv.y += alpha * pv.y;
            x.p[base][i] = xv;
        }
        p[i] = make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y);
        for (int k = 0; k < n; ++k) {
            if (k == base || !sh_act[k]) continue;
            const double ak = sh_as[k], bk = sh_bs[k], zk = sh_zn[k];
            const double2 pk = ps.p[k][i];
            double2 xv = x.p[k][i];
            xv.x += ak * pk.x;
            xv.y += ak * pk.y;
            x.p[k][i] = xv;
            ps.p[k][i] = make_double2(zk * rv.x + bk * pk.x, zk * rv.y + bk * pk.y);
        }
    }
    block_partial<1>(acc, qout);
}

__global__ __launch_bounds__(kBlock) void k_rational_sum(int n3, const double2* __restrict__ b, VecPtrs x,
                                                         const MsState* __restrict__ st,
                                                         double2* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n3) return;
    const double2 bv = b[i];
    const double c0 = st->c0;
    double2 s = make_double2(c0 * bv.x, c0 * bv.y);
    for (int k = 0; k < st->n; ++k) {
        const double2 v = x.p[k][i];
        const double ck = st->coef[k];
        s.x += ck * v.x;
        s.y += ck * v.y;
    }
    out[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_dot_re(int n3, const double2* __restrict__ a, const double2* __restrict__ b,
                                                   double* __restrict__ part) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double acc[1] = {0.0};
    if (i < n3) {
        const double2 u = a[i], v = b[i];
        acc[0] = u.x * v.x + u.y * v.y;
    }
    block_partial<1>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ part, int nb, int K,
                                                     double* __restrict__ out) {
    __shared__ double lds[4];
    for (int k = 0; k < K; ++k) {
        const double t = sum_partials(part + (size_t)k * nb, nb, lds);
        if (threadIdx.x == 0) out[k] = t;
        __syncthreads();
    }
}

inline int grid3(const Geom& g) { return (3 * g.vh + kBlock - 1) / kBlock; }

}  // namespace

int ms_update_grid(const Geom& g) { return grid3(g); }
int dot_grid(const Geom& g) { return grid3(g); }

void launch_ms_init(const Geom& g, const double2* b, double2* r, double2* p, VecPtrs x, VecPtrs ps,
                    const MsState* st, double* qout, hipStream_t s) {
    k_ms_init<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, b, r, p, x, ps, st, qout);
}

void launch_ms_step(const Geom& g, double2* r, const double2* Ap, double2* p, VecPtrs x, VecPtrs ps, MsState* st,
                    const double* dpart, int nb2, const double* qin, double* qout, int par, hipStream_t s) {
    k_ms_step<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, r, Ap, p, x, ps, st, dpart, nb2, qin, qout, par);
}

void launch_rational_sum(const Geom& g, const double2* b, VecPtrs x, const MsState* st, double2* out,
                         hipStream_t s) {
    k_rational_sum<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, b, x, st, out);
}

void launch_dot_re(const Geom& g, const double2* a, const double2* b, double* part, hipStream_t s) {
    k_dot_re<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, a, b, part);
}

void launch_finalize(const double* part, int nb, int K, double* out, hipStream_t s) {
    k_finalize<<<1, kBlock, 0, s>>>(part, nb, K, out);
}

}  // namespace stag
