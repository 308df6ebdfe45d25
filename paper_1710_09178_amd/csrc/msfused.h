// The fused multi-shift CG iteration (Sec. 4): the base system's update of
// step j-1 is folded into the D_oe launch of iteration j, which forms
// p_j = (r_{j-1} - alpha Ap_{j-1}) + beta p_{j-1} wherever it reads p_j (at
// the neighbours of its output sites, and once more for the even sites it
// owns, which it stores).  The shifted systems are updated per window by a
// separate flush launch.  Shared by the Dslash launcher (dslash.hip) and the
// flush kernels (blas.hip).
#pragma once

#include "common.h"

namespace stag {

// r_{j} = r_{j-1} - alpha Ap_{j-1} and p_j = r_j + beta p_{j-1} with explicit
// fused multiply-adds, so that the owner of a site and every block that forms
// the same value as a neighbour round identically.
__device__ __forceinline__ double2 cg_r_next(double2 r, double2 a, double alpha) {
    return make_double2(fma(-alpha, a.x, r.x), fma(-alpha, a.y, r.y));
}
__device__ __forceinline__ double2 cg_p_next(double2 rn, double2 p, double beta) {
    return make_double2(fma(beta, p.x, rn.x), fma(beta, p.y, rn.y));
}
// FP32 Krylov vectors: the same FP64 fused multiply-adds, rounded to FP32
// where the value is stored (and, identically, where a neighbour forms it)
__device__ __forceinline__ float2 cg_r_next(float2 r, float2 a, double alpha) {
    return make_float2((float)fma(-alpha, (double)a.x, (double)r.x), (float)fma(-alpha, (double)a.y, (double)r.y));
}
__device__ __forceinline__ float2 cg_p_next(float2 rn, float2 p, double beta) {
    return make_float2((float)fma(beta, (double)p.x, (double)rn.x), (float)fma(beta, (double)p.y, (double)rn.y));
}

// Launch constants of iteration j >= 1 of the fused loop; V: the Krylov
// vectors' precision (double2, or float2 for the FP32 form; the solutions
// stay FP64).
template <class V>
struct FusedIterT {
    V* ring;                // residual ring: r_i in slot i % lag
    const V* Ap;            // Ap_{j-1}
    const V* p_prev;        // p_{j-1}
    V* p_new;               // p_j (owned even sites)
    double2* x_base;        // solution of the base system
    MsState* st;
    const double* dpart;    // <p,Ap>, <r,Ap>, <Ap,Ap> partials of D_eo(j-1), nb2 each
    const double* qin;      // |r_{j-1}|^2 partials, nb2 of them
    double* qout;           // |r_j|^2 partials
    int nb2;                // blocks of the Dslash grid
    int par;                // j & 1: the launch reads done[par] and writes done[par ^ 1]
    int n, base, lag;
    int slot_prev, slot_new;   // (j - 1) % lag, j % lag
};
using FusedIter = FusedIterT<double2>;

// Scalars of step i = j - 1 from the block totals (rr = |r_i|^2 and the three
// dots of D_eo(i)), evaluated by wave 0, one lane per shift, with the same
// arithmetic as the unfused step kernel.  Block 0 writes the state of step j
// (or the final state when the solve stops), the window history of step i and
// the stop flag.  Returns alpha, beta, stop and whether the base system is
// still active, broadcast to the whole block.
struct StepOut {
    double alpha, beta;
    int stop, base_on;
};

// Step i's state as lane k of wave 0 needs it, loaded early (together with
// the partial sums) so that the scalars cost no extra memory round trip.
struct LaneState {
    double zeta, zeta_old, shift, alpha_old, beta_old, bb, tol2;
    int active, ipp, iter, bb_given, maxiter;
};

template <class FI>
__device__ __forceinline__ LaneState load_lane_state(const FI& f) {
    LaneState l{};
    const MsState* st = f.st;
    const MsIter& s = st->it[f.par ^ 1];
    const int k = threadIdx.x;
    if (k < 64) {
        if (k < f.n) {
            l.zeta = s.zeta[k];
            l.zeta_old = s.zeta_old[k];
            l.shift = st->shift[k];
            l.active = s.active[k];
            l.ipp = s.iters_per_pole[k];
        }
        l.alpha_old = s.alpha_old;
        l.beta_old = s.beta_old;
        l.bb = s.bb;
        l.tol2 = st->tol2;
        l.iter = s.iter;
        l.bb_given = st->bb_given;
        l.maxiter = st->maxiter;
    }
    return l;
}

template <class FI>
__device__ __forceinline__ StepOut fused_step_scalars(const FI& f, const double (&v)[4], const LaneState& ls) {
    __shared__ double sh_alpha, sh_beta;
    __shared__ int sh_stop, sh_base_on;
    MsState* st = f.st;
    const int n = f.n, base = f.base;
    const int k = threadIdx.x;
    const bool writer = blockIdx.x == 0;
    if (k < 64) {
        const int iter = ls.iter;
        const double rr = __shfl(v[0], 0), pAp = __shfl(v[1], 0), rAp = __shfl(v[2], 0), ApAp = __shfl(v[3], 0);
        const double bb = (iter == 0 && !ls.bb_given) ? rr : ls.bb;
        int nonfinite = !isfinite(rr);
        double alpha = 0.0, beta = 0.0;
        if (!nonfinite) {
            alpha = rr / pAp;
            double rr1 = rr - 2.0 * alpha * rAp + alpha * alpha * ApAp;
            if (rr1 < 0.0) rr1 = 0.0;
            beta = rr1 / rr;
        }
        int act = 0;
        double zn = 0.0, as = 0.0, bs = 0.0;
        if (k < n) {
            act = ls.active;
            if (act && ls.zeta * ls.zeta * rr <= ls.tol2 * bb) act = 0;
            const double z = ls.zeta, zo = ls.zeta_old;
            zn = z;
            if (k == base) {
                zn = 1.0;
                as = alpha;
                bs = beta;
            } else if (act) {
                const double a_old = ls.alpha_old, b_old = ls.beta_old;
                zn = z * zo * a_old / (alpha * b_old * (zo - z) + zo * a_old * (1.0 + ls.shift * alpha));
                const double q = zn / z;
                as = alpha * q;
                bs = beta * q * q;
            }
        }
        const unsigned long long any = __ballot(act != 0);
        if (any && !(isfinite(alpha) && isfinite(beta))) nonfinite = 1;
        const int stop = nonfinite || !any || iter >= ls.maxiter;
        if (writer && k < n) {
            MsIter& o = stop ? st->fin : st->it[f.par];
            o.active[k] = act;
            o.iters_per_pole[k] = (act && !stop) ? iter + 1 : (ls.active ? iter : ls.ipp);
            o.zeta[k] = stop ? ls.zeta : zn;
            o.zeta_old[k] = stop ? ls.zeta_old : ls.zeta;
            if (!stop) {
                MsHist& h = st->hist[f.slot_prev];
                h.as[k] = as;
                h.bs[k] = bs;
                h.zn[k] = zn;
                h.act[k] = act;
            }
        }
        const int base_act = __shfl(act, base);
        if (k == 0) {
            sh_alpha = alpha;
            sh_beta = beta;
            sh_stop = stop;
            sh_base_on = base_act;
            if (writer) {
                MsIter& o = stop ? st->fin : st->it[f.par];
                o.alpha_old = stop ? ls.alpha_old : alpha;
                o.beta_old = stop ? ls.beta_old : beta;
                o.bb = bb;
                o.rr = rr;
                o.iter = stop ? iter : iter + 1;
                o.nonfinite = nonfinite;
                if (stop) st->done[f.par ^ 1] = 1;
            }
        }
    }
    __syncthreads();
    return StepOut{sh_alpha, sh_beta, sh_stop, sh_base_on};
}

}  // namespace stag
