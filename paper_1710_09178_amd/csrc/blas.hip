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
#include "msfused.h"

namespace stag {

namespace {

// The init, restart and step kernels share one grid: EPT complex elements
// per thread (2, or 1 on small lattices, where more blocks shorten the
// latency-bound steps); the step sums the partials of init or of the previous
// step, one per block of that grid.
template <class V, int EPT>
__global__ __launch_bounds__(kBlock) void k_ms_init(int n3, const double2* __restrict__ b, V* __restrict__ r,
                                                    V* __restrict__ p, VecPtrs x, VecPtrs ps,
                                                    const MsState* __restrict__ st, double* __restrict__ qout) {
    const int n = st->n, base = st->base;
    double acc[1] = {0.0};
    for (int e = 0; e < EPT; ++e) {
        const int i = (blockIdx.x * EPT + e) * kBlock + threadIdx.x;
        if (i >= n3) continue;
        const double2 bv = b[i];
        const V bl = from_d2<V>(bv);
        r[i] = bl;
        p[i] = bl;
        for (int k = 0; k < n; ++k) {
            x.at<double2>(k)[i] = make_double2(0.0, 0.0);
            if (k != base) ps.at<V>(k)[i] = bl;
        }
        acc[0] += bv.x * bv.x + bv.y * bv.y;
    }
    block_partial<1>(acc, qout);
}

template <int EPT>
__global__ __launch_bounds__(kBlock) void k_cg_restart(int n3, const float2* __restrict__ r, float2* __restrict__ p,
                                                       double* __restrict__ qout) {
    double acc[1] = {0.0};
    for (int e = 0; e < EPT; ++e) {
        const int i = (blockIdx.x * EPT + e) * kBlock + threadIdx.x;
        if (i >= n3) continue;
        const float2 rv = r[i];
        p[i] = rv;
        const double2 d = to_d2(rv);
        acc[0] += d.x * d.x + d.y * d.y;
    }
    block_partial<1>(acc, qout);
}

// Non-temporal access for the per-pole streams (x_k, p_k): each is touched
// once per iteration, so they should not displace the links and the
// neighbour-shared vectors from the caches.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 nt_load(const double2* p) {
    const d2v t = __builtin_nontemporal_load((const d2v*)p);
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ float2 nt_load(const float2* p) {
    const f2v t = __builtin_nontemporal_load((const f2v*)p);
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ void nt_store(double2* p, double2 v) { __builtin_nontemporal_store(d2v{v.x, v.y}, (d2v*)p); }
__device__ __forceinline__ void nt_store(float2* p, float2 v) { __builtin_nontemporal_store(f2v{v.x, v.y}, (f2v*)p); }


// Iteration j (parity par):
//   rr_j   = sum of the <r,r> partials of the previous step (or of init)
//   freeze every shift with zeta_k^2 rr_j <= tol^2 <b,b>; stop if none is left
//   alpha  = rr_j / <p,Ap>,   rr_{j+1} = rr_j - 2 alpha <r,Ap> + alpha^2 <Ap,Ap>
//   beta   = rr_{j+1} / rr_j, zeta', alpha_s, beta_s from the shifted-CG recurrences
//   r_{j+1} = r_j - alpha Ap; x_base += alpha p; p = r_{j+1} + beta p;
//   for every active shift s: x_s += alpha_s p_s; p_s = zeta_s' r_{j+1} + beta_s p_s
// Every block evaluates the scalars itself (one thread per shift) from the
// partial sums, so all blocks agree bitwise without a grid barrier.
//
// The shifted updates are deferred over windows of L = st->lag iterations:
// r_j lives in ring slot j % L, the scalars of each iteration are kept in
// st->hist, and the last iteration of a window (or the stopping one) applies
// the window's updates to x_s and p_s in order, reading and writing each once
// instead of L times.  The arithmetic and its order are unchanged, so the
// results do not depend on L.
template <class V, int EPT>
__global__ __launch_bounds__(kBlock) void k_ms_step(int n3, V* __restrict__ ring, const V* __restrict__ Ap,
                                                    V* __restrict__ p, VecPtrs x, VecPtrs ps,
                                                    MsState* __restrict__ st, const double* __restrict__ dpart,
                                                    int nb2, const double* __restrict__ qin, double* __restrict__ qout,
                                                    int par, MsStepConst sc) {
    if (st->done[par]) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st->done[par ^ 1] = 1;
        return;
    }
    __shared__ double lds[16];
    __shared__ int sh_list[kMaxPoles];
    __shared__ double w_as[kLagMax][kMaxPoles], w_bs[kLagMax][kMaxPoles], w_zn[kLagMax][kMaxPoles];
    __shared__ int w_act[kLagMax][kMaxPoles];
    __shared__ double sh_alpha, sh_beta;
    __shared__ int sh_stop, sh_nact, sh_base_on;
    // n, base, lag and the ring slot come with the launch, so the stream
    // addresses below do not wait for the state
    const int n = sc.n, base = sc.base, L = sc.lag, slot = sc.slot;
    const MsIter& s = st->it[par];
    const int iter = s.iter;
    // Partial sums of the previous launches (<r,r> of the step or init, and
    // the three dots of the operator): each thread issues its first loads all
    // together, then the loads of the base system's streams, which do not
    // depend on this iteration's scalars, so that one memory round trip
    // covers all of them; the partials are still added in index order.
    constexpr int kUq = 4, kUd = 8;
    const int nbq = gridDim.x;  // init and step kernels use the same grid
    double tq[kUq], t1[kUd], t2[kUd], t3[kUd];
    // (unconditional loads from clamped indices, masked afterwards, so that
    // none of them sits behind a branch)
#pragma unroll
    for (int j = 0; j < kUq; ++j) tq[j] = qin[min((int)threadIdx.x + j * kBlock, nbq - 1)];
#pragma unroll
    for (int j = 0; j < kUd; ++j) {
        const int b = min((int)threadIdx.x + j * kBlock, nb2 - 1);
        t1[j] = dpart[b];
        t2[j] = dpart[nb2 + b];
        t3[j] = dpart[2 * nb2 + b];
    }
    double2 pre_r[EPT], pre_a[EPT], pre_p[EPT], pre_x[EPT];
    {
        const V* rc = ring + (size_t)slot * n3;
        const double2* xb = x.at<double2>(base);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = (blockIdx.x * EPT + e) * kBlock + threadIdx.x;
            if (i < n3) {
                pre_r[e] = to_d2(rc[i]);
                pre_a[e] = to_d2(Ap[i]);
                pre_p[e] = to_d2(p[i]);
                pre_x[e] = nt_load(xb + i);
            }
        }
    }
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kUq; ++j)
        if ((int)threadIdx.x + j * kBlock < nbq) v[0] += tq[j];
#pragma unroll
    for (int j = 0; j < kUd; ++j)
        if ((int)threadIdx.x + j * kBlock < nb2) {
            v[1] += t1[j];
            v[2] += t2[j];
            v[3] += t3[j];
        }
    for (int b = threadIdx.x + kUq * kBlock; b < nbq; b += kBlock) v[0] += qin[b];
    for (int b = threadIdx.x + kUd * kBlock; b < nb2; b += kBlock) {
        v[1] += dpart[b];
        v[2] += dpart[nb2 + b];
        v[3] += dpart[2 * nb2 + b];
    }
    block_sum<4>(v, lds);  // thread 0 holds the totals
    // Wave 0 evaluates the iteration's scalars, one lane per shift (n <= 48 < 64):
    // every lane computes alpha and beta from the same broadcast totals, and the
    // freezing test, the stop decision and the shift list use wave ballots.
    const int k = threadIdx.x;
    if (k < 64) {
        const double rr = __shfl(v[0], 0), pAp = __shfl(v[1], 0), rAp = __shfl(v[2], 0), ApAp = __shfl(v[3], 0);
        const double bb = (iter == 0 && !st->bb_given) ? rr : s.bb;
        int nonfinite = !isfinite(rr);
        double alpha = 0.0, beta = 0.0;
        if (!nonfinite) {
            alpha = rr / pAp;
            double rr1 = rr - 2.0 * alpha * rAp + alpha * alpha * ApAp;
            if (rr1 < 0.0) rr1 = 0.0;
            beta = rr1 / rr;
        }
        // freezing test and recurrences of shift k
        int act = 0;
        double zn = 0.0, as = 0.0, bs = 0.0;
        if (k < n) {
            act = s.active[k];
            if (act && s.zeta[k] * s.zeta[k] * rr <= st->tol2 * bb) act = 0;
            const double z = s.zeta[k], zo = s.zeta_old[k];
            zn = z;
            if (k == base) {
                zn = 1.0;
                as = alpha;
                bs = beta;
            } else if (act) {
                const double a_old = s.alpha_old, b_old = s.beta_old;
                zn = z * zo * a_old / (alpha * b_old * (zo - z) + zo * a_old * (1.0 + st->shift[k] * alpha));
                const double q = zn / z;
                as = alpha * q;
                bs = beta * q * q;
            }
        }
        const unsigned long long any = __ballot(act != 0);
        if (any && !(isfinite(alpha) && isfinite(beta))) nonfinite = 1;
        const int stop = nonfinite || !any || iter >= st->maxiter;
        // pending shifted updates: iterations iter - slot .. iter (.. iter - 1 when stopping)
        const int npend = stop ? slot : slot + 1;
        const int flush = npend > 0 && (stop || slot == L - 1);
        if (k < n) {
            if (flush) {
                for (int t = 0; t < slot; ++t) {
                    w_as[t][k] = st->hist[t].as[k];
                    w_bs[t][k] = st->hist[t].bs[k];
                    w_zn[t][k] = st->hist[t].zn[k];
                    w_act[t][k] = st->hist[t].act[k];
                }
                if (!stop) {
                    w_as[slot][k] = as;
                    w_bs[slot][k] = bs;
                    w_zn[slot][k] = zn;
                    w_act[slot][k] = act;
                }
            }
            if (blockIdx.x == 0 && blockIdx.y == 0) {
                // the state of the next iteration (or the final one)
                MsIter& o = stop ? st->fin : st->it[par ^ 1];
                o.active[k] = act;
                o.iters_per_pole[k] = (act && !stop) ? iter + 1 : (s.active[k] ? iter : s.iters_per_pole[k]);
                o.zeta[k] = stop ? s.zeta[k] : zn;
                o.zeta_old[k] = stop ? s.zeta_old[k] : s.zeta[k];
                if (!stop && !flush) {
                    st->hist[slot].as[k] = as;
                    st->hist[slot].bs[k] = bs;
                    st->hist[slot].zn[k] = zn;
                    st->hist[slot].act[k] = act;
                }
            }
        }
        // shifts to touch in a flush: those active in the window's first
        // iteration, in increasing order (this lane's own LDS write above)
        const int mine = flush && k < n && k != base && w_act[0][k];
        const unsigned long long lmask = __ballot(mine != 0);
        if (mine) sh_list[__popcll(lmask & ((1ull << k) - 1ull))] = k;
        const int base_act = __shfl(act, base);
        if (k == 0) {
            sh_alpha = alpha;
            sh_beta = beta;
            sh_stop = stop;
            sh_nact = __popcll(lmask);
            sh_base_on = base_act;
            if (blockIdx.x == 0 && blockIdx.y == 0) {
                MsIter& o = stop ? st->fin : st->it[par ^ 1];
                o.alpha_old = stop ? s.alpha_old : alpha;
                o.beta_old = stop ? s.beta_old : beta;
                o.bb = bb;
                o.rr = rr;
                o.iter = stop ? iter : iter + 1;
                o.nonfinite = nonfinite;
                if (stop) st->done[par ^ 1] = 1;
            }
        }
    }
    __syncthreads();
    const int stop = sh_stop;
    const int npend = stop ? slot : slot + 1;
    const bool flush = npend > 0 && (stop || slot == L - 1);
    if (stop && !flush) return;
    const double alpha = sh_alpha, beta = sh_beta;
    const bool base_on = sh_base_on;
    const int nact = sh_nact;
    V* r_next = ring + (size_t)((slot + 1) % L) * n3;
    // Launches at the end of a window of L >= 2 may carry gridDim.y > 1: row 0
    // updates the base system and every row takes the shift groups y,
    // y + gridDim.y, ... of the flush, so the flush of one element runs on
    // several blocks (each recomputes r_{j+1} from the same inputs, bitwise
    // alike).  Rows other than 0 read only what no block writes in this
    // launch: r_j (slot j % L, while r_{j+1} goes to another slot), Ap, the
    // older ring slots and their own shifts' x_s, p_s.
    const bool row0 = blockIdx.y == 0;
    double acc[1] = {0.0};
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = (blockIdx.x * EPT + e) * kBlock + threadIdx.x;
        if (i >= n3) continue;
        // r and p in the Krylov precision V, solutions accumulated in FP64
        const double2 r0 = pre_r[e];
        double2 rv = r0;
        if (!stop) {
            const double2 a = pre_a[e];
            const double2 pv = pre_p[e];
            double2* xb = x.at<double2>(base);
            rv.x -= alpha * a.x;
            rv.y -= alpha * a.y;
            const V rl = from_d2<V>(rv);
            rv = to_d2(rl);
            if (row0) {
                r_next[i] = rl;
                acc[0] += rv.x * rv.x + rv.y * rv.y;
                if (base_on) {
                    const double2 xbv = pre_x[e];
                    nt_store(xb + i, make_double2(xbv.x + alpha * pv.x, xbv.y + alpha * pv.y));
                }
                p[i] = from_d2<V>(make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y));
            }
        }
        if (!flush) continue;
        // residuals r_{i+1} of the pending iterations i = iter - slot + t
        double2 rw[kLagMax];
#pragma unroll
        for (int t = 0; t < kLagMax; ++t) {
            if (t >= npend) break;
            const int it_next = iter - slot + t + 1;
            if (it_next == iter + 1)
                rw[t] = rv;
            else if (it_next == iter)
                rw[t] = r0;
            else
                rw[t] = to_d2(ring[(size_t)(it_next % L) * n3 + i]);
        }
        // shifted poles in groups: all loads of a group are issued before its
        // stores (the pointers may not be proven distinct by the compiler)
        constexpr int G = kFlushGroup;
        for (int g0 = blockIdx.y * G; g0 < nact; g0 += gridDim.y * G) {
            double2 pk[G], xk[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (g0 + j < nact) {
                    const int q = sh_list[g0 + j];
                    pk[j] = to_d2(nt_load(ps.at<V>(q) + i));
                    xk[j] = nt_load(x.at<double2>(q) + i);
                }
            }
#pragma unroll
            for (int t = 0; t < kLagMax; ++t) {
                if (t >= npend) break;
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    if (g0 + j < nact) {
                        const int q = sh_list[g0 + j];
                        if (w_act[t][q]) {
                            const double aq = w_as[t][q], bq = w_bs[t][q], zq = w_zn[t][q];
                            xk[j] = make_double2(xk[j].x + aq * pk[j].x, xk[j].y + aq * pk[j].y);
                            // p_s is kept in the Krylov precision between iterations
                            pk[j] = to_d2(from_d2<V>(make_double2(zq * rw[t].x + bq * pk[j].x,
                                                                  zq * rw[t].y + bq * pk[j].y)));
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (g0 + j < nact) {
                    const int q = sh_list[g0 + j];
                    nt_store(x.at<double2>(q) + i, xk[j]);
                    nt_store(ps.at<V>(q) + i, from_d2<V>(pk[j]));
                }
            }
        }
    }
    if (row0) block_partial<1>(acc, qout);
}

// Window flush of the fused loop: the shifted systems' updates of npend
// consecutive steps i0 .. i0 + npend - 1 (i0 a multiple of L), applied in
// order to x_s, p_s of every shift active in step i0, from the scalars in
// st->hist[t] and the residuals r_{i0+t+1} in ring slot (t + 1) % L -- the
// arithmetic of the unfused step kernel's flush.  final = 0: launched after
// iteration j = i0 + L, npend = L, skipped once the solve has stopped (gate);
// final = 1: once after the loop, npend = fin.iter % L (the steps pending at
// the stop).  Block row y takes the shift groups y, y + gridDim.y, ...
template <class V, int EPT>
__global__ __launch_bounds__(kBlock) void k_ms_flush(int n3, const V* __restrict__ ring, VecPtrs x, VecPtrs ps,
                                                     const MsState* __restrict__ st, const int* __restrict__ gate,
                                                     int n, int base, int L, int final_flush) {
    if (!final_flush && *gate) return;
    const int npend = final_flush ? st->fin.iter % L : L;
    if (npend == 0) return;
    __shared__ double w_as[kLagMax][kMaxPoles], w_bs[kLagMax][kMaxPoles], w_zn[kLagMax][kMaxPoles];
    __shared__ int w_act[kLagMax][kMaxPoles];
    __shared__ int sh_list[kMaxPoles];
    __shared__ int sh_nact;
    const int k = threadIdx.x;
    if (k < 64) {
        if (k < n)
            for (int t = 0; t < npend; ++t) {
                w_as[t][k] = st->hist[t].as[k];
                w_bs[t][k] = st->hist[t].bs[k];
                w_zn[t][k] = st->hist[t].zn[k];
                w_act[t][k] = st->hist[t].act[k];
            }
        const int mine = k < n && k != base && st->hist[0].act[k];
        const unsigned long long lmask = __ballot(mine != 0);
        if (mine) sh_list[__popcll(lmask & ((1ull << k) - 1ull))] = k;
        if (k == 0) sh_nact = __popcll(lmask);
    }
    __syncthreads();
    const int nact = sh_nact;
    constexpr int G = kFlushGroup;
    for (int e = 0; e < EPT; ++e) {
        const int i = (blockIdx.x * EPT + e) * kBlock + threadIdx.x;
        if (i >= n3) continue;
        double2 rw[kLagMax];
#pragma unroll
        for (int t = 0; t < kLagMax; ++t) {
            if (t >= npend) break;
            rw[t] = to_d2(ring[(size_t)((t + 1) % L) * n3 + i]);
        }
        for (int g0 = blockIdx.y * G; g0 < nact; g0 += gridDim.y * G) {
            double2 pk[G], xk[G];
#pragma unroll
            for (int jj = 0; jj < G; ++jj) {
                if (g0 + jj < nact) {
                    const int q = sh_list[g0 + jj];
                    pk[jj] = to_d2(nt_load(ps.at<V>(q) + i));
                    xk[jj] = nt_load(x.at<double2>(q) + i);
                }
            }
#pragma unroll
            for (int t = 0; t < kLagMax; ++t) {
                if (t >= npend) break;
#pragma unroll
                for (int jj = 0; jj < G; ++jj) {
                    if (g0 + jj < nact) {
                        const int q = sh_list[g0 + jj];
                        if (w_act[t][q]) {
                            const double aq = w_as[t][q], bq = w_bs[t][q], zq = w_zn[t][q];
                            xk[jj] = make_double2(xk[jj].x + aq * pk[jj].x, xk[jj].y + aq * pk[jj].y);
                            // p_s is kept in the Krylov precision between steps
                            pk[jj] = to_d2(from_d2<V>(make_double2(zq * rw[t].x + bq * pk[jj].x,
                                                                   zq * rw[t].y + bq * pk[jj].y)));
                        }
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < G; ++jj) {
                if (g0 + jj < nact) {
                    const int q = sh_list[g0 + jj];
                    nt_store(x.at<double2>(q) + i, xk[jj]);
                    nt_store(ps.at<V>(q) + i, from_d2<V>(pk[jj]));
                }
            }
        }
    }
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
        const double2 v = x.at<double2>(k)[i];
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

// v *= 1 / sqrt(s2[0]) (normalisation inside the power iteration)
__global__ __launch_bounds__(kBlock) void k_scale_rsqrt(int n3, double2* __restrict__ v, const double* __restrict__ s2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n3) return;
    const double f = 1.0 / sqrt(s2[0]);
    const double2 a = v[i];
    v[i] = make_double2(f * a.x, f * a.y);
}

__global__ __launch_bounds__(kBlock) void k_finalize_pad(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out, int npad) {
    __shared__ double lds[4];
    const double t = sum_partials(part, nb, lds);
    for (int i = threadIdx.x; i < npad; i += kBlock) out[i] = (i == 0) ? t : 0.0;
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
// elements per thread of the init / step / restart kernels: 1 when two per
// thread would leave fewer than 512 blocks
inline int ms_ept(const Geom& g) { return (3 * g.vh + 2 * kBlock - 1) / (2 * kBlock) < 512 ? 1 : 2; }
inline int gridq(const Geom& g) {
    const int ept = ms_ept(g);
    return (3 * g.vh + kBlock * ept - 1) / (kBlock * ept);
}

}  // namespace

int ms_update_grid(const Geom& g) { return gridq(g); }
int dot_grid(const Geom& g) { return grid3(g); }

template <class V>
void launch_ms_init(const Geom& g, const double2* b, V* r, V* p, VecPtrs x, VecPtrs ps, const MsState* st,
                    double* qout, hipStream_t s) {
    if (ms_ept(g) == 1)
        k_ms_init<V, 1><<<gridq(g), kBlock, 0, s>>>(3 * g.vh, b, r, p, x, ps, st, qout);
    else
        k_ms_init<V, 2><<<gridq(g), kBlock, 0, s>>>(3 * g.vh, b, r, p, x, ps, st, qout);
}
template void launch_ms_init<double2>(const Geom&, const double2*, double2*, double2*, VecPtrs, VecPtrs,
                                      const MsState*, double*, hipStream_t);
template void launch_ms_init<float2>(const Geom&, const double2*, float2*, float2*, VecPtrs, VecPtrs,
                                     const MsState*, double*, hipStream_t);

template <class V>
void launch_ms_step(const Geom& g, V* r, const V* Ap, V* p, VecPtrs x, VecPtrs ps, MsState* st, const double* dpart,
                    int nb2, const double* qin, double* qout, int par, int rows, MsStepConst sc, hipStream_t s) {
    if (ms_ept(g) == 1)
        timed_launch(k_ms_step<V, 1>, dim3(gridq(g), rows), dim3(kBlock), s, 3 * g.vh, r, Ap, p, x, ps, st, dpart, nb2,
                     qin, qout, par, sc);
    else
        timed_launch(k_ms_step<V, 2>, dim3(gridq(g), rows), dim3(kBlock), s, 3 * g.vh, r, Ap, p, x, ps, st, dpart, nb2,
                     qin, qout, par, sc);
}
template void launch_ms_step<double2>(const Geom&, double2*, const double2*, double2*, VecPtrs, VecPtrs, MsState*,
                                      const double*, int, const double*, double*, int, int, MsStepConst,
                                      hipStream_t);
template void launch_ms_step<float2>(const Geom&, float2*, const float2*, float2*, VecPtrs, VecPtrs, MsState*,
                                     const double*, int, const double*, double*, int, int, MsStepConst,
                                     hipStream_t);

template <class V>
void launch_ms_flush(const Geom& g, const V* ring, VecPtrs x, VecPtrs ps, const MsState* st, const int* gate,
                     int n, int base, int L, bool final_flush, int rows, hipStream_t s) {
    if (ms_ept(g) == 1)
        timed_launch(k_ms_flush<V, 1>, dim3(gridq(g), rows), dim3(kBlock), s, 3 * g.vh, ring, x, ps, st, gate, n, base,
                     L, (int)final_flush);
    else
        timed_launch(k_ms_flush<V, 2>, dim3(gridq(g), rows), dim3(kBlock), s, 3 * g.vh, ring, x, ps, st, gate, n, base,
                     L, (int)final_flush);
}
template void launch_ms_flush<double2>(const Geom&, const double2*, VecPtrs, VecPtrs, const MsState*, const int*, int,
                                       int, int, bool, int, hipStream_t);
template void launch_ms_flush<float2>(const Geom&, const float2*, VecPtrs, VecPtrs, const MsState*, const int*, int,
                                      int, int, bool, int, hipStream_t);

void launch_cg_restart(const Geom& g, const float2* r, float2* p, double* qout, hipStream_t s) {
    if (ms_ept(g) == 1)
        k_cg_restart<1><<<gridq(g), kBlock, 0, s>>>(3 * g.vh, r, p, qout);
    else
        k_cg_restart<2><<<gridq(g), kBlock, 0, s>>>(3 * g.vh, r, p, qout);
}

void launch_rational_sum(const Geom& g, const double2* b, VecPtrs x, const MsState* st, double2* out,
                         hipStream_t s) {
    k_rational_sum<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, b, x, st, out);
}

void launch_dot_re(const Geom& g, const double2* a, const double2* b, double* part, hipStream_t s) {
    k_dot_re<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, a, b, part);
}

void launch_scale_rsqrt(const Geom& g, double2* v, const double* s2, hipStream_t s) {
    k_scale_rsqrt<<<grid3(g), kBlock, 0, s>>>(3 * g.vh, v, s2);
}

void launch_finalize_pad(const double* part, int nb, double* out, int npad, hipStream_t s) {
    k_finalize_pad<<<1, kBlock, 0, s>>>(part, nb, out, npad);
}

void launch_finalize(const double* part, int nb, int K, double* out, hipStream_t s) {
    k_finalize<<<1, kBlock, 0, s>>>(part, nb, K, out);
}

}  // namespace stag
