// extern "C" entry points of libstag: handle management, argument checks,
// field conversions, the multi-shift CG driver (Sec. 4), forces and the RHMC
// trajectory (Sec. 3.1).  All device work goes to one internal stream that is
// ordered after / before the caller's stream with events.
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "observables.h"

using namespace stag;

namespace {
thread_local std::string g_create_err;
}

namespace stag {
// |a - b|^2 and |b|^2 over n reals into out2[0..1] (force.hip)
void launch_diff_norm2(size_t n, const double* a, const double* b, double* part, double* out2, hipStream_t s);
}  // namespace stag

namespace stag {
stag_status fail(stag_ctx* c, stag_status code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return code;
}
}  // namespace stag

namespace {

bool aligned16(const void* p) { return p && ((uintptr_t)p % 16 == 0); }

stag_status check_rational(stag_ctx* c, const stag_rational* r, double mass) {
    if (!r) return fail(c, STAG_ERR_INVALID_ARG, "rational function is NULL");
    if (r->n < 1 || r->n > STAG_MAX_POLES)
        return fail(c, STAG_ERR_INVALID_ARG, "number of poles must be in [1, " + std::to_string(STAG_MAX_POLES) + "]");
    if (!r->pole || !r->residue) return fail(c, STAG_ERR_INVALID_ARG, "pole/residue arrays are NULL");
    double mn = 1e300;
    for (int k = 0; k < r->n; ++k) {
        if (!std::isfinite(r->pole[k]) || r->pole[k] < 0.0)
            return fail(c, STAG_ERR_INVALID_ARG, "poles must be finite and >= 0");
        if (!std::isfinite(r->residue[k])) return fail(c, STAG_ERR_INVALID_ARG, "residues must be finite");
        mn = std::min(mn, r->pole[k]);
    }
    if (!std::isfinite(r->c0)) return fail(c, STAG_ERR_INVALID_ARG, "c0 must be finite");
    if (!(4.0 * mass * mass + mn > 0.0))
        return fail(c, STAG_ERR_INVALID_ARG, "4 m^2 + smallest pole must be > 0 (operator would be singular)");
    return STAG_OK;
}

stag_status check_common(stag_ctx* c, bool need_gauge) {
    if (!c) return fail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (need_gauge && !c->has_gauge) return fail(c, STAG_ERR_NO_GAUGE, "no gauge field set (call stag_set_gauge)");
    return STAG_OK;
}

// order the internal stream after the caller's stream
stag_status enter(stag_ctx* c) {
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    HIP_OR_FAIL(c, hipEventRecord(c->ev_in, c->user));
    HIP_OR_FAIL(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    return STAG_OK;
}

// order the caller's stream after the internal stream
stag_status leave(stag_ctx* c) {
    HIP_OR_FAIL(c, hipGetLastError());
    HIP_OR_FAIL(c, hipEventRecord(c->ev_out, c->s));
    HIP_OR_FAIL(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    return STAG_OK;
}

stag_status finish_solve_status(stag_ctx* c, const SolveResult& res) {
    if (res.nonfinite) return fail(c, STAG_ERR_NONFINITE, "non-finite value in the solver (NaN/Inf in the input?)");
    if (!res.converged) return fail(c, STAG_ERR_NOT_CONVERGED, "multi-shift CG reached maxiter before convergence");
    return STAG_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

stag_status reduce_to_host(stag_ctx* c, double* out) {
    HIP_OR_FAIL(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    *out = c->scal_host[0];
    return STAG_OK;
}

// S_f = Re <phi, r(A) phi>; uses tmp_e
stag_status fermion_action_impl(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter,
                                const double2* phi, double* S, SolveResult& res) {
    stag_status e = ensure_pool(c, r->n);
    if (e != STAG_OK) return e;
    std::vector<double2*> xs(r->n);
    for (int k = 0; k < r->n; ++k) xs[k] = pool_vec(c->pool_x, c->g, k);
    if ((e = ms_solve(c, mass, r, tol, maxiter, phi, xs.data(), false, nullptr, nullptr, res)) != STAG_OK) return e;
    VecPtrs X{};
    for (int k = 0; k < r->n; ++k) X.p[k] = xs[k];
    launch_rational_sum(c->g, phi, X, c->st, c->tmp_e, c->s);
    launch_dot_re(c->g, phi, c->tmp_e, c->gpart, c->s);
    launch_finalize(c->gpart, dot_grid(c->g), 1, c->scal, c->s);
    return reduce_to_host(c, S);
}

// mom = F (dt == 0) or mom += dt F; sloppy != 0: the solve runs with FP32
// Krylov vectors and links in that format (no refinement)
stag_status fermion_force_impl(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter,
                               const double2* phi, double* mom, double dt, SolveResult& res, int sloppy = 0) {
    stag_status e = ensure_pool(c, r->n);
    if (e != STAG_OK) return e;
    const Geom& g = c->g;
    std::vector<double2*> xs(r->n);
    for (int k = 0; k < r->n; ++k) xs[k] = pool_vec(c->pool_x, g, k);
    e = sloppy ? ms_solve_sloppy(c, sloppy, mass, r, tol, maxiter, phi, xs.data(), res)
               : ms_solve(c, mass, r, tol, maxiter, phi, xs.data(), false, nullptr, nullptr, res);
    if (e != STAG_OK) return e;
    LinkSet ls;
    if ((e = get_links(c, -1, ls))) return e;
    VecPtrs X{}, Y{};
    for (int k = 0; k < r->n; ++k) {
        X.p[k] = xs[k];
        Y.p[k] = pool_vec(c->pool_y, g, k);
        launch_dslash(g, ls, xs[k], pool_vec(c->pool_y, g, k), 1, c->tps, nullptr, c->s);
    }
    const double* coef = (const double*)((const char*)c->st + offsetof(MsState, coef));
    launch_fermion_force(g, c->links, X, Y, coef, r->n, mom, dt, c->s, c->naik ? c->naik_c1 : 1.0);
    if (c->naik) {
        if (!c->naik_w3 && (e = dmalloc(c, &c->naik_w3, (size_t)72 * g.vh * sizeof(double2)))) return e;
        launch_naik_force3(g, c->links, X, Y, coef, r->n, c->naik_w3, c->naik_c3, mom, dt, c->s);
    }
    return STAG_OK;
}

// Rayleigh quotient <v, A v> / <v, v> after `iters` power iterations from the
// estimator-noise vector (seed, 0); v is normalised every 8 applications (the
// quotient does not depend on the scale).  Uses p, Ap and tmp_o.
stag_status power_rayleigh_impl(stag_ctx* c, double mass, int iters, uint64_t seed, double* lam) {
    const Geom& g = c->g;
    LinkSet ls;
    stag_status e = get_links(c, -1, ls);
    if (e) return e;
    const double m2 = 4.0 * mass * mass;
    double2 *v = c->p, *t = c->Ap;
    launch_random_source(g, seed, 0, v, c->s, kFieldNoise);
    for (int k = 0; k < iters; ++k) {
        launch_dslash(g, ls, v, c->tmp_o, 1, c->tps, nullptr, c->s);
        launch_dslash_axpy(g, ls, c->tmp_o, v, m2, t, c->tps, c->s);
        if (k % 8 == 7 || k == iters - 1) {
            launch_dot_re(g, t, t, c->gpart, c->s);
            launch_finalize(c->gpart, dot_grid(g), 1, c->scal, c->s);
            launch_scale_rsqrt(g, t, c->scal, c->s);
        }
        std::swap(v, t);
    }
    launch_dslash(g, ls, v, c->tmp_o, 1, c->tps, nullptr, c->s);
    launch_dslash_axpy(g, ls, c->tmp_o, v, m2, t, c->tps, c->s);
    launch_dot_re(g, v, t, c->gpart, c->s);
    launch_finalize(c->gpart, dot_grid(g), 1, c->scal, c->s);
    launch_dot_re(g, v, v, c->gpart, c->s);
    launch_finalize(c->gpart, dot_grid(g), 1, c->scal + 1, c->s);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->scal_host, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    *lam = c->scal_host[0] / c->scal_host[1];
    if (!std::isfinite(*lam)) return fail(c, STAG_ERR_NONFINITE, "non-finite value in the power iteration");
    return STAG_OK;
}

// Interval [xmin, xmax] of a rational table against the spectrum of A: the
// table must reach below 4m^2 (the exact lower bound) and above lambda_max,
// either for certain (xmax >= 4m^2 + dmax^2 with dmax = 8 >= |D_oe|, or
// 8 (|c1| + |c3|) for the improved operator) or with a margin of 10% over the
// power estimate after 100 iterations (which lies below lambda_max).
constexpr int kSpectrumIters = 100;
constexpr double kSpectrumMargin = 0.1;
stag_status spectrum_check_impl(stag_ctx* c, double mass, double xmin, double xmax, double* lam_out) {
    const double lo = 4.0 * mass * mass;
    if (lam_out) *lam_out = 0.0;
    if (xmin > lo) {
        char buf[160];
        snprintf(buf, sizeof buf, "rational interval starts at %.6g, above the lower spectral bound 4m^2 = %.6g", xmin,
                 lo);
        return fail(c, STAG_ERR_SPECTRUM, buf);
    }
    const double dmax = c->naik ? 8.0 * (std::fabs(c->naik_c1) + std::fabs(c->naik_c3)) : 8.0;
    if (xmax >= lo + dmax * dmax) return STAG_OK;
    double lam = 0.0;
    stag_status e = power_rayleigh_impl(c, mass, kSpectrumIters, 0, &lam);
    if (e) return e;
    if (lam_out) *lam_out = lam;
    if ((1.0 + kSpectrumMargin) * lam > xmax) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "rational interval ends at %.6g, below 1.1 x the estimated largest eigenvalue %.6g of A", xmax, lam);
        return fail(c, STAG_ERR_SPECTRUM, buf);
    }
    return STAG_OK;
}

stag_status gauge_action_impl(stag_ctx* c, double beta, double* S, double* plaq) {
    const int nb = launch_plaquette(c->g, c->links, c->gpart, c->s);
    launch_finalize(c->gpart, nb, 1, c->scal, c->s);
    double sum = 0.0;
    stag_status e = reduce_to_host(c, &sum);
    if (e != STAG_OK) return e;
    const double V = 2.0 * c->g.vh;
    if (S) *S = beta * (6.0 * V - sum / 3.0);
    if (plaq) *plaq = sum / (3.0 * 6.0 * V);
    return STAG_OK;
}

stag_status kinetic_impl(stag_ctx* c, const double* mom, double* K) {
    const int nb = launch_kinetic(c->g, mom, c->gpart, c->s);
    launch_finalize(c->gpart, nb, 1, c->scal, c->s);
    double sum = 0.0;
    stag_status e = reduce_to_host(c, &sum);
    if (e != STAG_OK) return e;
    *K = 0.5 * sum;
    return STAG_OK;
}

}  // namespace

extern "C" {

stag_status stag_create(stag_handle* out, const int dims[4], void* hip_stream) {
    if (!out || !dims) return fail(nullptr, STAG_ERR_INVALID_ARG, "out/dims is NULL");
    *out = nullptr;
    long long V = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 2 || dims[i] % 2)
            return fail(nullptr, STAG_ERR_INVALID_ARG, "every lattice extent must be even and >= 2");
        V *= dims[i];
    }
    if (V >= (1LL << 31) / 8) return fail(nullptr, STAG_ERR_INVALID_ARG, "lattice too large for 32-bit indexing");
    stag_ctx* c = new stag_ctx();
    for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
    c->g = Geom{dims[0], dims[1], dims[2], dims[3], dims[0] / 2, (int)(V / 2)};
    if (const char* e = std::getenv("STAG_TPS")) c->tps = std::atoi(e);
    if (c->tps != 1 && c->tps != 2 && c->tps != 4) c->tps = 2;
    if (const char* e = std::getenv("STAG_CHUNK")) c->chunk = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("STAG_FUSED")) c->fused = std::max(0, std::min(2, std::atoi(e)));
    if (const char* e = std::getenv("STAG_LINK_NT")) c->link_nt = std::max(0, std::min(2, std::atoi(e)));
    c->user = (hipStream_t)hip_stream;
    auto bail = [&](stag_status s) {
        g_create_err = c->err;
        stag_destroy(c);
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(nullptr, STAG_ERR_HIP, "no HIP device available");
    }
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->chunk_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->chunk_ev[1], hipEventDisableTiming) != hipSuccess) {
        c->err = "stream/event creation failed";
        return bail(STAG_ERR_HIP);
    }
    const Geom& g = c->g;
    const size_t hb = half_bytes(g);
    const size_t lb = (size_t)2 * 4 * 9 * g.vh * sizeof(double2);
    const size_t mb = (size_t)2 * 4 * 8 * g.vh * sizeof(double);
    stag_status s;
    if ((s = dmalloc(c, &c->links, lb)) || (s = dmalloc(c, &c->links_backup, lb)) || (s = dmalloc(c, &c->mom, mb)) ||
        (s = dmalloc(c, &c->r, kLagMax * hb)) || (s = dmalloc(c, &c->p, hb)) || (s = dmalloc(c, &c->p2, hb)) || (s = dmalloc(c, &c->Ap, hb)) ||
        (s = dmalloc(c, &c->w_o, hb)) || (s = dmalloc(c, &c->tmp_e, hb)) || (s = dmalloc(c, &c->tmp_o, hb)) ||
        (s = dmalloc(c, &c->xi, hb)) || (s = dmalloc(c, &c->phi, hb)) || (s = dmalloc(c, &c->st, sizeof(MsState))) ||
        (s = dmalloc(c, &c->scal, 64)))
        return bail(s);
    // one partial per block of the largest reduction grid (Dslash with 64 sites
    // per block, or the element-wise kernels with 256 elements per block)
    const size_t nparts = std::max<size_t>(4096, (size_t)g.vh / 32 + 16);
    if ((s = dmalloc(c, &c->dpart, nparts * 3 * sizeof(double))) ||
        (s = dmalloc(c, &c->qpart[0], nparts * sizeof(double))) ||
        (s = dmalloc(c, &c->qpart[1], nparts * sizeof(double))) ||
        (s = dmalloc(c, &c->gpart, nparts * 3 * sizeof(double))))
        return bail(s);
    if (hipHostMalloc((void**)&c->st_host, sizeof(MsState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->scal_host, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->done_host, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        c->err = "pinned host allocation failed";
        return bail(STAG_ERR_OOM);
    }
    if ((s = scratch_init(c))) return bail(s);
    launch_fill_zero(c->mom, mb, c->s);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        c->err = "initialisation kernels failed";
        return bail(STAG_ERR_HIP);
    }
    *out = c;
    return STAG_OK;
}

stag_status stag_destroy(stag_handle c) {
    if (!c) return STAG_OK;
    if (c->s) hipStreamSynchronize(c->s);
    void* bufs[] = {c->links_d12, c->links_s18, c->links_h12, c->long_d18, c->long_d12, c->long_s18, c->long_h12,
                    c->naik_w3, c->r32, c->p32, c->p2_32, c->Ap32, c->w32,
                    c->links, c->links_backup, c->mom, c->r, c->p, c->p2, c->Ap, c->w_o, c->tmp_e, c->tmp_o, c->xi,
                    c->phi, c->pool_x, c->pool_p, c->pool_y, c->st, c->dpart, c->qpart[0], c->qpart[1],
                    c->gpart, c->scal, c->mom_tmp, c->mom_aux, c->mom_judge};
    for (void* b : bufs)
        if (b) hipFree(b);
    if (c->st_host) hipHostFree(c->st_host);
    if (c->scal_host) hipHostFree(c->scal_host);
    if (c->done_host) hipHostFree(c->done_host);
    for (auto ev : c->prof_ev) hipEventDestroy(ev);
    for (auto& gr : c->graphs) hipGraphExecDestroy(gr.exec);
    hipEvent_t evs[] = {c->ev_in, c->ev_out, c->chunk_ev[0], c->chunk_ev[1]};
    for (auto ev : evs)
        if (ev) hipEventDestroy(ev);
    if (c->s) hipStreamDestroy(c->s);
    delete c;
    return STAG_OK;
}

const char* stag_last_error(stag_handle c) { return c ? c->err.c_str() : g_create_err.c_str(); }

size_t stag_field_bytes(stag_handle c, int kind) {
    if (!c) return 0;
    const size_t vh = c->g.vh, V = 2 * vh;
    switch (kind) {
        case STAG_FIELD_HALF_VEC: return 3 * vh * 16;
        case STAG_FIELD_MOM: return 64 * vh * 8;
        case STAG_FIELD_CANON_HALF_VEC: return 3 * vh * 16;
        case STAG_FIELD_CANON_GAUGE: return V * 4 * 9 * 16;
        case STAG_FIELD_CANON_MOM: return V * 4 * 8 * 8;
        default: return 0;
    }
}

stag_status stag_set_gauge(stag_handle c, const double* U) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(U)) return fail(c, STAG_ERR_INVALID_ARG, "gauge pointer is NULL or not 16-byte aligned");
    if ((e = enter(c))) return e;
    launch_gauge_to_internal(c->g, (const double2*)U, c->links, c->s);
    links_changed(c);
    c->has_gauge = true;
    return leave(c);
}

stag_status stag_get_gauge(stag_handle c, double* U) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(U)) return fail(c, STAG_ERR_INVALID_ARG, "gauge pointer is NULL or not 16-byte aligned");
    if ((e = enter(c))) return e;
    launch_gauge_to_canon(c->g, c->links, (double2*)U, c->s);
    return leave(c);
}

stag_status stag_vec_import(stag_handle c, void* out, const double* in, int parity) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in)) return fail(c, STAG_ERR_INVALID_ARG, "vector pointer NULL or misaligned");
    if (parity != 0 && parity != 1) return fail(c, STAG_ERR_INVALID_ARG, "parity must be 0 or 1");
    if (out == (const void*)in) return fail(c, STAG_ERR_INVALID_ARG, "in and out must differ");
    if ((e = enter(c))) return e;
    launch_vec_to_internal(c->g, (const double2*)in, (double2*)out, c->s);
    return leave(c);
}

stag_status stag_vec_export(stag_handle c, double* out, const void* in, int parity) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in)) return fail(c, STAG_ERR_INVALID_ARG, "vector pointer NULL or misaligned");
    if (parity != 0 && parity != 1) return fail(c, STAG_ERR_INVALID_ARG, "parity must be 0 or 1");
    if ((const void*)out == in) return fail(c, STAG_ERR_INVALID_ARG, "in and out must differ");
    if ((e = enter(c))) return e;
    launch_vec_to_canon(c->g, (const double2*)in, (double2*)out, c->s);
    return leave(c);
}

stag_status stag_mom_import(stag_handle c, void* out, const double* in) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || out == (const void*)in)
        return fail(c, STAG_ERR_INVALID_ARG, "momentum pointers NULL, misaligned or equal");
    if ((e = enter(c))) return e;
    launch_mom_to_internal(c->g, in, (double*)out, 0, c->s);
    return leave(c);
}

stag_status stag_mom_export(stag_handle c, double* out, const void* in) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || (const void*)out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "momentum pointers NULL, misaligned or equal");
    if ((e = enter(c))) return e;
    launch_mom_to_canon(c->g, (const double*)in, out, c->s);
    return leave(c);
}

stag_status stag_dslash(stag_handle c, void* out, const void* in, int out_parity) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "vector pointers NULL, misaligned or equal");
    if (out_parity != 0 && out_parity != 1) return fail(c, STAG_ERR_INVALID_ARG, "parity must be 0 or 1");
    if ((e = enter(c))) return e;
    LinkSet ls;
    if ((e = get_links(c, -1, ls))) return e;
    const bool timed = c->prof_on && c->prof_ev.size() >= 2;
    if (timed) next_launch_timing() = LaunchTiming{c->prof_ev[0], c->prof_ev[1]};
    launch_dslash(c->g, ls, (const double2*)in, (double2*)out, out_parity, c->tps, nullptr, c->s);
    if (timed) {
        // measurement mode: wait for the launch and book it as D_oe / D_eo
        HIP_OR_FAIL(c, hipEventSynchronize(c->prof_ev[1]));
        float ms = 0.f;
        HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->prof_ev[0], c->prof_ev[1]));
        const int kind = out_parity == 1 ? 0 : 1;
        c->prof_ms[kind] += ms;
        c->prof_cnt[kind] += 1;
        c->prof_samples[kind].push_back(ms);
    }
    return leave(c);
}

stag_status stag_mdagm(stag_handle c, void* out, const void* in, double mass) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "vector pointers NULL, misaligned or equal");
    if (!std::isfinite(mass)) return fail(c, STAG_ERR_INVALID_ARG, "mass must be finite");
    if ((e = enter(c))) return e;
    LinkSet ls;
    if ((e = get_links(c, -1, ls))) return e;
    launch_dslash(c->g, ls, (const double2*)in, c->tmp_o, 1, c->tps, nullptr, c->s);
    launch_dslash_axpy(c->g, ls, c->tmp_o, (const double2*)in, 4.0 * mass * mass, (double2*)out, c->tps, c->s);
    return leave(c);
}

stag_status stag_power_estimate(stag_handle c, double mass, int iters, uint64_t seed, double* lam_out) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!std::isfinite(mass) || iters < 0 || !lam_out)
        return fail(c, STAG_ERR_INVALID_ARG, "need a finite mass, iters >= 0 and lam_out");
    if ((e = enter(c))) return e;
    if ((e = power_rayleigh_impl(c, mass, iters, seed, lam_out))) return e;
    return leave(c);
}

stag_status stag_check_spectrum(stag_handle c, double mass, double xmin, double xmax, double* lam_out) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!std::isfinite(mass) || !std::isfinite(xmin) || !std::isfinite(xmax) || !(xmin < xmax))
        return fail(c, STAG_ERR_INVALID_ARG, "need a finite mass and xmin < xmax");
    if ((e = enter(c))) return e;
    const stag_status chk = spectrum_check_impl(c, mass, xmin, xmax, lam_out);
    if ((e = leave(c))) return e;
    return chk;
}

// The precision form's sloppy operator applied to FP64 vectors (input
// rounded to FP32, output widened): what the FP32 Krylov solves apply.
stag_status stag_dslash_sloppy(stag_handle c, void* out, const void* in, int out_parity, int format) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "vector pointers NULL, misaligned or equal");
    if (out_parity != 0 && out_parity != 1) return fail(c, STAG_ERR_INVALID_ARG, "parity must be 0 or 1");
    if (format != STAG_LINKS_F32_18 && format != STAG_LINKS_F16_12)
        return fail(c, STAG_ERR_INVALID_ARG, "sloppy format must be STAG_LINKS_F32_18 or STAG_LINKS_F16_12");
    if ((e = enter(c))) return e;
    LinkSet ls;
    if ((e = get_links(c, format, ls)) || (e = ensure_fp32_workspace(c))) return e;
    launch_vec_narrow(c->g, (const double2*)in, c->p32, c->s);
    launch_dslash32(c->g, ls, c->p32, c->w32, out_parity, c->tps, nullptr, c->s);
    launch_vec_widen(c->g, c->w32, (double2*)out, c->s);
    return leave(c);
}

stag_status stag_mdagm_sloppy(stag_handle c, void* out, const void* in, double mass, int format) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(out) || !aligned16(in) || out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "vector pointers NULL, misaligned or equal");
    if (!std::isfinite(mass)) return fail(c, STAG_ERR_INVALID_ARG, "mass must be finite");
    if (format != STAG_LINKS_F32_18 && format != STAG_LINKS_F16_12)
        return fail(c, STAG_ERR_INVALID_ARG, "sloppy format must be STAG_LINKS_F32_18 or STAG_LINKS_F16_12");
    if ((e = enter(c))) return e;
    LinkSet ls;
    if ((e = get_links(c, format, ls)) || (e = ensure_fp32_workspace(c))) return e;
    launch_vec_narrow(c->g, (const double2*)in, c->p32, c->s);
    launch_dslash32(c->g, ls, c->p32, c->w32, 1, c->tps, nullptr, c->s);
    launch_dslash32_axpy(c->g, ls, c->w32, c->p32, 4.0 * mass * mass, c->Ap32, c->tps, c->s);
    launch_vec_widen(c->g, c->Ap32, (double2*)out, c->s);
    return leave(c);
}

namespace {
stag_status solve_entry(stag_handle c, double mass, const stag_rational* r, double tol, int maxiter, const void* b,
                        void* const* x, void* sum, const stag_mixed_opts* mixed, stag_solve_info* info) {
    const double t0 = now_s();
    stag_status e = check_common(c, true);
    if (e) return e;
    if ((e = check_rational(c, r, mass))) return e;
    if (!(tol > 0.0) || maxiter < 1) return fail(c, STAG_ERR_INVALID_ARG, "need tol > 0 and maxiter >= 1");
    if (!aligned16(b)) return fail(c, STAG_ERR_INVALID_ARG, "source pointer NULL or misaligned");
    if (x)
        for (int k = 0; k < r->n; ++k) {
            if (!aligned16(x[k])) return fail(c, STAG_ERR_INVALID_ARG, "solution pointer NULL or misaligned");
            if (x[k] == b || x[k] == sum) return fail(c, STAG_ERR_INVALID_ARG, "outputs must not alias the source");
            for (int j = 0; j < k; ++j)
                if (x[j] == x[k]) return fail(c, STAG_ERR_INVALID_ARG, "solution pointers must be distinct");
        }
    if (sum && (!aligned16(sum) || sum == b)) return fail(c, STAG_ERR_INVALID_ARG, "sum pointer misaligned or aliases b");
    if (mixed) {
        if (mixed->sloppy != STAG_LINKS_F32_18 && mixed->sloppy != STAG_LINKS_F16_12)
            return fail(c, STAG_ERR_INVALID_ARG, "sloppy link format must be STAG_LINKS_F32_18 or STAG_LINKS_F16_12");
        if (!(mixed->tol_sloppy > 0.0) || mixed->tol_sloppy >= 1.0 || mixed->reliable_every < 1)
            return fail(c, STAG_ERR_INVALID_ARG, "need 0 < tol_sloppy < 1 and reliable_every >= 1");
    }
    if ((e = enter(c))) return e;
    if ((e = ensure_pool(c, r->n))) return e;
    std::vector<double2*> xs(r->n);
    for (int k = 0; k < r->n; ++k) xs[k] = x ? (double2*)x[k] : pool_vec(c->pool_x, c->g, k);
    SolveResult res;
    const bool want_resid = info && info->true_resid;
    double* ro = info ? info->true_resid : nullptr;
    int* ipp = info ? info->iters_per_pole : nullptr;
    if (mixed)
        e = ms_solve_mixed(c, mass, r, tol, maxiter, (const double2*)b, xs.data(), mixed, want_resid, ro, ipp, res);
    else
        e = ms_solve(c, mass, r, tol, maxiter, (const double2*)b, xs.data(), want_resid, ro, ipp, res);
    if (e) return e;
    if (sum) {
        VecPtrs X{};
        for (int k = 0; k < r->n; ++k) X.p[k] = xs[k];
        launch_rational_sum(c->g, (const double2*)b, X, c->st, (double2*)sum, c->s);
    }
    if ((e = leave(c))) return e;
    if (sum) HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    if (info) {
        info->iters = res.iters;
        info->n = r->n;
        info->seconds = now_s() - t0;
    }
    return finish_solve_status(c, res);
}
}  // namespace

stag_status stag_multishift_solve(stag_handle c, double mass, const stag_rational* r, double tol, int maxiter,
                                  const void* b, void* const* x, void* sum, stag_solve_info* info) {
    return solve_entry(c, mass, r, tol, maxiter, b, x, sum, nullptr, info);
}

stag_status stag_multishift_solve_mixed(stag_handle c, double mass, const stag_rational* r, double tol, int maxiter,
                                        const void* b, void* const* x, void* sum, const stag_mixed_opts* opts,
                                        stag_solve_info* info) {
    if (!opts) return fail(c, STAG_ERR_INVALID_ARG, "mixed-precision options are NULL");
    return solve_entry(c, mass, r, tol, maxiter, b, x, sum, opts, info);
}

// Allocates the derived link copies the FP64 operator of c needs (filled by
// get_links at the next operator call), so that operator calls themselves do
// not allocate.
stag_status alloc_link_copies(stag_ctx* c) {
    const size_t l12 = (size_t)48 * c->g.vh * sizeof(double2), l18 = (size_t)72 * c->g.vh * sizeof(double2);
    stag_status e;
    if (c->fmt64 == STAG_LINKS_F64_12 && !c->links_d12 && (e = dmalloc(c, &c->links_d12, l12))) return e;
    if (c->naik && !c->long_d18 && (e = dmalloc(c, &c->long_d18, l18))) return e;
    if (c->naik && c->fmt64 == STAG_LINKS_F64_12 && !c->long_d12 && (e = dmalloc(c, &c->long_d12, l12))) return e;
    if (c->naik && !c->naik_w3 && (e = dmalloc(c, &c->naik_w3, l18))) return e;
    return STAG_OK;
}

stag_status stag_set_link_format(stag_handle c, int format) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (format != STAG_LINKS_F64_18 && format != STAG_LINKS_F64_12)
        return fail(c, STAG_ERR_INVALID_ARG, "FP64 operator format must be STAG_LINKS_F64_18 or STAG_LINKS_F64_12");
    c->fmt64 = format;
    return alloc_link_copies(c);
}

stag_status stag_set_naik(stag_handle c, double c1, double c3) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!std::isfinite(c1) || !std::isfinite(c3))
        return fail(c, STAG_ERR_INVALID_ARG, "Naik weights must be finite");
    c->naik = !(c1 == 1.0 && c3 == 0.0);
    c->naik_c1 = c1;
    c->naik_c3 = c3;
    return alloc_link_copies(c);
}

stag_status stag_fermion_action(stag_handle c, double mass, const stag_rational* r, double tol, int maxiter,
                                const void* phi, double* S, stag_solve_info* info) {
    const double t0 = now_s();
    stag_status e = check_common(c, true);
    if (e) return e;
    if ((e = check_rational(c, r, mass))) return e;
    if (!(tol > 0.0) || maxiter < 1) return fail(c, STAG_ERR_INVALID_ARG, "need tol > 0 and maxiter >= 1");
    if (!aligned16(phi) || !S) return fail(c, STAG_ERR_INVALID_ARG, "phi NULL/misaligned or S_out NULL");
    if ((e = enter(c))) return e;
    SolveResult res;
    if ((e = fermion_action_impl(c, mass, r, tol, maxiter, (const double2*)phi, S, res))) return e;
    if ((e = leave(c))) return e;
    if (info) {
        info->iters = res.iters;
        info->n = r->n;
        info->seconds = now_s() - t0;
    }
    return finish_solve_status(c, res);
}

stag_status stag_fermion_force(stag_handle c, double mass, const stag_rational* r, double tol, int maxiter,
                               const void* phi, void* mom, double dt, stag_solve_info* info) {
    const double t0 = now_s();
    stag_status e = check_common(c, true);
    if (e) return e;
    if ((e = check_rational(c, r, mass))) return e;
    if (!(tol > 0.0) || maxiter < 1) return fail(c, STAG_ERR_INVALID_ARG, "need tol > 0 and maxiter >= 1");
    if (!aligned16(phi) || !aligned16(mom)) return fail(c, STAG_ERR_INVALID_ARG, "phi/mom NULL or misaligned");
    if (!std::isfinite(dt)) return fail(c, STAG_ERR_INVALID_ARG, "dt must be finite");
    if ((e = enter(c))) return e;
    SolveResult res;
    if ((e = fermion_force_impl(c, mass, r, tol, maxiter, (const double2*)phi, (double*)mom, dt, res))) return e;
    if ((e = leave(c))) return e;
    if (info) {
        info->iters = res.iters;
        info->n = r->n;
        info->seconds = now_s() - t0;
    }
    return finish_solve_status(c, res);
}

stag_status stag_gauge_force(stag_handle c, double beta, void* mom, double dt) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(mom) || !std::isfinite(beta) || !std::isfinite(dt))
        return fail(c, STAG_ERR_INVALID_ARG, "mom NULL/misaligned or beta/dt not finite");
    if ((e = enter(c))) return e;
    launch_gauge_force(c->g, c->links, beta, (double*)mom, dt, c->s);
    return leave(c);
}

stag_status stag_gauge_action(stag_handle c, double beta, double* S, double* plaq) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if ((e = enter(c))) return e;
    if ((e = gauge_action_impl(c, beta, S, plaq))) return e;
    return leave(c);
}

stag_status stag_polyakov_loop(stag_handle c, double* re, double* im) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if ((e = enter(c))) return e;
    const int nb = launch_polyakov(c->g, c->links, c->gpart, c->s);
    launch_finalize(c->gpart, nb, 2, c->scal, c->s);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->scal_host, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    const double ns = 3.0 * c->g.nx * c->g.ny * c->g.nz;
    if (re) *re = c->scal_host[0] / ns;
    if (im) *im = c->scal_host[1] / ns;
    return leave(c);
}

stag_status stag_chiral_condensate(stag_handle c, double mass, double tol, int maxiter, int n_noise, uint64_t seed,
                                   double* mean_out, double* err_out) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!(mass > 0.0) || !std::isfinite(mass) || !(tol > 0.0) || maxiter < 1 || n_noise < 1 || !mean_out)
        return fail(c, STAG_ERR_INVALID_ARG, "need mass > 0, tol > 0, maxiter >= 1, n_noise >= 1 and mean_out");
    const double residue = 1.0, pole = 0.0;
    const stag_rational r{1, 0.0, &residue, &pole};
    if ((e = enter(c))) return e;
    const double V = 2.0 * c->g.vh;
    double sum = 0.0, sum2 = 0.0;
    for (int k = 0; k < n_noise; ++k) {
        // noise k: Gaussian, E[eta eta^dag] = 1, from the estimator-noise
        // stream (seed, k), independent of the heat-bath sources
        launch_random_source(c->g, seed, (uint64_t)k, c->xi, c->s, kFieldNoise);
        SolveResult res;
        double S = 0.0;  // Re <eta, A^-1 eta>
        if ((e = fermion_action_impl(c, mass, &r, tol, maxiter, c->xi, &S, res))) return e;
        if (res.nonfinite || !res.converged) {
            if ((e = leave(c))) return e;
            return finish_solve_status(c, res);
        }
        const double v = 4.0 * mass * S / V;
        sum += v;
        sum2 += v * v;
    }
    if ((e = leave(c))) return e;
    const double mean = sum / n_noise;
    *mean_out = mean;
    if (err_out)
        *err_out = n_noise > 1 ? std::sqrt(std::max(0.0, (sum2 - n_noise * mean * mean) / (n_noise - 1)) / n_noise)
                               : 0.0;
    return STAG_OK;
}

stag_status stag_kinetic_energy(stag_handle c, const void* mom, double* K) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(mom) || !K) return fail(c, STAG_ERR_INVALID_ARG, "mom NULL/misaligned or K_out NULL");
    if ((e = enter(c))) return e;
    if ((e = kinetic_impl(c, (const double*)mom, K))) return e;
    return leave(c);
}

stag_status stag_link_update(stag_handle c, const void* mom, double dt) {
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!aligned16(mom) || !std::isfinite(dt)) return fail(c, STAG_ERR_INVALID_ARG, "mom NULL/misaligned or dt not finite");
    if ((e = enter(c))) return e;
    launch_link_update(c->g, c->links, (const double*)mom, dt, c->s);
    links_changed(c);
    return leave(c);
}

stag_status stag_random_momentum(stag_handle c, uint64_t seed, uint64_t traj, void* mom) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(mom)) return fail(c, STAG_ERR_INVALID_ARG, "mom NULL or misaligned");
    if ((e = enter(c))) return e;
    launch_random_momentum(c->g, seed, traj, (double*)mom, c->s);
    return leave(c);
}

stag_status stag_random_source(stag_handle c, uint64_t seed, uint64_t traj, void* xi) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (!aligned16(xi)) return fail(c, STAG_ERR_INVALID_ARG, "xi NULL or misaligned");
    if ((e = enter(c))) return e;
    launch_random_source(c->g, seed, traj, (double2*)xi, c->s);
    return leave(c);
}

stag_status stag_philox(const uint32_t ctr[4], const uint32_t key[2], size_t n, uint32_t* out, void* stream) {
    if (!ctr || !key || !out || ((uintptr_t)out % 4)) return fail(nullptr, STAG_ERR_INVALID_ARG, "bad philox arguments");
    if (n == 0) return STAG_OK;
    if (n > ((size_t)1 << 31)) return fail(nullptr, STAG_ERR_INVALID_ARG, "n too large");
    launch_philox(ctr, key, n, out, (hipStream_t)stream);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(nullptr, STAG_ERR_HIP, hipGetErrorString(err));
    return STAG_OK;
}

stag_status stag_md_trajectory(stag_handle c, const stag_hmc_params* p, stag_traj_info* info) {
    const double t0 = now_s();
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!p) return fail(c, STAG_ERR_INVALID_ARG, "params NULL");
    if (p->n_steps < 1 || !(p->tau > 0) || !std::isfinite(p->beta) || !(p->tol_md > 0) || !(p->tol_action > 0) ||
        p->maxiter < 1)
        return fail(c, STAG_ERR_INVALID_ARG, "need n_steps >= 1, tau > 0, tolerances > 0, maxiter >= 1");
    const bool ferm = !p->no_fermions;
    if (ferm) {
        if ((e = check_rational(c, &p->r_md, p->mass)) || (e = check_rational(c, &p->r_action, p->mass)) ||
            (e = check_rational(c, &p->r_heatbath, p->mass)))
            return e;
    }
    if ((p->inject_mom && !aligned16(p->inject_mom)) || (p->inject_xi && !aligned16(p->inject_xi)))
        return fail(c, STAG_ERR_INVALID_ARG, "injected fields misaligned");
    if (!(p->inject_u < 1.0)) return fail(c, STAG_ERR_INVALID_ARG, "inject_u must be < 1 (negative = draw)");
    if (p->coarse_force && (p->exact_every < 1 || p->n_steps % p->exact_every))
        return fail(c, STAG_ERR_INVALID_ARG, "coarse_force needs exact_every >= 1 and n_steps % exact_every == 0");
    if (p->record_pairs && (!p->surrogate || p->exact_every != 1))
        return fail(c, STAG_ERR_INVALID_ARG, "record_pairs needs a model and exact_every == 1");
    const bool judge = p->judge_model && p->surrogate && !p->no_fermions;
    if ((p->record_pairs || judge) && !c->mom_tmp) {
        stag_status e2 = dmalloc(c, &c->mom_tmp, (size_t)64 * c->g.vh * sizeof(double));
        if (e2) return e2;
    }
    if (judge && !c->mom_judge) {
        stag_status e2 = dmalloc(c, &c->mom_judge, (size_t)64 * c->g.vh * sizeof(double));
        if (e2) return e2;
    }
    if (p->inner_iters < 0 || (p->inner_iters > 0 && !p->surrogate))
        return fail(c, STAG_ERR_INVALID_ARG, "inner_iters must be >= 0 and needs a model");
    if (p->md_link_format != 0 && p->md_link_format != STAG_LINKS_F32_18 && p->md_link_format != STAG_LINKS_F16_12)
        return fail(c, STAG_ERR_INVALID_ARG, "md_link_format must be 0, STAG_LINKS_F32_18 or STAG_LINKS_F16_12");
    const int mdf = p->md_link_format;
    if (p->inner_iters > 0 && !c->mom_aux) {
        stag_status e2 = dmalloc(c, &c->mom_aux, (size_t)64 * c->g.vh * sizeof(double));
        if (e2) return e2;
    }
    if (ferm && (p->spectrum_lo != 0.0 || p->spectrum_hi != 0.0) &&
        !(std::isfinite(p->spectrum_lo) && std::isfinite(p->spectrum_hi) && p->spectrum_lo < p->spectrum_hi))
        return fail(c, STAG_ERR_INVALID_ARG, "spectrum interval must be finite with lo < hi (or both 0)");
    if ((e = enter(c))) return e;
    const Geom& g = c->g;
    const size_t mb = (size_t)64 * g.vh * sizeof(double);
    const size_t lb = (size_t)72 * g.vh * sizeof(double2);
    // the tables' interval against the spectrum of A on the starting links
    if (ferm && p->spectrum_hi != 0.0) {
        stag_status chk = spectrum_check_impl(c, p->mass, p->spectrum_lo, p->spectrum_hi, nullptr);
        if (chk) {
            leave(c);
            return chk;
        }
    }
    stag_traj_info I{};
    SolveResult res;
    int iters = 0, nsolve = 0;
    auto acc = [&](const SolveResult& r) {
        iters += r.iters;
        nsolve += 1;
    };
    // step 1: momenta and pseudofermion heat bath
    if (p->inject_mom)
        launch_copy(c->mom, p->inject_mom, mb, c->s);
    else
        launch_random_momentum(g, p->seed, p->traj_index, c->mom, c->s);
    if (ferm) {
        if (p->inject_xi)
            launch_copy(c->xi, p->inject_xi, half_bytes(g), c->s);
        else
            launch_random_source(g, p->seed, p->traj_index, c->xi, c->s);
        if ((e = ensure_pool(c, std::max(p->r_heatbath.n, std::max(p->r_md.n, p->r_action.n))))) return e;
        std::vector<double2*> xs(p->r_heatbath.n);
        for (int k = 0; k < p->r_heatbath.n; ++k) xs[k] = pool_vec(c->pool_x, g, k);
        if ((e = ms_solve(c, p->mass, &p->r_heatbath, p->tol_action, p->maxiter, c->xi, xs.data(), false, nullptr,
                          nullptr, res)))
            return e;
        if ((e = finish_solve_status(c, res))) return e;
        acc(res);
        VecPtrs X{};
        for (int k = 0; k < p->r_heatbath.n; ++k) X.p[k] = xs[k];
        launch_rational_sum(g, c->xi, X, c->st, c->phi, c->s);
    }
    launch_copy(c->links_backup, c->links, lb, c->s);
    // From here on the links change: every error return restores the links of
    // the trajectory's start (and detaches the model's auxiliary field), so a
    // caller that catches the error still holds a configuration of the chain.
    auto restore_after_error = [&](stag_status err) -> stag_status {
        launch_copy(c->links, c->links_backup, lb, c->s);
        links_changed(c);
        if (p->surrogate && p->inner_iters > 0) stag_surrogate_set_aux(p->surrogate, nullptr);
        leave(c);
        return err;
    };
    e = [&]() -> stag_status {
    // H at the start
    if ((e = kinetic_impl(c, c->mom, &I.K_old))) return e;
    if ((e = gauge_action_impl(c, p->beta, &I.Sg_old, nullptr))) return e;
    if (ferm) {
        if ((e = fermion_action_impl(c, p->mass, &p->r_action, p->tol_action, p->maxiter, c->phi, &I.Sf_old, res)))
            return e;
        if ((e = finish_solve_status(c, res))) return e;
        acc(res);
    }
    // step 2: leapfrog, kicks k = 0..n_steps.  With a model or the coarse
    // scheme, the exact pseudofermion force acts only on kicks
    // k % exact_every == 0 and the model (if any) on all the others.  coarse:
    // two-time-scale leapfrog, the exact kicks carry exact_every times the
    // impulse of the exact force minus the model's (the model alone acts on
    // the inner scale); without a model this is the ablation.
    const double dt = p->tau / p->n_steps;
    int kick_index = 0;
    double judge_sum = 0.0;
    int judge_n = 0;
    const int every = p->exact_every < 1 ? 1 : p->exact_every;
    const bool sched = p->surrogate != nullptr || p->coarse_force;
    // the model's auxiliary channel: the pseudofermion force of the current
    // links from the multi-shift solve of r_md stopped after inner_iters
    // iterations (a deterministic function of the links and phi), so it is
    // solved once per link field (link_version counts this trajectory's link
    // updates)
    int link_version = 0, aux_version = -1;
    auto truncated_aux = [&]() -> stag_status {
        if (aux_version == link_version) return STAG_OK;
        aux_version = link_version;
        SolveResult rt;
        stag_status e2 = fermion_force_impl(c, p->mass, &p->r_md, 0.0, p->inner_iters, c->phi, c->mom_aux, 0.0, rt);
        if (e2) return e2;
        if (rt.nonfinite) return fail(c, STAG_ERR_NONFINITE, "non-finite value in the truncated solve");
        acc(rt);
        return stag_surrogate_set_aux(p->surrogate, c->mom_aux);
    };
    auto model_force = [&](double h) -> stag_status {
        stag_status e2 = p->inner_iters > 0 ? truncated_aux() : STAG_OK;
        if (!e2) e2 = stag_surrogate_force(p->surrogate, c->mom, h);
        if (e2) return fail(c, e2, std::string("surrogate: ") + stag_surrogate_last_error(p->surrogate));
        return STAG_OK;
    };
    auto kick = [&](double h) -> stag_status {
        launch_gauge_force(g, c->links, p->beta, c->mom, h, c->s);
        const bool exact = !sched || (kick_index % every) == 0;
        ++kick_index;
        if (!ferm) return STAG_OK;
        if (!exact) return p->surrogate ? model_force(h) : STAG_OK;
        const double hf = p->coarse_force ? h * every : h;
        stag_status e2;
        // inner-scale model impulse h F_s, outer-scale correction hf (F - F_s)
        if (p->coarse_force && p->surrogate && every > 1 && (e2 = model_force(h - hf))) return e2;
        if (p->record_pairs || judge) {
            if ((e2 = fermion_force_impl(c, p->mass, &p->r_md, p->tol_md, p->maxiter, c->phi, c->mom_tmp, 0.0, res,
                                         mdf)))
                return e2;
            if ((e2 = finish_solve_status(c, res))) return e2;
            if (p->inner_iters > 0 && (e2 = truncated_aux())) return e2;
            if (p->record_pairs && stag_surrogate_pair_count(p->surrogate) < stag_surrogate_capacity(p->surrogate) &&
                (e2 = stag_surrogate_add_pair(p->surrogate, c->mom_tmp)))
                return fail(c, e2, std::string("surrogate: ") + stag_surrogate_last_error(p->surrogate));
            if (judge) {
                // the model on the same links (and auxiliary force) against the exact force
                if ((e2 = stag_surrogate_force(p->surrogate, c->mom_judge, 0.0)))
                    return fail(c, e2, std::string("surrogate: ") + stag_surrogate_last_error(p->surrogate));
                launch_diff_norm2((size_t)64 * g.vh, c->mom_judge, c->mom_tmp, c->gpart, c->scal, c->s);
                HIP_OR_FAIL(c, hipMemcpyAsync(c->scal_host, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                              c->s));
                HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
                if (c->scal_host[1] > 0) {
                    judge_sum += std::sqrt(c->scal_host[0] / c->scal_host[1]);
                    ++judge_n;
                }
            }
            launch_axpy_real((size_t)64 * g.vh, hf, c->mom_tmp, c->mom, c->s);
        } else {
            if ((e2 = fermion_force_impl(c, p->mass, &p->r_md, p->tol_md, p->maxiter, c->phi, c->mom, hf, res, mdf)))
                return e2;
            if ((e2 = finish_solve_status(c, res))) return e2;
        }
        acc(res);
        return STAG_OK;
    };
    if ((e = kick(0.5 * dt))) return e;
    for (int step = 0; step < p->n_steps; ++step) {
        launch_link_update(g, c->links, c->mom, dt, c->s);
        links_changed(c);
        ++link_version;
        if ((e = kick(step < p->n_steps - 1 ? dt : 0.5 * dt))) return e;
    }
    // step 3: Metropolis on the rational action
    if ((e = kinetic_impl(c, c->mom, &I.K_new))) return e;
    if ((e = gauge_action_impl(c, p->beta, &I.Sg_new, nullptr))) return e;
    if (ferm) {
        if ((e = fermion_action_impl(c, p->mass, &p->r_action, p->tol_action, p->maxiter, c->phi, &I.Sf_new, res)))
            return e;
        if ((e = finish_solve_status(c, res))) return e;
        acc(res);
    }
    if (p->inner_iters > 0) stag_surrogate_set_aux(p->surrogate, nullptr);
    I.dH = (I.K_new + I.Sg_new + I.Sf_new) - (I.K_old + I.Sg_old + I.Sf_old);
    I.model_force_err = judge_n > 0 ? judge_sum / judge_n : -1.0;
    I.used_model = (ferm && p->surrogate) ? 1 : 0;
    double u = p->inject_u;
    if (u < 0.0) {
        launch_uniform(p->seed, p->traj_index, c->scal, c->s);
        if ((e = reduce_to_host(c, &u))) return e;
    }
    I.accepted = (u < std::exp(-I.dH)) ? 1 : 0;
    return STAG_OK;
    }();
    if (e) return restore_after_error(e);
    if (!I.accepted) {
        launch_copy(c->links, c->links_backup, lb, c->s);
        links_changed(c);
    }
    if ((e = gauge_action_impl(c, p->beta, nullptr, &I.plaquette))) return e;
    if ((e = leave(c))) return e;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    I.cg_iters_total = iters;
    I.n_solves = nsolve;
    I.seconds = now_s() - t0;
    if (info) *info = I;
    return STAG_OK;
}

// A chain in which the exact force both judges the model and stands in for
// it: model trajectories are judged at their exact kicks, and a judged force
// error above the policy's bound, or a low acceptance over the last window of
// model trajectories, sends the chain to the exact force on every kick for
// exact_trajectories trajectories.  The decision for trajectory t uses the
// results of trajectories < t only.
stag_status stag_md_chain(stag_handle c, const stag_hmc_params* p, int n_traj, const stag_chain_policy* pol,
                          stag_traj_info* infos, int* n_done) {
    if (n_done) *n_done = 0;
    stag_status e = check_common(c, true);
    if (e) return e;
    if (!p || !pol || (!infos && n_traj > 0) || n_traj < 0)
        return fail(c, STAG_ERR_INVALID_ARG, "need params, policy, infos and n_traj >= 0");
    if (pol->window < 1 || pol->exact_trajectories < 1 || !(pol->max_model_err > 0) ||
        !(pol->min_acceptance >= 0.0 && pol->min_acceptance <= 1.0))
        return fail(c, STAG_ERR_INVALID_ARG,
                    "policy needs window >= 1, exact_trajectories >= 1, max_model_err > 0, 0 <= min_acceptance <= 1");
    stag_hmc_params q = *p;
    std::vector<int> recent;  // acceptances of the latest model trajectories
    int exact_left = 0;
    for (int t = 0; t < n_traj; ++t) {
        q.traj_index = p->traj_index + (uint64_t)t;
        const bool model = p->surrogate && exact_left == 0;
        if (p->surrogate) {  // without a model every trajectory keeps p's schedule
            q.surrogate = model ? p->surrogate : nullptr;
            q.judge_model = model ? 1 : 0;
            q.exact_every = model ? p->exact_every : 1;
            q.coarse_force = model ? p->coarse_force : 0;
            q.record_pairs = model ? p->record_pairs : 0;
            q.inner_iters = model ? p->inner_iters : 0;
        }
        if ((e = stag_md_trajectory(c, &q, &infos[t]))) return e;
        if (n_done) *n_done = t + 1;
        if (!model) {
            if (exact_left > 0) --exact_left;
            continue;
        }
        recent.push_back(infos[t].accepted);
        if ((int)recent.size() > pol->window) recent.erase(recent.begin());
        bool fall_back = infos[t].model_force_err > pol->max_model_err;
        if ((int)recent.size() == pol->window) {
            int acc = 0;
            for (int a : recent) acc += a;
            if ((double)acc < pol->min_acceptance * pol->window) fall_back = true;
        }
        if (fall_back) {
            exact_left = pol->exact_trajectories;
            recent.clear();
        }
    }
    return STAG_OK;
}

// ---- measurement support (not part of the method) --------------------------

// Record hipEvents around every Dslash and shift-update launch of subsequent
// solves (capacity: max_launches launches); 0 switches it off and clears.
stag_status stag_profile_enable(stag_handle c, int max_launches) {
    stag_status e = check_common(c, false);
    if (e) return e;
    for (auto ev : c->prof_ev) hipEventDestroy(ev);
    c->prof_ev.clear();
    c->prof_on = max_launches > 0;
    for (int i = 0; i < 3; ++i) c->prof_ms[i] = 0, c->prof_cnt[i] = 0, c->prof_samples[i].clear();
    if (!c->prof_on) return STAG_OK;
    c->prof_ev.resize((size_t)2 * max_launches);
    for (auto& ev : c->prof_ev)
        if (hipEventCreate(&ev) != hipSuccess) return fail(c, STAG_ERR_HIP, "event creation failed");
    return STAG_OK;
}

// Accumulated milliseconds and launch counts: [0] D_oe, [1] D_eo with the CG
// epilogue, [2] the fused shift update.
stag_status stag_profile_read(stag_handle c, double ms[3], long counts[3]) {
    stag_status e = check_common(c, false);
    if (e) return e;
    for (int i = 0; i < 3; ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (counts) counts[i] = c->prof_cnt[i];
    }
    return STAG_OK;
}

// The recorded launch durations of one kind, in order (microseconds).
stag_status stag_profile_samples(stag_handle c, int kind, float* us_out, int cap, int* n_out) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (kind < 0 || kind > 2 || cap < 0 || !n_out || (cap > 0 && !us_out))
        return fail(c, STAG_ERR_INVALID_ARG, "need kind in [0, 2], cap >= 0, n_out and us_out when cap > 0");
    const auto& v = c->prof_samples[kind];
    *n_out = (int)v.size();
    for (int i = 0; i < cap && i < (int)v.size(); ++i) us_out[i] = 1e3f * v[i];
    return STAG_OK;
}

// The fused FP64 multi-shift loop: 0 off, 1 on small grids (default), 2 always.
stag_status stag_set_fused_iteration(stag_handle c, int on) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (on < 0 || on > 2) return fail(c, STAG_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
    c->fused = on;
    return STAG_OK;
}

// How the FP64 operator loads its links: 0 plain loads, 1 non-temporal when
// the field exceeds the Infinity Cache (default), 2 always non-temporal.
stag_status stag_set_link_streaming(stag_handle c, int mode) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (mode < 0 || mode > 2) return fail(c, STAG_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
    c->link_nt = mode;
    return STAG_OK;
}

// Replay of captured iteration chunks on (1) or off (0).
stag_status stag_set_graphs(stag_handle c, int on) {
    stag_status e = check_common(c, false);
    if (e) return e;
    c->use_graph = on ? 1 : 0;
    return STAG_OK;
}

// Shift-update window of the multi-shift solver (1..8 iterations).
stag_status stag_set_shift_window(stag_handle c, int lag) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if (lag < 1 || lag > kLagMax) return fail(c, STAG_ERR_INVALID_ARG, "window must be 1..8");
    c->lag = lag;
    return STAG_OK;
}

// Set the Dslash work split (threads per site: 1, 2 or 4) and the number of
// iterations between convergence polls.
stag_status stag_tune(stag_handle c, int tps, int chunk) {
    stag_status e = check_common(c, false);
    if (e) return e;
    if ((tps != 1 && tps != 2 && tps != 4) || chunk < 1)
        return fail(c, STAG_ERR_INVALID_ARG, "tps must be 1, 2 or 4 and chunk >= 1");
    c->tps = tps;
    c->chunk = chunk;
    return STAG_OK;
}

}  // extern "C"
