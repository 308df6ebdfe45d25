// The library handle and the host-side helpers shared by abi.hip and solver.hip.
#pragma once

#include <string>
#include <utility>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "dslash.h"

struct stag_ctx {
    stag::Geom g{};
    int dims[4]{};
    int device = 0;
    hipStream_t user = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t chunk_ev[2]{};
    // gauge field: FP64 master copy plus copies derived on demand
    double2* links = nullptr;
    double2* links_backup = nullptr;
    double2* links_d12 = nullptr;
    float2* links_s18 = nullptr;
    void* links_h12 = nullptr;
    bool d12_ok = false, s18_ok = false, h12_ok = false;
    int fmt64 = STAG_LINKS_F64_18;  // storage used by the FP64 operator
    // Naik-improved operator: weights and long links (derived like the copies above)
    int naik = 0;
    double naik_c1 = 1.0, naik_c3 = 0.0;
    double2* long_d18 = nullptr;
    double2* long_d12 = nullptr;
    float2* long_s18 = nullptr;
    void* long_h12 = nullptr;
    bool long_ok = false, long_d12_ok = false, long_s18_ok = false, long_h12_ok = false;
    double2* naik_w3 = nullptr;  // link-shaped scratch of the three-hop force term
    double* mom = nullptr;
    double* mom_tmp = nullptr;   // force staging when a trajectory records training pairs
    double* mom_aux = nullptr;   // truncated-solve force fed to a learned model
    double* mom_judge = nullptr; // a model's force at an exact kick (judge_model)
    // FP64 Krylov workspace
    double2 *r = nullptr /* ring of kLagMax residuals */, *p = nullptr, *Ap = nullptr, *w_o = nullptr, *tmp_e = nullptr, *tmp_o = nullptr;
    double2* p2 = nullptr;   // second search direction (the fused loop double-buffers p)
    float2* p2_32 = nullptr; // the same for FP32 Krylov vectors
    double2 *xi = nullptr, *phi = nullptr;
    // FP32 Krylov workspace (precision form)
    float2 *r32 = nullptr, *p32 = nullptr, *Ap32 = nullptr, *w32 = nullptr;
    double2* pool_x = nullptr;   // n_cap even vectors: solutions
    double2* pool_p = nullptr;   // n_cap even vectors: shifted search directions (FP64 or FP32)
    double2* pool_y = nullptr;   // n_cap odd vectors: D_oe x_k for the force
    int n_cap = 0;
    stag::MsState* st = nullptr;
    stag::MsState* st_host = nullptr;  // pinned
    double* dpart = nullptr;             // CG dot partials of the D_eo kernel (3 x blocks)
    double* qpart[2] = {nullptr, nullptr};  // <r,r> partials, alternating by iteration parity
    double* gpart = nullptr;             // partials of the other reductions
    double* scal = nullptr;              // device scalars for reductions
    double* scal_host = nullptr;         // pinned
    int* done_host = nullptr;            // pinned [2]
    bool has_gauge = false;
    int tps = 4;                         // threads per site in the Dslash
    int chunk = 64;                      // iterations enqueued between convergence polls
    int lag = 8;                         // shift-update window of the multi-shift solver
    int use_graph = 1;                   // replay iteration chunks from captured hipGraphs
    int fused = 1;                       // FP64 solves fold the base update into the D_oe launch
    int link_nt = 1;                     // non-temporal FP64 link loads: 0 never, 1 by field size, 2 always
    // captured iteration chunks, keyed by every argument their launches take
    struct ChunkGraph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
        unsigned long long used = 0;
    };
    std::vector<ChunkGraph> graphs;
    unsigned long long graph_clock = 0;
    // profiling of the solver kernels (hipEvent pairs)
    int prof_on = 0;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
    double prof_ms[3] = {0, 0, 0};       // D_oe, D_eo + CG epilogue, multi-shift step
    long prof_cnt[3] = {0, 0, 0};
    std::vector<float> prof_samples[3];  // every recorded launch's milliseconds
    std::string err;
    int last_iters = 0;
    // iterations the last solve of each kind took (key: poles, tolerance,
    // mass term, window, precision, loop), the chunk scheduler's estimate
    std::unordered_map<uint64_t, int> iter_hint;
};

namespace stag {

stag_status fail(stag_ctx* c, stag_status code, const std::string& msg);

#define HIP_OR_FAIL(c, expr)                                                                           \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::stag::fail((c), STAG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
stag_status dmalloc(stag_ctx* c, T** p, size_t bytes) {
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, STAG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return STAG_OK;
}

inline size_t half_bytes(const Geom& g) { return (size_t)3 * g.vh * sizeof(double2); }
inline double2* pool_vec(double2* pool, const Geom& g, int k) { return pool + (size_t)k * 3 * g.vh; }

stag_status ensure_pool(stag_ctx* c, int n);
// device address of the allocation-free operator's scratch array on c's device
stag_status scratch_init(stag_ctx* c);
// FP32 Krylov vectors (ring of residuals, p, Ap, odd w), allocated on first use
stag_status ensure_fp32_workspace(stag_ctx* c);
// the link copies needed by the FP64 operator and (fmt32 >= 0) the FP32 one, refreshed if stale
stag_status get_links(stag_ctx* c, int fmt32, LinkSet& ls);
inline void links_changed(stag_ctx* c) {
    c->d12_ok = c->s18_ok = c->h12_ok = false;
    c->long_ok = c->long_d12_ok = c->long_s18_ok = c->long_h12_ok = false;
}

struct SolveResult {
    int iters = 0;
    bool fused = false;   // ran the fused loop
    int nonfinite = 0;
    int converged = 1;
    double bb = 0.0;
};

// FP64 multi-shift CG on A + pole_k; x[k] receive the solutions
stag_status ms_solve(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter, const double2* b,
                     double2* const* x, bool want_resid, double* resid_out, int* ipp_out, SolveResult& res);
// FP32 multi-shift (x_k in FP64) down to opts->tol_sloppy, then per-pole CG in
// FP32 with FP64 reliable updates every opts->reliable_every iterations until
// the FP64 true residual of every pole is below tol
// FP32 Krylov multi-shift (links in `sloppy` format, FP64 solutions and
// reductions) to the recursive tolerance tol, without refinement.
stag_status ms_solve_sloppy(stag_ctx* c, int sloppy, double mass, const stag_rational* r, double tol, int maxiter,
                            const double2* b, double2* const* x, SolveResult& res);
stag_status ms_solve_mixed(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter,
                           const double2* b, double2* const* x, const stag_mixed_opts* opts, bool want_resid,
                           double* resid_out, int* ipp_out, SolveResult& res);

}  // namespace stag
