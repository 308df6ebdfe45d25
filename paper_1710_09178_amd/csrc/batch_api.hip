// extern "C" entry points of the batched form: many lattices of uneven volume
// with several right-hand sides, all poles of a rational function, solved by
// one multi-shift CG whose every kernel launch covers the whole batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <unordered_map>
#include <vector>

#include "batch.h"

using namespace stag;

namespace stag {
void launch_gauge_to_internal(const Geom& g, const double2* canon, double2* links, hipStream_t s);
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
}

struct stag_batch {
    int n_inst = 0, nrhs = 0, n_sys = 0;
    int device = 0;
    hipStream_t user = nullptr, s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, chunk_ev[2]{};
    std::vector<BInst> inst_h;
    std::vector<BTile> tiles_h;
    BInst* inst_d = nullptr;
    BTile* tiles_d = nullptr;
    int tps = 2;
    int link_nt = -1;            // links loaded non-temporally: -1 by field size, 0 no, 1 yes (tuned)
    int link12 = 0;              // operators read 12 reals per link (rows 0-1, row 2 rebuilt)
    int lag = 8;                 // shift-update window (divides the 16-iteration chunk)
    int tiles_cap = 0;
    size_t total_vh = 0;
    double2* links64 = nullptr;
    float2* links32 = nullptr;
    bool l32_ok = false;
    std::vector<int> gauge_set;
    // batched vectors (3 * nrhs * total_vh complex entries)
    // r: ring of kLagMax residuals (batched vectors); the others one batched vector each
    double2 *b = nullptr, *r = nullptr, *p = nullptr, *Ap = nullptr, *w = nullptr, *e = nullptr, *res = nullptr;
    double2* pool_x = nullptr;   // n_cap solution vectors (FP64)
    double2* pool_p = nullptr;   // n_cap shifted search directions (FP64 or FP32)
    int n_cap = 0;
    BState st{};
    double* dpart = nullptr;
    double* qpart[2] = {nullptr, nullptr};
    double* gpart = nullptr;
    double* sums = nullptr;
    int* done_host = nullptr;    // pinned [2 * n_inst]
    double* sums_host = nullptr;  // pinned [n_sys]
    // captured iteration chunks, keyed by every launch argument (LRU)
    struct BGraph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
        unsigned long long used = 0;
    };
    std::vector<BGraph> graphs;
    unsigned long long graph_clock = 0;
    // iterations the last solve of each kind took (the chunk scheduler's estimate)
    std::unordered_map<uint64_t, int> iter_hint;
    std::string err;
};

namespace {

thread_local std::string g_batch_err;

stag_status bfail(stag_batch* c, stag_status code, const std::string& m) {
    if (c)
        c->err = m;
    else
        g_batch_err = m;
    return code;
}

#define BHIP(c, expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return bfail((c), STAG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
stag_status balloc(stag_batch* c, T** p, size_t bytes) {
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return bfail(c, STAG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return STAG_OK;
}

size_t bvec_len(const stag_batch* c) { return (size_t)3 * c->nrhs * c->total_vh; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// (re)build the tile table for the current work split
stag_status build_tiles(stag_batch* c) {
    const int sb = kBlock / c->tps;
    c->tiles_h.clear();
    for (int i = 0; i < c->n_inst; ++i) {
        BInst& I = c->inst_h[i];
        I.tile0 = (int)c->tiles_h.size();
        I.ntiles = (I.g.vh + sb - 1) / sb;
        for (int t = 0; t < I.ntiles; ++t) c->tiles_h.push_back(BTile{i, t * sb});
    }
    const int nt = (int)c->tiles_h.size();
    if (nt > c->tiles_cap) {
        hipFree(c->tiles_d);
        hipFree(c->dpart);
        hipFree(c->qpart[0]);
        hipFree(c->qpart[1]);
        hipFree(c->gpart);
        c->tiles_d = nullptr;
        stag_status e;
        if ((e = balloc(c, &c->tiles_d, nt * sizeof(BTile))) || (e = balloc(c, &c->dpart, (size_t)nt * 12 * 8)) ||
            (e = balloc(c, &c->qpart[0], (size_t)nt * kMaxRhs * 8)) ||
            (e = balloc(c, &c->qpart[1], (size_t)nt * kMaxRhs * 8)) || (e = balloc(c, &c->gpart, (size_t)nt * kMaxRhs * 8)))
            return e;
        c->tiles_cap = nt;
    }
    BHIP(c, hipMemcpyAsync(c->tiles_d, c->tiles_h.data(), nt * sizeof(BTile), hipMemcpyHostToDevice, c->s));
    BHIP(c, hipMemcpyAsync(c->inst_d, c->inst_h.data(), c->n_inst * sizeof(BInst), hipMemcpyHostToDevice, c->s));
    BHIP(c, hipStreamSynchronize(c->s));
    return STAG_OK;
}

BatchDev bdev(const stag_batch* c) {
    // the links of all lattices are streamed from HBM by every operator
    // application once they exceed what the Infinity Cache keeps (FP64:
    // 1.2 GB for the 64-lattice batch; the single-lattice operator's rule)
    const size_t link_bytes = (size_t)(c->link12 ? 48 : 72) * c->total_vh * 16;
    const int nt = c->link_nt >= 0 ? c->link_nt : (link_bytes > ((size_t)512 << 20) ? 1 : 0);
    return BatchDev{c->inst_d, c->tiles_d, (int)c->tiles_h.size(), kBlock / c->tps, c->nrhs, nt, c->link12};
}

stag_status ensure_bpool(stag_batch* c, int n) {
    if (n <= c->n_cap) return STAG_OK;
    BHIP(c, hipStreamSynchronize(c->s));
    hipFree(c->pool_x);
    hipFree(c->pool_p);
    c->pool_x = c->pool_p = nullptr;
    c->n_cap = 0;
    stag_status e;
    if ((e = balloc(c, &c->pool_x, bvec_len(c) * n * sizeof(double2))) ||
        (e = balloc(c, &c->pool_p, bvec_len(c) * n * sizeof(double2))))
        return e;
    c->n_cap = n;
    return STAG_OK;
}

stag_status ensure_links32(stag_batch* c) {
    if (c->l32_ok) return STAG_OK;
    stag_status e;
    if (!c->links32 && (e = balloc(c, &c->links32, (size_t)72 * c->total_vh * sizeof(float2)))) return e;
    launch_blinks_to_f32(c->links64, c->links32, (size_t)72 * c->total_vh, c->s);
    c->l32_ok = true;
    return STAG_OK;
}

// Multi-shift CG over the whole batch in Krylov precision V.  x: n batched
// FP64 solution vectors; source b (FP64 internal).  When refine_pole >= 0 the
// solve is a single-pole CG whose convergence is measured against |b_orig|^2
// kept from the previous solve (st.bb_given).
template <class V>
stag_status bsolve_t(stag_batch* c, int n, const double* poles, const double* masses, double tol, int maxiter,
                     const double2* b, double2** x, bool from_fin, bool use_graph, int& iters_out, bool& conv_out) {
    const BatchDev bd = bdev(c);
    const void* links = std::is_same<V, double2>::value ? (const void*)c->links64 : (const void*)c->links32;
    int base = 0;
    for (int k = 1; k < n; ++k)
        if (poles[k] < poles[base]) base = k;
    BState& st = c->st;
    st.n = n;
    st.base = base;
    st.maxiter = maxiter;
    st.tol2 = tol * tol;
    st.bb_given = from_fin ? 1 : 0;
    st.lag = n > 1 ? c->lag : 1;
    st.ring_stride = bvec_len(c);
    for (int k = 0; k < n; ++k) st.shift[k] = poles[k] - poles[base];
    std::vector<double> s0(c->n_inst);
    for (int i = 0; i < c->n_inst; ++i) s0[i] = 4.0 * masses[i] * masses[i] + poles[base];
    BHIP(c, hipMemcpyAsync(st.sigma0_term, s0.data(), c->n_inst * sizeof(double), hipMemcpyHostToDevice, c->s));
    launch_bstate_init(st, from_fin ? 1 : 0, c->s);
    V* r = (V*)c->r;
    V* p = (V*)c->p;
    V* Ap = (V*)c->Ap;
    V* w = (V*)c->w;
    VecPtrs X{}, P{};
    for (int k = 0; k < n; ++k) {
        X.p[k] = x[k];
        P.p[k] = (V*)c->pool_p + (size_t)k * bvec_len(c);
    }
    launch_bms_init<V>(bd, b, r, p, X, P, st, c->qpart[0], c->s);
    // a multiple of 2 and of the window: the parity and ring patterns repeat
    // across chunks; near the expected stop (the last solve of this kind)
    // chunks shrink to 8 iterations and one is in flight past it
    const int chunk = 16, small = 8;
    uint64_t kind = 1469598103934665603ull;
    auto mix = [&](const void* q, size_t nb) {
        const unsigned char* u = static_cast<const unsigned char*>(q);
        for (size_t i = 0; i < nb; ++i) kind = (kind ^ u[i]) * 1099511628211ull;
    };
    mix(&n, sizeof n);
    mix(st.shift, sizeof(double) * n);
    mix(&st.tol2, sizeof st.tol2);
    mix(&st.lag, sizeof st.lag);
    mix(&st.bb_given, sizeof st.bb_given);
    mix(s0.data(), sizeof(double) * s0.size());
    const int fp64 = std::is_same<V, double2>::value;
    mix(&fp64, sizeof fp64);
    mix(&bd.link12, sizeof bd.link12);
    const auto hint = c->iter_hint.find(kind);
    const int pred = hint == c->iter_hint.end() ? 0 : hint->second;
    auto enqueue_chunk = [&](int len) {
        for (int it = 0; it < len; ++it) {
            const int par = it & 1;
            const V* rj = r + (size_t)(it % st.lag) * st.ring_stride;
            const int* gate = st.inst_done + par * c->n_inst;
            launch_bdslash<V>(bd, c->tps, links, p, w, 1, gate, c->s);
            launch_bdslash_cg<V>(bd, c->tps, links, w, p, rj, Ap, st, gate, c->dpart, c->s);
            launch_bms_scalars(bd, st, c->dpart, c->qpart[par], par, c->s);
            launch_bms_step<V>(bd, r, Ap, p, X, P, st, c->dpart, c->qpart[par], c->qpart[par ^ 1], par, c->s);
        }
    };
    // one captured graph per chunk length and launch arguments, kept across solves
    auto graph_for = [&](int len, hipGraphExec_t& exec) -> stag_status {
        exec = nullptr;
        if (!use_graph) return STAG_OK;
        std::vector<unsigned char> key;
        auto put = [&](const void* q, size_t nb) {
            const unsigned char* u = static_cast<const unsigned char*>(q);
            key.insert(key.end(), u, u + nb);
        };
        // (field by field where a struct may hold uninitialised padding;
        // c->st is value-initialised with the handle)
        put(&bd.inst, sizeof bd.inst);
        put(&bd.tiles, sizeof bd.tiles);
        const int bdi[5] = {bd.ntiles, bd.tile_sites, bd.nrhs, bd.link_nt, bd.link12};
        put(bdi, sizeof bdi);
        put(&st, sizeof st);
        put(&links, sizeof links);
        put(&r, sizeof r);
        put(&p, sizeof p);
        put(&Ap, sizeof Ap);
        put(&w, sizeof w);
        put(&X, sizeof X);
        put(&P, sizeof P);
        put(&c->dpart, sizeof c->dpart);
        put(c->qpart, sizeof c->qpart);
        put(&c->tps, sizeof c->tps);
        put(&len, sizeof len);
        put(&fp64, sizeof fp64);
        for (auto& e : c->graphs)
            if (e.key == key) {
                e.used = ++c->graph_clock;
                exec = e.exec;
                return STAG_OK;
            }
        hipGraph_t graph = nullptr;
        BHIP(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
        enqueue_chunk(len);
        BHIP(c, hipStreamEndCapture(c->s, &graph));
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ie != hipSuccess) return bfail(c, STAG_ERR_HIP, "hipGraphInstantiate failed");
        constexpr size_t kMaxGraphs = 6;
        if (c->graphs.size() >= kMaxGraphs) {
            size_t lru = 0;
            for (size_t i = 1; i < c->graphs.size(); ++i)
                if (c->graphs[i].used < c->graphs[lru].used) lru = i;
            hipGraphExecDestroy(c->graphs[lru].exec);
            c->graphs.erase(c->graphs.begin() + lru);
        }
        stag_batch::BGraph g;
        g.key = std::move(key);
        g.exec = exec;
        g.used = ++c->graph_clock;
        c->graphs.push_back(std::move(g));
        return STAG_OK;
    };
    hipGraphExec_t exec = nullptr, exec_small = nullptr;
    stag_status ge;
    if ((ge = graph_for(chunk, exec))) return ge;
    if (pred > 0 && (ge = graph_for(small, exec_small))) return ge;
    int* dh = c->done_host;
    int it_issued = 0;
    auto issue = [&](int slot) {
        // the scalar launch of device iteration pred (the expected stop) sets the flags
        const int len = (pred > 0 && it_issued + chunk > pred + 1) ? small : chunk;
        hipGraphExec_t ex = len == chunk ? exec : exec_small;
        if (ex)
            hipGraphLaunch(ex, c->s);
        else
            enqueue_chunk(len);
        it_issued += len;
        // chunks are even: the next iteration reads the parity-0 flags
        hipMemcpyAsync(dh + slot * c->n_inst, st.inst_done, c->n_inst * sizeof(int), hipMemcpyDeviceToHost, c->s);
        hipEventRecord(c->chunk_ev[slot], c->s);
    };
    auto past_estimate = [&]() { return pred > 0 && it_issued > pred; };
    int q[2], nq = 0, next_slot = 0;
    auto push = [&]() {
        issue(next_slot);
        q[nq++] = next_slot;
        next_slot ^= 1;
    };
    push();
    if (!past_estimate()) push();
    stag_status status = STAG_OK;
    for (;;) {
        const int cur = q[0];
        q[0] = q[1];
        --nq;
        if (hipEventSynchronize(c->chunk_ev[cur]) != hipSuccess) {
            status = bfail(c, STAG_ERR_HIP, "batched solve failed on the device");
            break;
        }
        bool all = true;
        for (int i = 0; i < c->n_inst; ++i) all &= dh[cur * c->n_inst + i] != 0;
        if (all) break;
        const int cap = past_estimate() ? 1 : 2;
        while (nq < cap) push();
    }
    hipStreamSynchronize(c->s);
    if (status) return status;
    BHIP(c, hipGetLastError());
    std::vector<MsIter> fin(c->n_sys);
    BHIP(c, hipMemcpy(fin.data(), st.fin, c->n_sys * sizeof(MsIter), hipMemcpyDeviceToHost));
    iters_out = 0;
    conv_out = true;
    for (auto& f : fin) {
        iters_out = std::max(iters_out, f.iter);
        if (f.nonfinite) return bfail(c, STAG_ERR_NONFINITE, "non-finite value in the batched solve");
        for (int k = 0; k < n; ++k) conv_out &= !f.active[k];
    }
    c->iter_hint[kind] = iters_out;
    return STAG_OK;
}

// per-system FP64 |b - (A_i + pole) x|^2 into sums_host; residual vector in c->res when want_vec
stag_status bresid(stag_batch* c, double pole, const double2* x, const double2* b, bool want_vec) {
    const BatchDev bd = bdev(c);
    launch_bdslash<double2>(bd, c->tps, c->links64, x, c->w, 1, nullptr, c->s);
    launch_bdslash_resid(bd, c->tps, c->links64, c->w, x, b, pole, c->gpart, want_vec ? c->res : nullptr, c->s);
    launch_bsys_sum(bd, c->n_inst, c->gpart, c->sums, c->s);
    BHIP(c, hipMemcpyAsync(c->sums_host, c->sums, c->n_sys * sizeof(double), hipMemcpyDeviceToHost, c->s));
    BHIP(c, hipStreamSynchronize(c->s));
    return STAG_OK;
}

}  // namespace

extern "C" {

stag_status stag_batch_create(stag_batch_handle* out, int n_inst, const int* dims, int nrhs, void* stream) {
    if (!out || !dims || n_inst < 1 || nrhs < 1 || nrhs > STAG_BATCH_MAX_RHS)
        return bfail(nullptr, STAG_ERR_INVALID_ARG, "need out, dims, n_inst >= 1 and 1 <= nrhs <= 4");
    *out = nullptr;
    long long total = 0;
    for (int i = 0; i < n_inst; ++i) {
        long long V = 1;
        for (int d = 0; d < 4; ++d) {
            const int n = dims[4 * i + d];
            if (n < 2 || n % 2) return bfail(nullptr, STAG_ERR_INVALID_ARG, "every lattice extent must be even and >= 2");
            V *= n;
        }
        total += V / 2;
    }
    if (total * 3 * nrhs * 16 >= (1LL << 40)) return bfail(nullptr, STAG_ERR_INVALID_ARG, "batch too large");
    stag_batch* c = new stag_batch();
    c->n_inst = n_inst;
    c->nrhs = nrhs;
    c->n_sys = n_inst * nrhs;
    c->user = (hipStream_t)stream;
    c->total_vh = (size_t)total;
    c->gauge_set.assign(n_inst, 0);
    int off = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int* d = dims + 4 * i;
        BInst I{};
        I.g = Geom{d[0], d[1], d[2], d[3], d[0] / 2, d[0] * d[1] * d[2] * d[3] / 2};
        I.off = off;
        off += I.g.vh;
        c->inst_h.push_back(I);
    }
    auto bail = [&](stag_status s) {
        g_batch_err = c->err;
        stag_batch_destroy(c);
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return bfail(nullptr, STAG_ERR_HIP, "no HIP device available");
    }
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->chunk_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->chunk_ev[1], hipEventDisableTiming) != hipSuccess) {
        c->err = "stream/event creation failed";
        return bail(STAG_ERR_HIP);
    }
    const size_t vb = bvec_len(c) * sizeof(double2);
    stag_status s;
    BState& st = c->st;
    st.n_inst = n_inst;
    st.nrhs = nrhs;
    if ((s = balloc(c, &c->inst_d, n_inst * sizeof(BInst))) ||
        (s = balloc(c, &c->links64, (size_t)72 * c->total_vh * sizeof(double2))) || (s = balloc(c, &c->b, vb)) ||
        (s = balloc(c, &c->r, kLagMax * vb)) || (s = balloc(c, &c->p, vb)) || (s = balloc(c, &c->Ap, vb)) ||
        (s = balloc(c, &c->w, vb)) || (s = balloc(c, &c->e, vb)) || (s = balloc(c, &c->res, vb)) ||
        (s = balloc(c, &st.it[0], c->n_sys * sizeof(MsIter))) || (s = balloc(c, &st.it[1], c->n_sys * sizeof(MsIter))) ||
        (s = balloc(c, &st.fin, c->n_sys * sizeof(MsIter))) || (s = balloc(c, &st.sys_done, 2 * c->n_sys * sizeof(int))) ||
        (s = balloc(c, &st.inst_done, 2 * n_inst * sizeof(int))) ||
        (s = balloc(c, &st.t_done, (c->n_sys + 1) * sizeof(unsigned long long))) ||
        (s = balloc(c, &st.sigma0_term, n_inst * sizeof(double))) ||
        (s = balloc(c, &st.hist, (size_t)c->n_sys * kLagMax * sizeof(MsHist))) ||
        (s = balloc(c, &st.scal, c->n_sys * sizeof(BScal))) ||
        (s = balloc(c, &st.w_tab, (size_t)c->n_sys * 3 * kWinTab * sizeof(double))) ||
        (s = balloc(c, &st.w_act, (size_t)c->n_sys * kWinTab * sizeof(int))) || (s = balloc(c, &c->sums, c->n_sys * sizeof(double))))
        return bail(s);
    if (hipHostMalloc((void**)&c->done_host, 2 * n_inst * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->sums_host, c->n_sys * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        c->err = "pinned host allocation failed";
        return bail(STAG_ERR_OOM);
    }
    if ((s = build_tiles(c))) return bail(s);
    launch_fill_zero(c->p, vb, c->s);
    launch_fill_zero(c->links64, (size_t)72 * c->total_vh * sizeof(double2), c->s);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        c->err = "initialisation kernels failed";
        return bail(STAG_ERR_HIP);
    }
    *out = c;
    return STAG_OK;
}

stag_status stag_batch_destroy(stag_batch_handle c) {
    if (!c) return STAG_OK;
    if (c->s) hipStreamSynchronize(c->s);
    void* bufs[] = {c->inst_d, c->tiles_d, c->links64, c->links32, c->b, c->r, c->p, c->Ap, c->w, c->e, c->res,
                    c->pool_x, c->pool_p, c->st.it[0], c->st.it[1], c->st.fin, c->st.sys_done, c->st.inst_done,
                    c->st.t_done, c->st.sigma0_term, c->st.hist, c->st.scal, c->st.w_tab, c->st.w_act, c->dpart, c->qpart[0], c->qpart[1], c->gpart, c->sums};
    for (void* b : bufs)
        if (b) hipFree(b);
    for (auto& g : c->graphs)
        if (g.exec) hipGraphExecDestroy(g.exec);
    if (c->done_host) hipHostFree(c->done_host);
    if (c->sums_host) hipHostFree(c->sums_host);
    hipEvent_t evs[] = {c->ev_in, c->ev_out, c->chunk_ev[0], c->chunk_ev[1]};
    for (auto ev : evs)
        if (ev) hipEventDestroy(ev);
    if (c->s) hipStreamDestroy(c->s);
    delete c;
    return STAG_OK;
}

const char* stag_batch_last_error(stag_batch_handle c) { return c ? c->err.c_str() : g_batch_err.c_str(); }

size_t stag_batch_vec_bytes(stag_batch_handle c) { return c ? bvec_len(c) * sizeof(double2) : 0; }

stag_status stag_batch_set_gauge(stag_batch_handle c, int inst, const double* U) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (inst < 0 || inst >= c->n_inst) return bfail(c, STAG_ERR_INVALID_ARG, "instance index out of range");
    if (!U || (uintptr_t)U % 16) return bfail(c, STAG_ERR_INVALID_ARG, "gauge pointer NULL or misaligned");
    BHIP(c, hipSetDevice(c->device));
    BHIP(c, hipEventRecord(c->ev_in, c->user));
    BHIP(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    const BInst& I = c->inst_h[inst];
    launch_gauge_to_internal(I.g, (const double2*)U, c->links64 + blink_base(I), c->s);
    c->l32_ok = false;
    c->gauge_set[inst] = 1;
    BHIP(c, hipGetLastError());
    BHIP(c, hipEventRecord(c->ev_out, c->s));
    BHIP(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    return STAG_OK;
}

stag_status stag_batch_solve(stag_batch_handle c, const double* masses, const stag_rational* r, const void* b_canon,
                             void* x_canon, const stag_batch_opts* o, stag_batch_info* info) {
    const double t0 = now_s();
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (!masses || !r || !o || !b_canon || !x_canon || (uintptr_t)b_canon % 16 || (uintptr_t)x_canon % 16)
        return bfail(c, STAG_ERR_INVALID_ARG, "NULL or misaligned argument");
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->gauge_set[i]) return bfail(c, STAG_ERR_NO_GAUGE, "gauge field of lattice " + std::to_string(i) + " not set");
    if (r->n < 1 || r->n > STAG_MAX_POLES || !r->pole) return bfail(c, STAG_ERR_INVALID_ARG, "bad pole list");
    double pmin = 1e300;
    for (int k = 0; k < r->n; ++k) {
        if (!std::isfinite(r->pole[k]) || r->pole[k] < 0) return bfail(c, STAG_ERR_INVALID_ARG, "poles must be >= 0");
        pmin = std::min(pmin, r->pole[k]);
    }
    for (int i = 0; i < c->n_inst; ++i)
        if (!std::isfinite(masses[i]) || !(4 * masses[i] * masses[i] + pmin > 0))
            return bfail(c, STAG_ERR_INVALID_ARG, "4 m^2 + smallest pole must be > 0 for every lattice");
    if (!(o->tol > 0) || o->maxiter < 1 || (o->precision != 0 && o->precision != 1) ||
        (o->precision == 1 && !(o->tol_sloppy > 0 && o->tol_sloppy < 1)))
        return bfail(c, STAG_ERR_INVALID_ARG, "bad options (tol, tol_sloppy, maxiter, precision)");
    if ((const char*)x_canon < (const char*)b_canon + stag_batch_vec_bytes(c) &&
        (const char*)b_canon < (const char*)x_canon + r->n * stag_batch_vec_bytes(c))
        return bfail(c, STAG_ERR_INVALID_ARG, "x must not overlap b");
    BHIP(c, hipSetDevice(c->device));
    BHIP(c, hipEventRecord(c->ev_in, c->user));
    BHIP(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    stag_status e;
    if ((e = ensure_bpool(c, r->n))) return e;
    // the residual kernels take 4 m_i^2 from the instance table
    bool mass_changed = false;
    for (int i = 0; i < c->n_inst; ++i) {
        const double m2 = 4.0 * masses[i] * masses[i];
        mass_changed |= c->inst_h[i].four_m2 != m2;
        c->inst_h[i].four_m2 = m2;
    }
    if (mass_changed) {
        BHIP(c, hipMemcpyAsync(c->inst_d, c->inst_h.data(), c->n_inst * sizeof(BInst), hipMemcpyHostToDevice, c->s));
        BHIP(c, hipStreamSynchronize(c->s));
    }
    const BatchDev bd = bdev(c);
    const size_t L = bvec_len(c);
    launch_bvec_import(bd, (const double2*)b_canon, c->b, c->s);
    std::vector<double2*> xs(r->n);
    for (int k = 0; k < r->n; ++k) xs[k] = c->pool_x + (size_t)k * L;
    int iters = 0, refine = 0;
    bool conv = true;
    launch_b_timestamp(c->st.t_done + c->n_sys, c->s);
    if (o->precision == 0) {
        if ((e = bsolve_t<double2>(c, r->n, r->pole, masses, o->tol, o->maxiter, c->b, xs.data(), false, o->use_graph,
                                   iters, conv)))
            return e;
    } else {
        // the sloppy stage only provides starting guesses: the refinement
        // below decides convergence
        bool sloppy_conv = true;
        if ((e = ensure_links32(c))) return e;
        if ((e = bsolve_t<float2>(c, r->n, r->pole, masses, std::max(o->tol, o->tol_sloppy), o->maxiter, c->b,
                                  xs.data(), false, o->use_graph, iters, sloppy_conv)))
            return e;
    }
    std::vector<unsigned long long> td(c->n_sys + 1);
    BHIP(c, hipMemcpy(td.data(), c->st.t_done, (c->n_sys + 1) * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    std::vector<MsIter> fin(c->n_sys);
    BHIP(c, hipMemcpy(fin.data(), c->st.fin, c->n_sys * sizeof(MsIter), hipMemcpyDeviceToHost));
    if (o->precision == 1) {
        // FP64 CG refinement of every pole, all systems of the batch at once;
        // convergence is measured against |b| of each system.  The correction
        // solve aims at tol/2 so that the rounding of x + e leaves the true
        // residual below tol.
        for (int k = 0; k < r->n; ++k) {
            if ((e = bresid(c, r->pole[k], xs[k], c->b, true))) return e;
            bool all_ok = true;
            for (int s = 0; s < c->n_sys; ++s) all_ok &= c->sums_host[s] <= o->tol * o->tol * fin[s].bb;
            if (all_ok) continue;
            BHIP(c, hipMemcpy(c->st.fin, fin.data(), c->n_sys * sizeof(MsIter), hipMemcpyHostToDevice));
            double2* ev[1] = {c->e};
            int it = 0;
            bool rconv = true;
            if ((e = bsolve_t<double2>(c, 1, &r->pole[k], masses, 0.5 * o->tol, o->maxiter, c->res, ev, true,
                                       o->use_graph, it, rconv)))
                return e;
            conv &= rconv;
            launch_baxpy(L, xs[k], c->e, c->s);
            refine += it;
        }
    }
    for (int k = 0; k < r->n; ++k) launch_bvec_export(bd, xs[k], (double2*)x_canon + (size_t)k * L, c->s);
    if (info && info->true_resid) {
        for (int k = 0; k < r->n; ++k) {
            if ((e = bresid(c, r->pole[k], xs[k], c->b, false))) return e;
            for (int s = 0; s < c->n_sys; ++s)
                info->true_resid[(size_t)s * r->n + k] = fin[s].bb > 0 ? std::sqrt(c->sums_host[s] / fin[s].bb) : 0.0;
        }
    }
    BHIP(c, hipGetLastError());
    BHIP(c, hipEventRecord(c->ev_out, c->s));
    BHIP(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    BHIP(c, hipStreamSynchronize(c->s));
    if (info) {
        int rate_khz = 0;
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device);
        const double hz = rate_khz > 0 ? rate_khz * 1e3 : 1e8;
        info->iters = iters;
        info->refine_iters = refine;
        info->seconds = now_s() - t0;
        for (int s = 0; s < c->n_sys; ++s) {
            if (info->latency) info->latency[s] = (double)(td[s] - td[c->n_sys]) / hz;
            if (info->iters_sys) info->iters_sys[s] = fin[s].iter;
            if (info->iters_per_pole)
                for (int k = 0; k < r->n; ++k) info->iters_per_pole[(size_t)s * r->n + k] = fin[s].iters_per_pole[k];
        }
    }
    if (!conv) return bfail(c, STAG_ERR_NOT_CONVERGED, "some system reached maxiter before the tolerance");
    return STAG_OK;
}

stag_status stag_batch_set_shift_window(stag_batch_handle c, int lag) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (lag != 1 && lag != 2 && lag != 4 && lag != 8) return bfail(c, STAG_ERR_INVALID_ARG, "window must be 1, 2, 4 or 8");
    c->lag = lag;
    return STAG_OK;
}

stag_status stag_batch_set_link_format(stag_batch_handle c, int format) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (format != STAG_LINKS_F64_18 && format != STAG_LINKS_F64_12)
        return bfail(c, STAG_ERR_INVALID_ARG, "format must be STAG_LINKS_F64_18 or STAG_LINKS_F64_12");
    c->link12 = format == STAG_LINKS_F64_12;
    return STAG_OK;
}

stag_status stag_batch_set_tps(stag_batch_handle c, int tps) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (tps != 1 && tps != 2 && tps != 4 && tps != 8)
        return bfail(c, STAG_ERR_INVALID_ARG, "threads per site must be 1, 2, 4 or 8");
    c->tps = tps;
    return build_tiles(c);
}

// The autotuner's key for a batch: device, precision, right-hand sides and the
// multiset of lattice shapes.
std::string tune_key(stag_batch* c, int precision) {
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
    for (auto& ch : dev)
        if (ch == ' ' || ch == '|') ch = '_';
    std::map<std::string, int> shapes;
    for (const BInst& I : c->inst_h) {
        char b[64];
        snprintf(b, sizeof b, "%dx%dx%dx%d", I.g.nx, I.g.ny, I.g.nz, I.g.nt);
        shapes[b] += 1;
    }
    std::ostringstream k;
    k << dev << "|p" << precision << "|r" << c->nrhs << "|l" << (c->link12 ? 12 : 18) << "|";
    for (auto& kv : shapes) k << kv.first << "*" << kv.second << ",";
    return k.str();
}

extern "C" stag_status stag_batch_autotune(stag_batch_handle c, int precision, const char* cache_path, double* us_out,
                                           int* choice_out) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (precision != 0 && precision != 1) return bfail(c, STAG_ERR_INVALID_ARG, "precision must be 0 or 1");
    // candidates: threads per site (tile of 256/tps sites) x link loads
    const int cand_tps[7] = {1, 2, 4, 1, 2, 4, 8};
    const int cand_nt[7] = {0, 0, 0, 1, 1, 1, 0};
    if (us_out)
        for (int q = 0; q < 7; ++q) us_out[q] = -1.0;
    const std::string key = tune_key(c, precision);
    stag_status e;
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int tps = 0, nt = -1;
            if ((ls >> k >> tps >> nt) && k == key && (tps == 1 || tps == 2 || tps == 4 || tps == 8) &&
                (nt == 0 || nt == 1)) {
                c->tps = tps;
                c->link_nt = nt;
                if (choice_out) choice_out[0] = tps, choice_out[1] = nt, choice_out[2] = 1;
                return build_tiles(c);
            }
        }
    }
    if (precision == 1 && (e = ensure_links32(c))) return e;
    hipEvent_t a, b;
    BHIP(c, hipEventCreate(&a));
    BHIP(c, hipEventCreate(&b));
    double best = 1e300;
    int best_q = 0;
    for (int q = 0; q < 7; ++q) {
        c->tps = cand_tps[q];
        c->link_nt = cand_nt[q];
        if ((e = build_tiles(c))) return e;
        const BatchDev bd = bdev(c);
        auto run = [&]() {
            if (precision == 0)
                launch_bdslash<double2>(bd, c->tps, c->links64, c->p, c->w, 1, nullptr, c->s);
            else
                launch_bdslash<float2>(bd, c->tps, c->links32, (const float2*)c->p, (float2*)c->w, 1, nullptr, c->s);
        };
        run();
        hipEventRecord(a, c->s);
        const int reps = 10;
        for (int i = 0; i < reps; ++i) run();
        hipEventRecord(b, c->s);
        BHIP(c, hipEventSynchronize(b));
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        const double us = 1e3 * ms / reps;
        if (us_out) us_out[q] = us;
        if (us < best) {
            best = us;
            best_q = q;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    c->tps = cand_tps[best_q];
    c->link_nt = cand_nt[best_q];
    if (choice_out) choice_out[0] = c->tps, choice_out[1] = c->link_nt, choice_out[2] = 0;
    if (cache_path && *cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << key << " " << c->tps << " " << c->link_nt << " " << best << "\n";
    }
    return build_tiles(c);
}

stag_status stag_batch_tune(stag_batch_handle c, int precision, double* us_out) {
    if (!c) return bfail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (precision != 0 && precision != 1) return bfail(c, STAG_ERR_INVALID_ARG, "precision must be 0 or 1");
    stag_status e;
    if (precision == 1 && (e = ensure_links32(c))) return e;
    hipEvent_t a, b;
    BHIP(c, hipEventCreate(&a));
    BHIP(c, hipEventCreate(&b));
    double best = 1e300;
    int best_tps = c->tps;
    const int cand[4] = {1, 2, 4, 8};
    for (int q = 0; q < 4; ++q) {
        c->tps = cand[q];
        if ((e = build_tiles(c))) return e;
        const BatchDev bd = bdev(c);
        auto run = [&]() {
            if (precision == 0)
                launch_bdslash<double2>(bd, c->tps, c->links64, c->p, c->w, 1, nullptr, c->s);
            else
                launch_bdslash<float2>(bd, c->tps, c->links32, (const float2*)c->p, (float2*)c->w, 1, nullptr, c->s);
        };
        run();
        hipEventRecord(a, c->s);
        const int reps = 10;
        for (int i = 0; i < reps; ++i) run();
        hipEventRecord(b, c->s);
        BHIP(c, hipEventSynchronize(b));
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        const double us = 1e3 * ms / reps;
        if (us_out) us_out[q] = us;
        if (us < best) {
            best = us;
            best_tps = cand[q];
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    c->tps = best_tps;
    return build_tiles(c);
}

}  // extern "C"
