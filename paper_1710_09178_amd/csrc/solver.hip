// Host drivers of the multi-shift CG (Sec. 4, eq. ratapprx) in FP64 and in
// mixed precision.  The host only enqueues kernels and polls one device flag
// per chunk of iterations; all scalars of the iteration stay on the GPU.
#include <cmath>
#include <cstddef>
#include <cstring>

#include "ctx.h"
#include "msfused.h"

namespace stag {

stag_status fail(stag_ctx* c, stag_status code, const std::string& msg);

stag_status ensure_pool(stag_ctx* c, int n) {
    if (n <= c->n_cap) return STAG_OK;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    hipFree(c->pool_x);
    hipFree(c->pool_p);
    hipFree(c->pool_y);
    c->pool_x = c->pool_p = c->pool_y = nullptr;
    c->n_cap = 0;
    const size_t hb = half_bytes(c->g);
    stag_status st;
    if ((st = dmalloc(c, &c->pool_x, hb * n)) != STAG_OK) return st;
    if ((st = dmalloc(c, &c->pool_p, hb * n)) != STAG_OK) return st;
    if ((st = dmalloc(c, &c->pool_y, hb * n)) != STAG_OK) return st;
    c->n_cap = n;
    return STAG_OK;
}

// Link fields up to this size are served largely by the 256 MB Infinity
// Cache between the Dslash launches of a solve: the 151 MB FP64 field of
// 32^3x8 stays there, and even the 302 MB of links and long links of the
// improved operator at 32^3x8 run 6% slower with non-temporal loads.  Larger
// fields are streamed from HBM every time (48^3x16, 1.02 GB: D_oe 221 -> 201 us
// with non-temporal loads).
constexpr size_t kLinkCacheBytes = (size_t)512 << 20;

stag_status get_links(stag_ctx* c, int fmt32, LinkSet& ls) {
    const Geom& g = c->g;
    const size_t l12 = (size_t)48 * g.vh;  // complex entries of a 12-real field
    std::memset(&ls, 0, sizeof(ls));
    ls.fmt64 = c->fmt64;
    ls.fmt32 = fmt32 < 0 ? STAG_LINKS_F32_18 : fmt32;
    ls.d18 = c->links;
    // FP64 operator fields (links, and long links) beyond kLinkCacheBytes are
    // streamed with non-temporal loads; STAG_LINK_NT = 0 / 1 / 2 forces never /
    // by size (default) / always
    {
        const size_t per_field = (size_t)2 * 4 * (c->fmt64 == STAG_LINKS_F64_12 ? 96 : 144) * g.vh;
        const size_t bytes = per_field * (c->naik ? 2 : 1);
        ls.nt = c->link_nt == 2 || (c->link_nt == 1 && bytes > kLinkCacheBytes);
    }
    stag_status e;
    if (c->fmt64 == STAG_LINKS_F64_12) {
        if (!c->links_d12 && (e = dmalloc(c, &c->links_d12, l12 * sizeof(double2)))) return e;
        if (!c->d12_ok) launch_links_to_d12(g, c->links, c->links_d12, c->s);
        c->d12_ok = true;
        ls.d12 = c->links_d12;
    }
    if (fmt32 == STAG_LINKS_F32_18) {
        if (!c->links_s18 && (e = dmalloc(c, &c->links_s18, (size_t)72 * g.vh * sizeof(float2)))) return e;
        if (!c->s18_ok) launch_links_to_s18(g, c->links, c->links_s18, c->s);
        c->s18_ok = true;
        ls.s18 = c->links_s18;
    } else if (fmt32 == STAG_LINKS_F16_12) {
        if (!c->links_h12 && (e = dmalloc(c, &c->links_h12, l12 * 4))) return e;
        if (!c->h12_ok) launch_links_to_h12(g, c->links, c->links_h12, c->s);
        c->h12_ok = true;
        ls.h12 = c->links_h12;
    }
    if (!c->naik) return STAG_OK;
    // improved operator: long links from the master field, then their copies
    ls.naik = 1;
    ls.c1 = c->naik_c1;
    ls.c3 = c->naik_c3;
    if (!c->long_d18 && (e = dmalloc(c, &c->long_d18, (size_t)72 * g.vh * sizeof(double2)))) return e;
    if (!c->long_ok) launch_long_links(g, c->links, c->long_d18, c->s);
    c->long_ok = true;
    ls.ld18 = c->long_d18;
    if (c->fmt64 == STAG_LINKS_F64_12) {
        if (!c->long_d12 && (e = dmalloc(c, &c->long_d12, l12 * sizeof(double2)))) return e;
        if (!c->long_d12_ok) launch_links_to_d12(g, c->long_d18, c->long_d12, c->s);
        c->long_d12_ok = true;
        ls.ld12 = c->long_d12;
    }
    if (fmt32 == STAG_LINKS_F32_18) {
        if (!c->long_s18 && (e = dmalloc(c, &c->long_s18, (size_t)72 * g.vh * sizeof(float2)))) return e;
        if (!c->long_s18_ok) launch_links_to_s18(g, c->long_d18, c->long_s18, c->s);
        c->long_s18_ok = true;
        ls.ls18 = c->long_s18;
    } else if (fmt32 == STAG_LINKS_F16_12) {
        if (!c->long_h12 && (e = dmalloc(c, &c->long_h12, l12 * 4))) return e;
        if (!c->long_h12_ok) launch_links_to_h12(g, c->long_d18, c->long_h12, c->s);
        c->long_h12_ok = true;
        ls.lh12 = c->long_h12;
    }
    return STAG_OK;
}

namespace {

using EvRec = std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>>;

// the next launch records its own start/end timestamps into an event pair
void prof_begin(stag_ctx* c, hipEvent_t* a) {
    *a = nullptr;
    if (!c->prof_on || c->prof_used + 2 > c->prof_ev.size()) return;
    *a = c->prof_ev[c->prof_used];
    next_launch_timing() = LaunchTiming{*a, c->prof_ev[c->prof_used + 1]};
}
void prof_end(stag_ctx* c, hipEvent_t a, int kind, EvRec& rec) {
    if (!a) return;
    rec.push_back({{a, c->prof_ev[c->prof_used + 1]}, kind});
    c->prof_used += 2;
}
// kernel times of iterations 0..iter (the last one only detects convergence in
// its step kernel, after full Dslash launches)
// Books the launches that did work: a solve that stops at step S runs S + 1
// iterations' Dslash launches and S steps (three-launch loop), or S fused
// D_oe launches after the eager iteration 0, S D_eo launches and S / L
// window flushes (fused loop); launches queued behind the stop are not booked.
void prof_collect(stag_ctx* c, const EvRec& rec, int iters, bool fused = false, int lag = 1) {
    long seen[3] = {0, 0, 0};
    const long lim[3] = {fused ? (long)iters : iters + 1L, fused ? (long)iters : iters + 1L,
                         fused ? (long)(iters / lag) : (long)iters};
    for (auto& q : rec) {
        const int kind = q.second;
        if (seen[kind]++ >= lim[kind]) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.first.first, q.first.second) == hipSuccess) {
            c->prof_ms[kind] += ms;
            c->prof_cnt[kind] += 1;
            c->prof_samples[kind].push_back(ms);
        }
    }
}

// Krylov workspace and operator of one precision
template <class V>
struct Krylov;

template <>
struct Krylov<double2> {
    double2 *r, *p, *Ap, *w, *p2;
    explicit Krylov(stag_ctx* c) : r(c->r), p(c->p), Ap(c->Ap), w(c->w_o), p2(c->p2) {}
    static void doe(const Geom& g, const LinkSet& ls, const double2* in, double2* out, int tps, const int* gate,
                    hipStream_t s) {
        launch_dslash(g, ls, in, out, 1, tps, gate, s);
    }
    static void deo_cg(const Geom& g, const LinkSet& ls, const double2* w, const double2* p, const double2* r,
                       double2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mt) {
        launch_dslash_cg(g, ls, w, p, r, Ap, gate, dpart, tps, s, mt);
    }
};

template <>
struct Krylov<float2> {
    float2 *r, *p, *Ap, *w, *p2;
    explicit Krylov(stag_ctx* c) : r(c->r32), p(c->p32), Ap(c->Ap32), w(c->w32), p2(c->p2_32) {}
    static void doe(const Geom& g, const LinkSet& ls, const float2* in, float2* out, int tps, const int* gate,
                    hipStream_t s) {
        launch_dslash32(g, ls, in, out, 1, tps, gate, s);
    }
    static void deo_cg(const Geom& g, const LinkSet& ls, const float2* w, const float2* p, const float2* r,
                       float2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mt) {
        launch_dslash32_cg(g, ls, w, p, r, Ap, gate, dpart, tps, s, mt);
    }
};

// Fill the pinned host copy of the state for a solve with the given poles.
void init_state(MsState* h, int n, const double* pole, const double* residue, double c0, double mass, double tol,
                int maxiter, int& base) {
    base = 0;
    for (int k = 1; k < n; ++k)
        if (pole[k] < pole[base]) base = k;
    const double s0 = pole[base];
    std::memset(h, 0, sizeof(MsState));
    h->n = n;
    h->base = base;
    h->maxiter = maxiter;
    h->lag = 1;
    h->tol2 = tol * tol;
    h->mass_term = 4.0 * mass * mass + s0;
    h->c0 = c0;
    for (int k = 0; k < n; ++k) {
        h->shift[k] = pole[k] - s0;
        h->coef[k] = residue ? residue[k] : 0.0;
        h->it[0].zeta[k] = h->it[0].zeta_old[k] = 1.0;
        h->it[0].active[k] = 1;
    }
    h->it[0].alpha_old = 1.0;
    h->it[0].beta_old = 0.0;
}

// Everything the launches of one chunk depend on; two chunks with equal keys
// enqueue identical work, so a captured graph of one can replay the other.
struct ChunkKey {
    Geom g;
    LinkSet ls;
    const void* vec[5];
    VecPtrs X, P;
    const void* st;
    const void* dpart;
    const void* qpart[2];
    double mt;
    int tps, lag, chunk, nb2, v64, n, base, fused, rows;
};

hipGraphExec_t cached_graph(stag_ctx* c, const ChunkKey& key) {
    const unsigned char* k = reinterpret_cast<const unsigned char*>(&key);
    for (auto& e : c->graphs)
        if (e.key.size() == sizeof(ChunkKey) && std::memcmp(e.key.data(), k, sizeof(ChunkKey)) == 0) {
            e.used = ++c->graph_clock;
            return e.exec;
        }
    return nullptr;
}

void store_graph(stag_ctx* c, const ChunkKey& key, hipGraphExec_t exec) {
    constexpr size_t kMaxGraphs = 8;
    if (c->graphs.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < c->graphs.size(); ++i)
            if (c->graphs[i].used < c->graphs[lru].used) lru = i;
        hipGraphExecDestroy(c->graphs[lru].exec);
        c->graphs.erase(c->graphs.begin() + lru);
    }
    stag_ctx::ChunkGraph e;
    const unsigned char* k = reinterpret_cast<const unsigned char*>(&key);
    e.key.assign(k, k + sizeof(ChunkKey));
    e.exec = exec;
    e.used = ++c->graph_clock;
    c->graphs.push_back(std::move(e));
}

// Enqueue iterations in chunks and poll the device "done" flag once per chunk,
// keeping two chunks in flight.  between_chunks(par_next) may enqueue extra
// work after every chunk (reliable updates); it receives the parity of the
// next iteration.  Without extra work or profiling, a chunk is captured once
// into a hipGraph (kernel nodes only) and replayed: the chunk length is a
// multiple of 2 and of the window, so every chunk repeats the same launches.
// Issue chunks into the two flag slots in turn and wait for them in order:
// up to two in flight (one with two_in_flight false, and one once
// past_estimate() holds), until a chunk's flag says the solve has stopped.
template <class Issue, class Past>
stag_status drive_chunks(stag_ctx* c, Issue& issue_chunk, bool two_in_flight, Past past_estimate) {
    int q[2], nq = 0, next_slot = 0;
    auto issue = [&]() {
        issue_chunk(next_slot);
        q[nq++] = next_slot;
        next_slot ^= 1;
    };
    issue();
    if (two_in_flight && !past_estimate()) issue();
    for (;;) {
        const int s0 = q[0];
        q[0] = q[1];
        --nq;
        HIP_OR_FAIL(c, hipEventSynchronize(c->chunk_ev[s0]));
        if (c->done_host[s0]) break;
        const int cap = (!two_in_flight || past_estimate()) ? 1 : 2;
        while (nq < cap) issue();
    }
    HIP_OR_FAIL(c, hipGetLastError());
    return STAG_OK;
}

//
// pred > 0: the iterations the solve is expected to take (the last solve of
// the same kind).  Chunks that would run past it shrink to `small`
// iterations, and once pred iterations are issued the next chunk waits for
// the flag: a converged solve then leaves fewer early-exit launches queued.
// Results do not depend on the chunking.
inline int small_chunk(int chunk, int L) {
    const int s = L % 2 == 0 ? L : 2 * L;
    return s < chunk ? s : chunk;
}

template <class V, class Between>
stag_status run_iterations(stag_ctx* c, const LinkSet& ls, const Krylov<V>& K, VecPtrs X, VecPtrs P, int chunk,
                           EvRec& rec, Between between_chunks, bool two_in_flight = true,
                           bool extra_work = false, int pred = 0) {
    const Geom& g = c->g;
    const double mt = c->st_host->mass_term;
    const int L = c->st_host->lag;
    const int nb2 = dslash_grid(g, c->tps);
    const int small = small_chunk(chunk, L);
    int it_issued = 0;
    auto enqueue_chunk = [&](int len) {
        for (int it = 0; it < len; ++it, ++it_issued) {
            const int par = it_issued & 1;
            hipEvent_t a;
            prof_begin(c, &a);
            const int* gate = &c->st->done[par];
            Krylov<V>::doe(g, ls, K.p, K.w, c->tps, gate, c->s);
            prof_end(c, a, 0, rec);
            prof_begin(c, &a);
            // residual r_j sits in slot j % L of the ring starting at K.r
            const V* rj = K.r + (size_t)(it_issued % L) * 3 * g.vh;
            Krylov<V>::deo_cg(g, ls, K.w, K.p, rj, K.Ap, gate, c->dpart, c->tps, c->s, mt);
            prof_end(c, a, 1, rec);
            prof_begin(c, &a);
            // the last iteration of a window flushes the shifted updates; on
            // lattices whose step grid is small the flush is latency-bound,
            // and up to one block row per group of shifts spreads it (up to
            // ~512 blocks in all).  Not with a window of 1, where r_{j+1}
            // overwrites r_j in place (only the thread that read r_j may
            // write it).
            const int nsh = c->st_host->n - 1;
            const int rows = (L > 1 && it_issued % L == L - 1 && nsh > 0)
                                 ? std::max(1, std::min((nsh + kFlushGroup - 1) / kFlushGroup, 512 / ms_update_grid(g)))
                                 : 1;
            // every launch that runs has device iteration it_issued (a
            // stopped solve's later launches exit at the flag), and a
            // replayed chunk starts at a multiple of its length, hence of L
            const MsStepConst sc{c->st_host->n, c->st_host->base, L, it_issued % L};
            launch_ms_step<V>(g, K.r, K.Ap, K.p, X, P, c->st, c->dpart, nb2, c->qpart[par], c->qpart[par ^ 1], par,
                              rows, sc, c->s);
            prof_end(c, a, 2, rec);
        }
    };
    const bool graphs = c->use_graph && !c->prof_on && !extra_work && chunk % 2 == 0 && chunk % L == 0;
    // one captured graph per chunk length; every replay starts at a multiple
    // of 2 and of L, like the capture
    auto graph_for = [&](int len, hipGraphExec_t& exec) -> stag_status {
        exec = nullptr;
        if (!graphs) return STAG_OK;
        ChunkKey key;
        std::memset(&key, 0, sizeof(key));
        key.g = g;
        key.ls = ls;
        key.vec[0] = K.r;
        key.vec[1] = K.p;
        key.vec[2] = K.Ap;
        key.vec[3] = K.w;
        key.X = X;
        key.P = P;
        key.st = c->st;
        key.dpart = c->dpart;
        key.qpart[0] = c->qpart[0];
        key.qpart[1] = c->qpart[1];
        key.mt = mt;
        key.tps = c->tps;
        key.lag = L;
        key.n = c->st_host->n;
        key.base = c->st_host->base;
        key.chunk = len;
        key.nb2 = nb2;
        key.v64 = sizeof(V) == sizeof(double2);
        exec = cached_graph(c, key);
        if (!exec) {
            hipGraph_t graph = nullptr;
            const int saved = it_issued;
            it_issued = 0;
            HIP_OR_FAIL(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
            enqueue_chunk(len);
            HIP_OR_FAIL(c, hipStreamEndCapture(c->s, &graph));
            it_issued = saved;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(c, STAG_ERR_HIP, "hipGraphInstantiate failed");
            store_graph(c, key, exec);
        }
        return STAG_OK;
    };
    hipGraphExec_t exec = nullptr, exec_small = nullptr;
    stag_status e;
    if ((e = graph_for(chunk, exec))) return e;
    if (pred > 0 && small < chunk && (e = graph_for(small, exec_small))) return e;
    auto issue_chunk = [&](int slot) {
        // the launch of device iteration pred (the expected stop) sets the flag
        const int len = (pred > 0 && it_issued + chunk > pred + 1) ? small : chunk;
        hipGraphExec_t ex = len == chunk ? exec : exec_small;
        if (ex) {
            hipGraphLaunch(ex, c->s);
            it_issued += len;
        } else {
            enqueue_chunk(len);
        }
        between_chunks(it_issued & 1);
        // the flag the next iteration would read
        hipMemcpyAsync(&c->done_host[slot], &c->st->done[it_issued & 1], sizeof(int), hipMemcpyDeviceToHost, c->s);
        hipEventRecord(c->chunk_ev[slot], c->s);
    };
    return drive_chunks(c, issue_chunk, two_in_flight, [&]() { return pred > 0 && it_issued > pred; });
}

// The fused loop (FP64 or FP32 Krylov vectors, window L >= 2): iteration j is
//   D_oe launch j: step j-1's scalars, r_j, p_j, x_base, w = D_oe p_j
//   D_eo launch j: Ap_j and the three dots
//   flush after iterations j with j % L == 0 (shifted systems, steps j-L..j-1)
// with p double-buffered by parity (K.p, K.p2).  Iteration 0 is enqueued
// eagerly, then chunks of `chunk` iterations from j = 1 (a multiple of 2 and
// of L, so a captured chunk replays for every later one), and once the solve
// has stopped a final flush for the steps of its last, partial window.
constexpr int kFusedMaxBlocks = 512;

template <class V>
stag_status run_fused(stag_ctx* c, const LinkSet& ls, const Krylov<V>& K, VecPtrs X, VecPtrs P, int chunk,
                      EvRec& rec, int pred = 0) {
    const Geom& g = c->g;
    const double mt = c->st_host->mass_term;
    const int n = c->st_host->n, base = c->st_host->base;
    const int L = c->st_host->lag;
    const int nb2 = dslash_fused_grid(g);   // both Dslash launches: 4 threads per site
    const size_t n3 = (size_t)3 * g.vh;
    V* pbuf[2] = {K.p, K.p2};
    const int nsh = n - 1;
    const int rows = nsh > 0 ? std::max(1, std::min((nsh + kFlushGroup - 1) / kFlushGroup, 512 / ms_update_grid(g)))
                             : 1;
    auto iter_args = [&](int j) {
        const int par = j & 1;
        FusedIterT<V> f{};
        f.ring = K.r;
        f.Ap = K.Ap;
        f.p_prev = pbuf[par ^ 1];
        f.p_new = pbuf[par];
        f.x_base = X.at<double2>(base);
        f.st = c->st;
        f.dpart = c->dpart;
        f.qin = c->qpart[par ^ 1];
        f.qout = c->qpart[par];
        f.nb2 = nb2;
        f.par = par;
        f.n = n;
        f.base = base;
        f.lag = L;
        f.slot_prev = (j + L - 1) % L;
        f.slot_new = j % L;
        return f;
    };
    // iteration 0: w = D_oe p_0 (p_0 = r_0 = b, both written by the init
    // kernel), |r_0|^2 partials in the D_oe grid's layout into qpart[0]
    {
        FusedIterT<V> f0 = iter_args(0);
        f0.p_prev = pbuf[0];
        f0.slot_prev = 0;
        launch_dslash_fused(g, ls, f0, K.w, true, c->s);
        launch_dslash_cg_fused(g, ls, K.w, pbuf[0], K.r, K.Ap, &c->st->done[1], c->dpart, c->s, mt);
    }
    int it_issued = 1;
    const int small = small_chunk(chunk, L);
    auto enqueue_chunk = [&](int len) {
        for (int it = 0; it < len; ++it, ++it_issued) {
            const int j = it_issued, par = j & 1;
            const FusedIterT<V> f = iter_args(j);
            hipEvent_t a;
            prof_begin(c, &a);
            launch_dslash_fused(g, ls, f, K.w, false, c->s);
            prof_end(c, a, 0, rec);
            prof_begin(c, &a);
            launch_dslash_cg_fused(g, ls, K.w, pbuf[par], K.r + (size_t)(j % L) * n3, K.Ap,
                                   &c->st->done[par ^ 1], c->dpart, c->s, mt);
            prof_end(c, a, 1, rec);
            if (j % L == 0 && nsh > 0) {
                prof_begin(c, &a);
                launch_ms_flush(g, (const V*)K.r, X, P, c->st, &c->st->done[par ^ 1], n, base, L, false, rows, c->s);
                prof_end(c, a, 2, rec);
            }
        }
    };
    const bool graphs = c->use_graph && !c->prof_on && chunk % 2 == 0 && chunk % L == 0;
    // one captured graph per chunk length, captured from j = 1; every replay
    // starts at j = 1 mod L and odd, like the capture
    auto graph_for = [&](int len, hipGraphExec_t& exec) -> stag_status {
        exec = nullptr;
        if (!graphs) return STAG_OK;
        ChunkKey key;
        std::memset(&key, 0, sizeof(key));
        key.g = g;
        key.ls = ls;
        key.vec[0] = K.r;
        key.vec[1] = pbuf[0];
        key.vec[2] = K.Ap;
        key.vec[3] = K.w;
        key.vec[4] = pbuf[1];
        key.X = X;
        key.P = P;
        key.st = c->st;
        key.dpart = c->dpart;
        key.qpart[0] = c->qpart[0];
        key.qpart[1] = c->qpart[1];
        key.mt = mt;
        key.tps = 4;
        key.lag = L;
        key.n = n;
        key.base = base;
        key.chunk = len;
        key.nb2 = nb2;
        key.v64 = sizeof(V) == sizeof(double2);
        key.fused = 1;
        key.rows = rows;
        exec = cached_graph(c, key);
        if (!exec) {
            hipGraph_t graph = nullptr;
            const int saved = it_issued;
            it_issued = 1;
            HIP_OR_FAIL(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
            enqueue_chunk(len);
            HIP_OR_FAIL(c, hipStreamEndCapture(c->s, &graph));
            it_issued = saved;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(c, STAG_ERR_HIP, "hipGraphInstantiate failed");
            store_graph(c, key, exec);
        }
        return STAG_OK;
    };
    hipGraphExec_t exec = nullptr, exec_small = nullptr;
    stag_status e;
    if ((e = graph_for(chunk, exec))) return e;
    if (pred > 0 && small < chunk && (e = graph_for(small, exec_small))) return e;
    auto issue_chunk = [&](int slot) {
        // the D_oe launch of iteration pred + 1 evaluates step pred (the
        // expected stop) and sets the flag
        const int len = (pred > 0 && it_issued + chunk > pred + 2) ? small : chunk;
        hipGraphExec_t ex = len == chunk ? exec : exec_small;
        if (ex) {
            hipGraphLaunch(ex, c->s);
            it_issued += len;
        } else {
            enqueue_chunk(len);
        }
        // the flag the next D_oe launch would read
        hipMemcpyAsync(&c->done_host[slot], &c->st->done[it_issued & 1], sizeof(int), hipMemcpyDeviceToHost, c->s);
        hipEventRecord(c->chunk_ev[slot], c->s);
    };
    if ((e = drive_chunks(c, issue_chunk, true, [&]() { return pred > 0 && it_issued > pred + 1; }))) return e;
    if (nsh > 0) launch_ms_flush(g, (const V*)K.r, X, P, c->st, nullptr, n, base, L, true, rows, c->s);
    HIP_OR_FAIL(c, hipGetLastError());
    return STAG_OK;
}

// Multi-shift CG in Krylov precision V (x_k always FP64).
// A key for solves that take about the same number of iterations: the poles,
// residues, tolerance and mass term of the state, its window, and the loop,
// precision and operator (FNV-1a over their bytes).
uint64_t solve_kind(const MsState* h, bool fused, bool fp64, int naik, int fmt64, int fmt32) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) x = (x ^ b[i]) * 1099511628211ull;
    };
    mix(&h->n, sizeof h->n);
    mix(h->shift, sizeof(double) * h->n);
    mix(&h->tol2, sizeof h->tol2);
    mix(&h->mass_term, sizeof h->mass_term);
    mix(&h->lag, sizeof h->lag);
    const int tag[5] = {fused, fp64, naik, fmt64, fmt32};
    mix(tag, sizeof tag);
    return x;
}

template <class V>
stag_status ms_solve_t(stag_ctx* c, const LinkSet& ls, double mass, const stag_rational* r, double tol, int maxiter,
                       const double2* b, double2* const* x, int* ipp_out, SolveResult& res, EvRec& rec) {
    const Geom& g = c->g;
    const int n = r->n;
    stag_status e = ensure_pool(c, n);
    if (e != STAG_OK) return e;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));  // st_host is reused
    MsState* h = c->st_host;
    int base;
    init_state(h, n, r->pole, r->residue, r->c0, mass, tol, maxiter, base);
    // the fused loop (window >= 2; it keeps r_{j-1} and r_j in the ring
    // at once): by default on grids of at most kFusedMaxBlocks Dslash blocks,
    // where an iteration is latency-bound; with on = 2 at every size
    const bool fused = c->lag >= 2 &&
                       (c->fused == 2 || (c->fused == 1 && dslash_fused_grid(g) <= kFusedMaxBlocks));
    h->lag = fused ? c->lag : (n > 1 ? c->lag : 1);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->st, h, sizeof(MsState), hipMemcpyHostToDevice, c->s));
    Krylov<V> K(c);
    VecPtrs X{}, P{};
    for (int k = 0; k < n; ++k) {
        X.p[k] = x[k];
        P.p[k] = (V*)c->pool_p + (size_t)k * 3 * g.vh;
    }
    launch_ms_init<V>(g, b, K.r, K.p, X, P, c->st, c->qpart[0], c->s);
    res.fused = fused;
    // the iterations of the last solve of this kind, as the chunk scheduler's
    // estimate (a hint only: the solve runs until its own stop)
    const uint64_t kind = solve_kind(h, fused, sizeof(V) == sizeof(double2), c->naik, ls.fmt64, ls.fmt32);
    const auto hint = c->iter_hint.find(kind);
    const int pred = hint == c->iter_hint.end() ? 0 : hint->second;
    if (fused)
        e = run_fused<V>(c, ls, K, X, P, c->chunk, rec, pred);
    else
        e = run_iterations<V>(c, ls, K, X, P, c->chunk, rec, [](int) {}, true, false, pred);
    if (e) return e;
    HIP_OR_FAIL(c, hipMemcpyAsync(h, c->st, sizeof(MsState), hipMemcpyDeviceToHost, c->s));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    const MsIter& f = h->fin;
    res.iters = f.iter;
    c->iter_hint[kind] = f.iter;
    res.nonfinite = f.nonfinite;
    res.bb = f.bb;
    res.converged = 1;
    for (int k = 0; k < n; ++k) {
        if (f.active[k]) res.converged = 0;
        if (ipp_out) ipp_out[k] = f.iters_per_pole[k];
    }
    return STAG_OK;
}

// FP64 true residuals |b - (A + pole_k) x_k|^2 into st->true_res2[k]
void true_residuals(stag_ctx* c, const LinkSet& ls, double mass, const stag_rational* r, const double2* b,
                    double2* const* x) {
    const Geom& g = c->g;
    const int nbr = dslash_grid(g, c->tps);
    for (int k = 0; k < r->n; ++k) {
        launch_dslash(g, ls, x[k], c->tmp_o, 1, c->tps, nullptr, c->s);
        launch_dslash_resid(g, ls, c->tmp_o, x[k], b, 4.0 * mass * mass + r->pole[k], c->gpart, c->tps, c->s);
        double* slot = (double*)((char*)c->st + offsetof(MsState, true_res2)) + k;
        launch_finalize(c->gpart, nbr, 1, slot, c->s);
    }
}

// CG in FP32 on (A + pole) for one pole, started from the FP64 residual of x
// (FP64), whose residual is recomputed in FP64 every `every` iterations and
// copied into the FP32 Krylov residual (reliable update; the search direction
// is kept).  Returns the iterations run.
stag_status refine_pole(stag_ctx* c, const LinkSet& ls, double mass, double pole, double tol, int maxiter,
                        const double2* b, double2* x, double bb, int every, int& iters_out, bool& converged) {
    const Geom& g = c->g;
    const int nbr = dslash_grid(g, c->tps);
    const int nq = ms_update_grid(g);
    const double coef = 4.0 * mass * mass + pole;
    Krylov<float2> K(c);
    iters_out = 0;
    converged = false;
    EvRec rec;
    // reliable update: r32 = b - (A + pole) x computed in FP64, |r|^2 partials for the next step
    auto reliable = [&](double* qdst) {
        launch_dslash(g, ls, x, c->tmp_o, 1, c->tps, nullptr, c->s);
        launch_dslash_resid(g, ls, c->tmp_o, x, b, coef, c->gpart, c->tps, c->s, K.r);
        launch_finalize_pad(c->gpart, nbr, qdst, nq, c->s);
    };
    for (int restart = 0; restart < 8 && iters_out < maxiter; ++restart) {
        HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
        MsState* h = c->st_host;
        int base;
        const double one = 1.0;
        init_state(h, 1, &pole, &one, 0.0, mass, tol, maxiter - iters_out, base);
        h->bb_given = 1;
        h->it[0].bb = bb;
        HIP_OR_FAIL(c, hipMemcpyAsync(c->st, h, sizeof(MsState), hipMemcpyHostToDevice, c->s));
        reliable(c->gpart + 4 * (size_t)nbr);  // r32 from the FP64 residual (partials unused)
        launch_cg_restart(g, K.r, K.p, c->qpart[0], c->s);
        VecPtrs X{}, P{};
        X.p[0] = x;
        stag_status e = run_iterations<float2>(
            c, ls, K, X, P, every, rec, [&](int par_next) { reliable(c->qpart[par_next]); }, false, true);
        if (e) return e;
        HIP_OR_FAIL(c, hipMemcpyAsync(h, c->st, sizeof(MsState), hipMemcpyDeviceToHost, c->s));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
        iters_out += h->fin.iter;
        if (h->fin.nonfinite) return fail(c, STAG_ERR_NONFINITE, "non-finite value in the refinement CG");
        // the step kernel may have stopped on a recursive residual: check in FP64
        launch_dslash(g, ls, x, c->tmp_o, 1, c->tps, nullptr, c->s);
        launch_dslash_resid(g, ls, c->tmp_o, x, b, coef, c->gpart, c->tps, c->s);
        launch_finalize(c->gpart, nbr, 1, c->scal, c->s);
        HIP_OR_FAIL(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
        if (c->scal_host[0] <= tol * tol * bb) {
            converged = true;
            break;
        }
        if (h->fin.iter == 0) break;  // no progress possible
    }
    return STAG_OK;
}

}  // namespace

stag_status ms_solve(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter, const double2* b,
                     double2* const* x, bool want_resid, double* resid_out, int* ipp_out, SolveResult& res) {
    LinkSet ls;
    stag_status e = get_links(c, -1, ls);
    if (e) return e;
    EvRec rec;
    c->prof_used = 0;
    if ((e = ms_solve_t<double2>(c, ls, mass, r, tol, maxiter, b, x, ipp_out, res, rec))) return e;
    prof_collect(c, rec, res.iters, res.fused, c->st_host->lag);
    if (want_resid) {
        true_residuals(c, ls, mass, r, b, x);
        HIP_OR_FAIL(c, hipMemcpyAsync(c->st_host, c->st, sizeof(MsState), hipMemcpyDeviceToHost, c->s));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    }
    for (int k = 0; k < r->n && resid_out; ++k)
        resid_out[k] = (want_resid && res.bb > 0) ? std::sqrt(c->st_host->true_res2[k] / res.bb) : -1.0;
    c->last_iters = res.iters;
    return STAG_OK;
}

stag_status ensure_fp32_workspace(stag_ctx* c) {
    const Geom& g = c->g;
    stag_status e;
    if (!c->r32) {
        if ((e = dmalloc(c, &c->r32, kLagMax * half_bytes(g) / 2)) || (e = dmalloc(c, &c->p32, half_bytes(g) / 2)) ||
            (e = dmalloc(c, &c->p2_32, half_bytes(g) / 2)) || (e = dmalloc(c, &c->Ap32, half_bytes(g) / 2)) ||
            (e = dmalloc(c, &c->w32, half_bytes(g) / 2)))
            return e;
    }
    return STAG_OK;
}

stag_status ms_solve_sloppy(stag_ctx* c, int sloppy, double mass, const stag_rational* r, double tol, int maxiter,
                            const double2* b, double2* const* x, SolveResult& res) {
    LinkSet ls;
    stag_status e = get_links(c, sloppy, ls);
    if (e || (e = ensure_fp32_workspace(c))) return e;
    EvRec rec;
    c->prof_used = 0;
    int ipp[kMaxPoles];
    if ((e = ms_solve_t<float2>(c, ls, mass, r, tol, maxiter, b, x, ipp, res, rec))) return e;
    c->last_iters = res.iters;
    return STAG_OK;
}

stag_status ms_solve_mixed(stag_ctx* c, double mass, const stag_rational* r, double tol, int maxiter,
                           const double2* b, double2* const* x, const stag_mixed_opts* opts, bool want_resid,
                           double* resid_out, int* ipp_out, SolveResult& res) {
    LinkSet ls;
    stag_status e = get_links(c, opts->sloppy, ls);
    if (e || (e = ensure_fp32_workspace(c))) return e;
    EvRec rec;
    c->prof_used = 0;
    int ipp[kMaxPoles];
    SolveResult r1;
    // phase 1: FP32 multi-shift to tol_sloppy
    if ((e = ms_solve_t<float2>(c, ls, mass, r, std::max(opts->tol_sloppy, tol), maxiter, b, x, ipp, r1, rec)))
        return e;
    prof_collect(c, rec, r1.iters, r1.fused, c->st_host->lag);
    if (r1.nonfinite) {
        res = r1;
        return STAG_OK;
    }
    res.bb = r1.bb;
    res.iters = r1.iters;
    res.converged = 1;
    if (r1.bb > 0) {
        // phase 2: every pole to the FP64 true residual tol, smallest pole
        // first.  The refinement's sloppy operator uses FP32-18 links even when
        // the multi-shift phase ran on FP16-12 links: CG on an operator with
        // relative error delta only contracts the true residual when
        // delta |(A + pole)^-1| |A| < 1, which FP16 links (delta ~ 5e-4)
        // violate for light poles.
        LinkSet lr;
        if ((e = get_links(c, STAG_LINKS_F32_18, lr))) return e;
        for (int k = 0; k < r->n; ++k) {
            int it = 0;
            bool conv = false;
            if ((e = refine_pole(c, lr, mass, r->pole[k], tol, std::max(1, maxiter - res.iters), b, x[k], r1.bb,
                                 std::max(1, opts->reliable_every), it, conv)))
                return e;
            ipp[k] += it;
            res.iters += it;
            if (!conv) res.converged = 0;
        }
    }
    for (int k = 0; k < r->n && ipp_out; ++k) ipp_out[k] = ipp[k];
    if (want_resid) {
        true_residuals(c, ls, mass, r, b, x);
        HIP_OR_FAIL(c, hipMemcpyAsync(c->st_host, c->st, sizeof(MsState), hipMemcpyDeviceToHost, c->s));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->s));
    }
    for (int k = 0; k < r->n && resid_out; ++k)
        resid_out[k] = (want_resid && res.bb > 0) ? std::sqrt(c->st_host->true_res2[k] / res.bb) : -1.0;
    c->last_iters = res.iters;
    return STAG_OK;
}

}  // namespace stag
