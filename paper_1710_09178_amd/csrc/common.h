// Internal declarations shared by the HIP sources of libstag (gfx950 only).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/stag.h"

namespace stag {

// ---------------------------------------------------------------------------
// Lattice geometry.  Internal site index: (parity, cb) with cb = l >> 1, which
// is the rank of the site among the sites of its parity in lexicographic
// order because Nx is even.
struct Geom {
    int nx, ny, nz, nt;
    int nxh;   // nx / 2
    int vh;    // sites per parity
};

__device__ __forceinline__ void cb_coords(const Geom& g, int par, int cb, int& x, int& y, int& z, int& t) {
    int xh = cb % g.nxh;
    int r = cb / g.nxh;
    y = r % g.ny;
    r /= g.ny;
    z = r % g.nz;
    t = r / g.nz;
    x = 2 * xh + ((par + y + z + t) & 1);
}

__device__ __forceinline__ int cb_index(const Geom& g, int x, int y, int z, int t) {
    return (x >> 1) + g.nxh * (y + g.ny * (z + g.nz * t));
}

// ---------------------------------------------------------------------------
// Internal layouts (device):
//   half vector  double2 v[3][Vh]                        colour plane major
//   links        double2 U[2 parities][4 mu][9 entries][Vh], entry = 3*row+col
//   momentum     double  P[2 parities][4 mu][8][Vh]
__host__ __device__ __forceinline__ size_t link_off(const Geom& g, int par, int mu, int e) {
    return ((size_t)((par * 4 + mu) * 9 + e)) * g.vh;
}
// compressed links keep rows 0 and 1: [2][4][6][Vh]
__host__ __device__ __forceinline__ size_t link12_off(const Geom& g, int par, int mu, int e) {
    return ((size_t)((par * 4 + mu) * 6 + e)) * g.vh;
}
__host__ __device__ __forceinline__ size_t mom_off(const Geom& g, int par, int mu, int a) {
    return ((size_t)((par * 4 + mu) * 8 + a)) * g.vh;
}

// ---------------------------------------------------------------------------
// Complex and SU(3) helpers on double2.
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// float2 versions for the single-precision operator
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// conversions between the vector precisions
template <class V>
__device__ __forceinline__ V from_d2(double2 a);
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }

struct M3 {
    double2 e[9];
};

__device__ __forceinline__ M3 m3_mul(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double2 s = cmul(a.e[3 * i], b.e[k]);
            s = cadd(s, cmul(a.e[3 * i + 1], b.e[3 + k]));
            s = cadd(s, cmul(a.e[3 * i + 2], b.e[6 + k]));
            c.e[3 * i + k] = s;
        }
    return c;
}
__device__ __forceinline__ M3 m3_dag(const M3& a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) c.e[3 * i + k] = cconj(a.e[3 * k + i]);
    return c;
}
__device__ __forceinline__ M3 m3_add(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 9; ++i) c.e[i] = cadd(a.e[i], b.e[i]);
    return c;
}

// Im tr(T_a M), a = 0..7, T_a = lambda_a / 2 (Gell-Mann), written out.
__device__ __forceinline__ void im_tr_ta(const M3& m, double f[8]) {
    const double h = 0.5;
    // tr(lambda_1 M) = M10 + M01, etc.; Im of (1/2) tr(lambda_a M)
    f[0] = h * (m.e[3].y + m.e[1].y);
    f[1] = h * (m.e[1].x - m.e[3].x);   // Im(-i M10 + i M01) = -Re M10 + Re M01
    f[2] = h * (m.e[0].y - m.e[4].y);
    f[3] = h * (m.e[6].y + m.e[2].y);
    f[4] = h * (m.e[2].x - m.e[6].x);
    f[5] = h * (m.e[7].y + m.e[5].y);
    f[6] = h * (m.e[5].x - m.e[7].x);
    f[7] = h * (m.e[0].y + m.e[4].y - 2.0 * m.e[8].y) * 0.57735026918962576451;  // 1/sqrt(3)
}

// ---------------------------------------------------------------------------
// Wave/block reductions in FP64 with a fixed order (deterministic results).
constexpr int kBlock = 256;

template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
}

// Sums v over the block; thread 0 receives the totals.  Needs kBlock threads.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds /* >= 4*K */) {
    wave_sum<K>(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = lds[k] + lds[K + k] + lds[2 * K + k] + lds[3 * K + k];
    }
    __syncthreads();
}

// Block partial sums: thread 0 stores the block's K totals at
// out[k*gridDim.x + blockIdx.x].  Consumers add the partials in block order
// after the kernel boundary (no inter-block synchronisation inside a kernel).
template <int K>
__device__ __forceinline__ void block_partial(double (&v)[K], double* out) {
    __shared__ double lds[4 * K];
    block_sum<K>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) out[(size_t)k * gridDim.x + blockIdx.x] = v[k];
}

// Fixed-order sum of nb partials (one per block of the producer) by one block;
// thread 0 receives the result.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, double* lds4) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += part[b];
    block_sum<1>(v, lds4);
    return v[0];
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so each XCD works
// on one contiguous range of tiles (neighbouring sites share its L2).  The map
// is a permutation of [0, nb) for any nb.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int nx = 8;
    const int q = nb / nx, r = nb % nx;
    const int xcd = b % nx, k = b / nx;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Tiles of SB consecutive half-lattice sites for a kernel whose neighbour
// reads reach +-1 in every direction.  When tiles tile the (z, t) planes
// evenly (W tiles per plane, or one tile per SB/plane planes) and the number
// of tile rows along z is a multiple of 8, XCD k gets the z-slab k of 8 over
// all t, so only the two z faces of each slab are read from another XCD's part
// of the lattice (t-slices, the contiguous ranges, would put both t faces of
// every slice there).  Otherwise the contiguous-range map above.  A
// permutation of [0, nb).
__device__ __forceinline__ int xcd_tile_slab(int b, int nb, const Geom& g, int SB) {
    const int plane = g.nx * g.ny / 2;  // half-lattice sites of one (z, t) plane
    int NZ = 0, W = 0;                  // tile rows along z, tiles per row
    if (plane % SB == 0) {
        NZ = g.nz;
        W = plane / SB;
    } else if (SB % plane == 0 && g.nz % (SB / plane) == 0) {
        NZ = g.nz / (SB / plane);
        W = 1;
    }
    if (NZ > 0 && NZ % 8 == 0 && nb % 8 == 0 && (long long)nb * SB == g.vh) {
        const int nz8 = NZ / 8;
        const int xcd = b % 8, j = b / 8;
        const int w = j % W, rest = j / W;
        const int zl = rest % nz8, t = rest / nz8;
        return (t * NZ + xcd * nz8 + zl) * W + w;
    }
    return xcd_tile(b, nb);
}

// ---------------------------------------------------------------------------
// Multi-shift CG state kept on the device (scalars never leave the GPU inside
// the iteration loop).
constexpr int kMaxPoles = STAG_MAX_POLES;

// Scalars of one iteration; two copies alternate so that every block of the
// update kernel can read iteration k while block 0 writes iteration k+1.
struct MsIter {
    double zeta[kMaxPoles], zeta_old[kMaxPoles];
    double alpha_old, beta_old;
    double bb;          // <b, b> (known from iteration 0 on)
    double rr;          // <r_k, r_k>
    int active[kMaxPoles];
    int iters_per_pole[kMaxPoles];
    int iter;
    int nonfinite;
};

// Shifted systems are updated once per window of `lag` iterations (at most
// kLagMax); the scalars of the pending iterations wait in MsState::hist.
constexpr int kLagMax = 8;

struct MsHist {
    double as[kMaxPoles], bs[kMaxPoles], zn[kMaxPoles];
    int act[kMaxPoles];
};

struct MsState {
    // constants of the solve, set by the host
    int n, base, maxiter;
    int lag;            // shift-update window (1 = every iteration)
    double tol2;        // tol^2
    double mass_term;   // 4 m^2 + sigma_0
    double c0;          // rational constant term
    double shift[kMaxPoles];   // pole_k - sigma_0
    double coef[kMaxPoles];    // rational residues
    int bb_given;       // 1: it[0].bb is set by the host (refinement of a residual)
    // iteration state
    MsIter it[2];
    // done[j & 1] is read by the launches of iteration j; the step kernel of
    // iteration j sets done[(j + 1) & 1] when the solve stops and carries a
    // set flag forward, so no launch reads a flag that its own blocks write
    int done[2];
    MsIter fin;         // copy of the state at termination
    double true_res2[kMaxPoles];  // |b - (A+sigma_k) x_k|^2 (final check)
    MsHist hist[kLagMax];         // scalars of iteration i at hist[i % lag]
};

// Pointer bundles passed by value to kernels.
struct VecPtrs {
    void* p[kMaxPoles];
    template <class T>
    __host__ __device__ T* at(int k) const { return (T*)p[k]; }
};

// ---------------------------------------------------------------------------
// Optional timing of the next launch: when set, launchers that support it
// dispatch through hipExtLaunchKernelGGL so that the two events carry the
// kernel's own start and end timestamps (the same interval a kernel trace
// reports).  Host-side, per thread.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchTiming& next_launch_timing() {
    static thread_local LaunchTiming t;
    return t;
}

template <class K, class... Args>
inline void timed_launch(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    LaunchTiming& t = next_launch_timing();
    if (t.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, t.stop, 0, args...);
        t.start = t.stop = nullptr;
    } else {
        kernel<<<grid, block, 0, s>>>(args...);
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files).
void launch_gauge_to_internal(const Geom& g, const double2* canon, double2* links, hipStream_t s);
void launch_gauge_to_canon(const Geom& g, const double2* links, double2* canon, hipStream_t s);
void launch_vec_to_internal(const Geom& g, const double2* canon, double2* vec, hipStream_t s);
void launch_vec_to_canon(const Geom& g, const double2* vec, double2* canon, hipStream_t s);
void launch_mom_to_internal(const Geom& g, const double* canon, double* mom, int par_offset, hipStream_t s);
void launch_mom_to_canon(const Geom& g, const double* mom, double* canon, hipStream_t s);
void launch_vec_narrow(const Geom& g, const double2* in, float2* out, hipStream_t s);
void launch_vec_widen(const Geom& g, const float2* in, double2* out, hipStream_t s);
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// y += a x over n doubles
void launch_axpy_real(size_t n, double a, const double* x, double* y, hipStream_t s);

// Multi-shift CG pieces
int ms_update_grid(const Geom& g);
// r = p = p_k = b (in the Krylov precision V), x_k = 0, partials of |b|^2
template <class V>
void launch_ms_init(const Geom& g, const double2* b, V* r, V* p, VecPtrs x, VecPtrs ps, const MsState* st,
                    double* qout, hipStream_t s);
// Shifted systems updated together per thread in a window flush.
constexpr int kFlushGroup = 4;
// Constants of one step launch: MsState's n, base and lag, and the ring slot
// j % lag of its iteration j.
struct MsStepConst {
    int n, base, lag, slot;
};
// one iteration's scalars (from the partials of the previous kernels) and the
// fused r, p, x_k, p_k update; par = iteration parity.  x_k stay FP64.
// rows > 1 spreads a window flush's shift groups over that many block rows
// (any rows >= 1 gives the same results).
template <class V>
void launch_ms_step(const Geom& g, V* r, const V* Ap, V* p, VecPtrs x, VecPtrs ps, MsState* st, const double* dpart,
                    int nb2, const double* qin, double* qout, int par, int rows, MsStepConst sc, hipStream_t s);
// Window flush of the fused loop (see blas.hip): final = false after iteration
// j (j % L == 0, gated by the stop flag that iteration's D_oe launch writes),
// true once after the loop for the steps pending at the stop; V: the Krylov
// precision of the ring and of the shifted p_k (x_k stay FP64)
template <class V>
void launch_ms_flush(const Geom& g, const V* ring, VecPtrs x, VecPtrs ps, const MsState* st, const int* gate,
                     int n, int base, int L, bool final_flush, int rows, hipStream_t s);
// p = r and partials of |r|^2 (restart of a CG from a given residual)
void launch_cg_restart(const Geom& g, const float2* r, float2* p, double* qout, hipStream_t s);
// out = c0 b + sum_k coef_k x_k with c0, coef, n read from st
void launch_rational_sum(const Geom& g, const double2* b, VecPtrs x, const MsState* st, double2* out,
                         hipStream_t s);
// block partials of Re <a, b>
void launch_dot_re(const Geom& g, const double2* a, const double2* b, double* part, hipStream_t s);
int dot_grid(const Geom& g);
// out[k] = sum_b part[k*nb + b], k < K, in block order (one block)
void launch_finalize(const double* part, int nb, int K, double* out, hipStream_t s);
// out[0] = sum of nb partials, out[1..npad) = 0 (a partial array of another grid)
void launch_finalize_pad(const double* part, int nb, double* out, int npad, hipStream_t s);
// v *= 1 / sqrt(s2[0]), s2 a device scalar
void launch_scale_rsqrt(const Geom& g, double2* v, const double* s2, hipStream_t s);

// Forces and MD
// w1 weights the one-hop term (c1 of the improved operator, 1 otherwise)
void launch_fermion_force(const Geom& g, const double2* links, VecPtrs X, VecPtrs Y, const double* coef,
                          int n, double* mom, double dt, hipStream_t s, double w1 = 1.0);
// the three-hop term of the improved operator's force, added to mom (w3: a
// link-shaped scratch field, 144 B per link)
void launch_naik_force3(const Geom& g, const double2* links, VecPtrs X, VecPtrs Y, const double* coef, int n,
                        double2* w3, double c3, double* mom, double dt, hipStream_t s);
void launch_gauge_force(const Geom& g, const double2* links, double beta, double* mom, double dt,
                        hipStream_t s);
void launch_link_update(const Geom& g, double2* links, const double* mom, double dt, hipStream_t s);
// block partials (grid returned) of sum Re tr P and of sum p_a^2
int launch_plaquette(const Geom& g, const double2* links, double* part, hipStream_t s);
int launch_kinetic(const Geom& g, const double* mom, double* part, hipStream_t s);

// Random fields
void launch_random_momentum(const Geom& g, uint64_t seed, uint64_t traj, double* mom, hipStream_t s);
constexpr uint32_t kFieldSource = 1, kFieldNoise = 3;
void launch_random_source(const Geom& g, uint64_t seed, uint64_t traj, double2* xi, hipStream_t s,
                          uint32_t field = kFieldSource);
void launch_philox(const uint32_t ctr[4], const uint32_t key[2], size_t n, uint32_t* out, hipStream_t s);
void launch_uniform(uint64_t seed, uint64_t traj, double* out, hipStream_t s);

}  // namespace stag
