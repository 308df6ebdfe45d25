// Batched multi-shift CG over many lattices of uneven volume, several right-
// hand sides each, in one launch per kernel.
#pragma once

#include "common.h"

namespace stag {

constexpr int kMaxRhs = 4;

// One lattice of the batch.  Half-lattice sites of all instances are
// concatenated: instance i owns sites [off, off + g.vh).
struct BInst {
    Geom g;
    int off;              // first concatenated half-lattice site
    int tile0, ntiles;    // its tiles in the tile table
    double four_m2;       // 4 m_i^2
};

// A tile is tile_sites consecutive output sites of one instance.
struct BTile {
    int inst;
    int cb0;
};

// Window tables of one system: [lag][n] entries at stride n.
constexpr int kWinTab = kLagMax * kMaxPoles;

// Scalars of one system for the step kernel.
struct BScal {
    double alpha, beta;
    int stop, flush, npend, nact, base_on, slot;
    int list[kMaxPoles];  // shifts to update in a flush, increasing
};

// Per-system state (system s = instance * nrhs + rhs), double-buffered by parity.
struct BState {
    int n_inst, nrhs, n, base, maxiter;
    int bb_given;         // 1: it[0][s].bb holds |b_s|^2 of the original source (refinement)
    double tol2;
    double shift[kMaxPoles];
    MsIter* it[2];        // [n_sys]
    MsIter* fin;          // [n_sys]
    // [2][n_sys] by iteration parity like inst_done: 1 once the system has stopped
    int* sys_done;
    // [2][n_inst] by iteration parity: flag [j & 1] is read by the launches of
    // iteration j; the scalar kernel of iteration j writes [(j + 1) & 1]
    int* inst_done;
    unsigned long long* t_done;  // [n_sys] device wall clock at the stop
    double* sigma0_term;  // [n_inst] 4 m_i^2 + sigma_0
    int lag;              // shift-update window (1..kLagMax); residual ring of `lag` vectors
    MsHist* hist;         // [n_sys][kLagMax] scalars of the pending iterations
    size_t ring_stride;   // entries between ring slots (one batched vector)
    BScal* scal;          // [n_sys] this iteration's scalars (written by the scalar kernel)
    double* w_tab;        // [n_sys][3][kWinTab] alpha_s, beta_s, zeta_s of the window's iterations
    int* w_act;           // [n_sys][kWinTab] shift active in the window's iterations
};

// Internal batched vector: instance i's block starts at 3*R*off_i and holds
// [rhs][colour][site] planes of vh_i entries.
__host__ __device__ __forceinline__ size_t bvec_off(const BInst& I, int R, int rhs, int c) {
    return (size_t)3 * R * I.off + (size_t)(rhs * 3 + c) * I.g.vh;
}
// Links of instance i: [2][4][9][vh_i] starting at 72*off_i entries.
__host__ __device__ __forceinline__ size_t blink_base(const BInst& I) { return (size_t)72 * I.off; }

struct BatchDev {
    const BInst* inst;
    const BTile* tiles;
    int ntiles;
    int tile_sites;
    int nrhs;
    int link_nt;   // links streamed with non-temporal loads (fields beyond the Infinity Cache)
    int link12;    // read rows 0-1 of every link and rebuild row 2 = conj(row 0 x row 1)
};

// Launchers (batch.hip).  V = double2 (FP64 links, FP64 Krylov vectors) or
// float2 (FP32 links, FP32 Krylov vectors); solutions are FP64 in both.
template <class V>
void launch_bdslash(const BatchDev& bd, int tps, const void* links, const V* in, V* out, int out_par,
                    const int* inst_done, hipStream_t s);
template <class V>
void launch_bdslash_cg(const BatchDev& bd, int tps, const void* links, const V* w_o, const V* p, const V* r, V* Ap,
                       BState st, const int* inst_done, double* dpart, hipStream_t s);
// |b - (c_i x - D_eo w_o)|^2 per (tile, rhs), c_i = 4 m_i^2 + pole; optional residual output
void launch_bdslash_resid(const BatchDev& bd, int tps, const double2* links, const double2* w_o, const double2* x,
                          const double2* b, double pole, double* part, double2* rout, hipStream_t s);
template <class V>
void launch_bms_init(const BatchDev& bd, const double2* b, V* r, V* p, VecPtrs x, VecPtrs ps, BState st,
                     double* qout, hipStream_t s);
// One block per instance: sums the instance's partials and evaluates the
// scalars of its systems into st.scal / st.w_tab / st.w_act.
void launch_bms_scalars(const BatchDev& bd, BState st, const double* dpart, const double* qin, int par,
                        hipStream_t s);
// r: the residual ring (st.lag slots of st.ring_stride entries)
template <class V>
void launch_bms_step(const BatchDev& bd, V* r, const V* Ap, V* p, VecPtrs x, VecPtrs ps, BState st,
                     const double* dpart, const double* qin, double* qout, int par, hipStream_t s);
// per system: sum of the (tile, rhs) partials over the instance's tiles
void launch_bsys_sum(const BatchDev& bd, int n_inst, const double* part, double* out, hipStream_t s);
void launch_bvec_import(const BatchDev& bd, const double2* canon, double2* vec, hipStream_t s);
void launch_bvec_export(const BatchDev& bd, const double2* vec, double2* canon, hipStream_t s);
void launch_blinks_to_f32(const double2* d, float2* f, size_t n, hipStream_t s);
void launch_b_timestamp(unsigned long long* t, hipStream_t s);
// fresh iteration state for every system; bb taken from fin[s].bb when from_fin
void launch_bstate_init(BState st, int from_fin, hipStream_t s);
// x += e over n complex entries
void launch_baxpy(size_t n, double2* x, const double2* e, hipStream_t s);

}  // namespace stag
