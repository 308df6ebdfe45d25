/*
 * stag.h -- C ABI of the MI355X (gfx950) staggered-fermion RHMC library.
 *
 * The library implements the hot path of two-flavour staggered RHMC as set
 * out in Gupta & Majumdar, arXiv:1710.09178: the even-odd staggered Dirac
 * operator (Sec. 3.2), the multi-shift conjugate gradient for the
 * partial-fraction rational functions of eq. (ratapprx) (Sec. 4), the
 * pseudofermion and gauge forces and the leapfrog molecular dynamics of the
 * HMC trajectory (Sec. 3.1), with the Metropolis test on the rational action.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: dims = {Nx, Ny, Nz, Nt}, all even and >= 2.  Site (x,y,z,t) has the
 *   0-based lexicographic address l = x + Nx*(y + Ny*(z + Nz*t)) (Sec. 2) and
 *   checkerboard parity (x+y+z+t) mod 2 (0 = even).  V = Nx*Ny*Nz*Nt, Vh = V/2.
 * Operator: M = 2m + D (Sec. 3.2); D carries the Kogut-Susskind phases
 *   eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z) and an
 *   antiperiodic time boundary; the stored links are plain SU(3) matrices and
 *   the signs are applied on the fly.  A = (M^dag M)_ee = 4m^2 - D_eo D_oe.
 * Canonical (boundary) formats, little-endian IEEE doubles, C order:
 *   gauge     complex128 U[t][z][y][x][mu][3][3]           (V*4*9*16 bytes)
 *   half vec  complex128 psi[k][3], k = rank of the site among the sites of
 *             one parity in lexicographic order              (Vh*3*16 bytes)
 *   momentum  float64 P[t][z][y][x][mu][8], coordinates of sum_a P_a lambda_a/2
 * Internal formats (what the compute entry points take): structure-of-arrays
 *   device buffers sized by stag_field_bytes(); convert with the *_import /
 *   *_export calls.  Their byte layout is private to the library.
 * Pointers: every array argument is a DEVICE pointer (hipMalloc / torch CUDA
 *   tensor), at least 16-byte aligned, owned by the caller, unless the
 *   parameter says "host".  Host arrays are read during the call only.
 * Streams: all work is ordered after prior work on the stream given to
 *   stag_create and later work on that stream sees its results.  Calls that
 *   return host-side numbers (solve info, actions, trajectory info) block until
 *   those numbers are ready; the others return without waiting.
 * Errors: every call returns a stag_status.  Arguments are validated before
 *   any work is enqueued; on error nothing is modified and stag_last_error()
 *   describes the problem.  STAG_ERR_NOT_CONVERGED is non-fatal: outputs hold
 *   the last iterate and the info structure is filled.
 * Threading: a handle must not be used by two threads at once.
 * Memory: the library allocates its workspace in stag_create, on the first
 *   solve that needs more shift vectors than any earlier one, and on the first
 *   use of an optional feature (compressed or FP32/FP16 link copies, the FP32
 *   Krylov workspace, trajectory staging buffers, captured iteration graphs);
 *   it never allocates inside an iteration.
 */
#ifndef STAG_H
#define STAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stag_ctx* stag_handle;

typedef enum {
    STAG_OK = 0,
    STAG_ERR_INVALID_ARG = -1,   /* bad pointer, size, dims, parity, pole list */
    STAG_ERR_NO_GAUGE = -2,      /* a compute call before stag_set_gauge */
    STAG_ERR_NOT_CONVERGED = -3, /* solver hit maxiter; info is filled */
    STAG_ERR_NONFINITE = -4,     /* NaN/Inf met in a reduction */
    STAG_ERR_SPECTRUM = -5,      /* a rational table's interval does not cover the spectrum of A */
    STAG_ERR_HIP = -6,           /* a HIP runtime call failed */
    STAG_ERR_OOM = -7            /* device allocation failed */
} stag_status;

typedef enum {
    STAG_FIELD_HALF_VEC = 0,        /* internal half-lattice colour vector */
    STAG_FIELD_MOM = 1,             /* internal momentum / force field */
    STAG_FIELD_CANON_HALF_VEC = 2,  /* canonical complex128 [Vh][3] */
    STAG_FIELD_CANON_GAUGE = 3,     /* canonical complex128 [V][4][3][3] */
    STAG_FIELD_CANON_MOM = 4        /* canonical float64 [V][4][8] */
} stag_field_kind;

/* Rational function r(x) = c0 + sum_k residue[k] / (x + pole[k])
 * (eq. ratapprx).  pole[k] >= 0, at most STAG_MAX_POLES terms; host arrays. */
#define STAG_MAX_POLES 48
typedef struct {
    int n;
    double c0;
    const double* residue;
    const double* pole;
} stag_rational;

/* Filled by the solver entry points.  true_resid / iters_per_pole may be NULL;
 * otherwise they are host arrays of length n (the number of poles). */
typedef struct {
    int iters;                  /* multi-shift iterations run */
    int n;                      /* number of poles */
    double* true_resid;         /* |b - (A + pole_k) x_k| / |b| per pole, FP64 */
    int* iters_per_pole;        /* iteration at which pole k was frozen */
    double seconds;             /* wall time of the call */
} stag_solve_info;

/* ---- lifecycle -------------------------------------------------------- */

/* Create a handle for one lattice.  dims: host int[4] {Nx,Ny,Nz,Nt}, all even
 * and >= 2, V < 2^31.  hip_stream: a hipStream_t (NULL = the null stream).
 * Allocates the gauge field and the fixed workspace on the current device. */
stag_status stag_create(stag_handle* out, const int dims[4], void* hip_stream);
stag_status stag_destroy(stag_handle h);
/* Message of the last failed call on h (or of the last failed stag_create when
 * h is NULL).  The string lives until the next call on h. */
const char* stag_last_error(stag_handle h);
/* Bytes of one field of the given kind for this handle's lattice. */
size_t stag_field_bytes(stag_handle h, int kind);

/* ---- fields (Sec. 2 layouts) --------------------------------------------- */

/* Copy a canonical gauge field into the handle (converted to the internal
 * layout).  The links are used as given; they should be SU(3). */
stag_status stag_set_gauge(stag_handle h, const double* U_canon);
/* Write the handle's gauge field in the canonical layout. */
stag_status stag_get_gauge(stag_handle h, double* U_canon_out);
/* Convert a canonical half vector of parity 0/1 to the internal layout and back. */
stag_status stag_vec_import(stag_handle h, void* out_internal, const double* canon_in, int parity);
stag_status stag_vec_export(stag_handle h, double* canon_out, const void* in_internal, int parity);
/* Convert a canonical momentum field to the internal layout and back. */
stag_status stag_mom_import(stag_handle h, void* out_internal, const double* canon_in);
stag_status stag_mom_export(stag_handle h, double* canon_out, const void* in_internal);

/* ---- operators (Sec. 3.2) ----------------------------------------------- */

/* out = D_oe in (out_parity = 1, in even) or D_eo in (out_parity = 0, in odd).
 * in and out must not overlap. */
stag_status stag_dslash(stag_handle h, void* out, const void* in, int out_parity);
/* out_even = A in_even = (4 m^2 - D_eo D_oe) in_even.  in and out must not overlap. */
stag_status stag_mdagm(stag_handle h, void* out_even, const void* in_even, double mass);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operator as stag_mdagm, the same kernels and bitwise the same result, with
 * the odd temporary D_oe in_even held in a library-owned static device array
 * of 32 MiB per GPU (resolved by stag_create, kept until the process ends)
 * instead of the handle's workspace.  Makes no hipMalloc/hipFree call: the
 * link copies a 12-real format or the Naik improvement needs are allocated by
 * stag_set_link_format / stag_set_naik (STAG_ERR_INVALID_ARG if missing).
 * STAG_ERR_INVALID_ARG when the odd half vector (48 B x Vh) exceeds 32 MiB
 * (Vh > 699050 sites), for NULL, misaligned or equal pointers or a non-finite
 * mass; STAG_ERR_NO_GAUGE before stag_set_gauge.  All handles on one GPU share
 * the array: calls that overlap in time on one GPU (different streams or
 * threads) race on it; calls ordered on one stream do not.  Asynchronous like
 * stag_mdagm. */
stag_status stag_mdagm_noalloc(stag_handle h, void* out_even, const void* in_even, double mass);

/* ---- multi-shift CG (Sec. 4, eq. ratapprx) ------------------------------- */

/* Solve (A + pole_k) x_k = b for all poles of r with one Krylov space, base
 * system = smallest pole; pole k is frozen when its recursive residual falls
 * below tol*|b|.  x_even: NULL or n internal even vectors (device pointers,
 * held in a host array) receiving x_k.  sum_even: NULL or an internal even
 * vector receiving r(A) b = c0 b + sum_k residue_k x_k.  b may not alias any
 * output.  info may be NULL.  Returns NOT_CONVERGED if maxiter is reached. */
stag_status stag_multishift_solve(stag_handle h, double mass, const stag_rational* r, double tol,
                                  int maxiter, const void* b_even, void* const* x_even,
                                  void* sum_even, stag_solve_info* info);

/* ---- spectral range (Appendix) ------------------------------------------ */

/* Power iteration of A = 4m^2 - D_eo D_oe on the handle's links: starting
 * from the estimator-noise vector (seed, 0) of stag_chiral_condensate, A is
 * applied iters times (normalising on the way) and lam_out receives the
 * Rayleigh quotient <v, A v> / <v, v>: a lower estimate of the largest
 * eigenvalue that rises to it with iters.  Host out. */
stag_status stag_power_estimate(stag_handle h, double mass, int iters, uint64_t seed, double* lam_out);
/* Does the interval [xmin, xmax] of a rational table cover the spectrum of A?
 * The Appendix needs the approximation interval to reach below the smallest
 * eigenvalue (2m)^2 and above the largest.  A = 4m^2 + D_oe^dag D_oe, so 4m^2
 * is a lower bound and 4m^2 + 64 an upper one (|D_oe| <= 8).  Returns
 * STAG_ERR_SPECTRUM (message in stag_last_error) when xmin > 4m^2, or when
 * xmax < 4m^2 + 64 and 1.1 times the power estimate after 100 iterations
 * exceeds xmax; STAG_OK otherwise.  lam_out (may be NULL): the estimate, or 0
 * when the certain bound made it unnecessary. */
stag_status stag_check_spectrum(stag_handle h, double mass, double xmin, double xmax, double* lam_out);

/* ---- precision form ------------------------------------------------------ */

/* Storage of the links read by the Dirac operator.  The 12-real formats keep
 * rows 0 and 1 and rebuild row 2 = conj(row0 x row1), exact for SU(3). */
typedef enum {
    STAG_LINKS_F64_18 = 0,   /* FP64, 18 reals per link (default) */
    STAG_LINKS_F64_12 = 1,   /* FP64, 12 reals per link */
    STAG_LINKS_F32_18 = 2,   /* FP32, 18 reals (FP32 Krylov solves only) */
    STAG_LINKS_F16_12 = 3    /* IEEE FP16, 12 reals (FP32 Krylov solves only) */
} stag_link_format;

/* Storage used by every FP64 operator application of h (Dslash, A, solves,
 * forces): STAG_LINKS_F64_18 or STAG_LINKS_F64_12.  The compressed copy is
 * derived from the handle's links whenever they change. */
stag_status stag_set_link_format(stag_handle h, int format);

/* Operator improvement (Sec. 8 Summary: "improved" staggered quarks, whose
 * stencil reaches past the nearest neighbours).  With (c1, c3) != (1, 0)
 * every operator application of h -- stag_dslash, stag_mdagm, the sloppy
 * operators and all solves -- uses the Naik-improved hopping term
 *   c1 sum_mu s_mu(x) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)]
 * + c3 sum_mu s3_mu(x) [L_mu(x) psi(x+3mu) - L_mu(x-3mu)^dag psi(x-3mu)],
 * L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu), with the staggered phase of
 * direction mu once per path and -1 per link of the path that leaves the last
 * time slice.  Tree-level improvement is c1 = 9/8, c3 = -1/24; (1, 0) restores
 * the one-hop operator.  The long links are derived from the links (in the
 * format set by stag_set_link_format, and the sloppy formats on demand) at
 * the first operator call after every change of the links; the first use
 * allocates them (144 B per link in FP64), together with a link-shaped
 * scratch field of the pseudofermion force (another 144 B per link).  The
 * pseudofermion force, and with it every trajectory, then differentiates the
 * improved action: each link moves in its one-hop term and at the three
 * positions of the three-link paths through it.  Returns
 * STAG_ERR_INVALID_ARG for non-finite weights. */
stag_status stag_set_naik(stag_handle h, double c1, double c3);

/* The sloppy operator of the precision form, applied to FP64 internal vectors
 * so that its error against the FP64 operator can be measured: in is rounded
 * to FP32, D (stag_dslash_sloppy: out_parity 1 = D_oe, 0 = D_eo) or
 * A = 4m^2 - D_eo D_oe (stag_mdagm_sloppy) is applied in FP32 arithmetic with
 * the links stored in `format` (STAG_LINKS_F32_18 or STAG_LINKS_F16_12, row 2
 * rebuilt as conj(row0 x row1) in FP32), exactly as inside the FP32 Krylov
 * solves, and the result is widened to FP64 in out (Sec. 3.2 operator; the
 * paper's remarks on FP32 and link compression).  in and out must not
 * overlap.  The first call allocates the link copy and the FP32 vectors. */
stag_status stag_dslash_sloppy(stag_handle h, void* out, const void* in, int out_parity, int format);
stag_status stag_mdagm_sloppy(stag_handle h, void* out_even, const void* in_even, double mass, int format);

typedef struct {
    int sloppy;              /* STAG_LINKS_F32_18 or STAG_LINKS_F16_12 (FP32 vectors in both) */
    double tol_sloppy;       /* FP32 multi-shift phase stops at this relative residual, e.g. 1e-5 */
    int reliable_every;      /* FP64 true-residual recompute interval of the refinement CG, e.g. 50 */
} stag_mixed_opts;

/* Same contract as stag_multishift_solve (outputs, tolerance meaning: FP64
 * true residual |b - (A+pole_k) x_k| <= tol |b| for every pole), computed in
 * mixed precision: an FP32 multi-shift CG with FP64 solution accumulators and
 * FP64 reductions down to tol_sloppy, then for each pole a CG in FP32 started
 * from the FP64 residual whose residual is recomputed in FP64 (with FP64 links)
 * every reliable_every iterations.  info->iters counts all iterations of both
 * phases; info->iters_per_pole[k] = multi-shift iterations of pole k plus its
 * refinement iterations. */
stag_status stag_multishift_solve_mixed(stag_handle h, double mass, const stag_rational* r, double tol,
                                        int maxiter, const void* b_even, void* const* x_even,
                                        void* sum_even, const stag_mixed_opts* opts,
                                        stag_solve_info* info);

/* ---- actions and forces (eq. pfact; Sec. 3.1) ---------------------------- */

/* S_f = phi^dag r(A) phi with r the action's rational function (host out). */
stag_status stag_fermion_action(stag_handle h, double mass, const stag_rational* r, double tol,
                                int maxiter, const void* phi_even, double* S_out,
                                stag_solve_info* info);
/* Pseudofermion force F = -dS_f/dw for S_f = phi^dag r(A) phi, per link in
 * algebra coordinates (with the operator set by stag_set_naik).  dt == 0:
 * mom = F; otherwise mom += dt * F. */
stag_status stag_fermion_force(stag_handle h, double mass, const stag_rational* r, double tol,
                               int maxiter, const void* phi_even, void* mom, double dt,
                               stag_solve_info* info);
/* Wilson gauge force for S_g = beta sum_{x,mu<nu} (1 - Re tr P/3); same dt rule. */
stag_status stag_gauge_force(stag_handle h, double beta, void* mom, double dt);
/* S_g of the handle's links and the mean plaquette <Re tr P / 3> (host outs, may be NULL). */
stag_status stag_gauge_action(stag_handle h, double beta, double* S_out, double* plaq_out);
/* Polyakov loop of the handle's links: (1 / (3 Nx Ny Nz)) times the sum over
 * spatial sites x of tr [U_t(x,0) U_t(x,1) ... U_t(x,Nt-1)], the ordered
 * product of the time links closing around the periodic time direction; a
 * gauge-invariant observable of the sampled configurations (expectation
 * values, Sec. 2).  Host outs re and im, either may be NULL.  Errors: no
 * gauge field set (STAG_ERR_NO_GAUGE), HIP failures. */
stag_status stag_polyakov_loop(stag_handle h, double* re_out, double* im_out);
/* Chiral condensate of one staggered field, (1/V) Tr M^{-1} for M = 2m + D,
 * estimated with n_noise Gaussian noise vectors on the even sites (the
 * distribution of stag_random_source, drawn from a separate estimator-noise
 * field of the counter (seed, k), k < n_noise, so never equal to a heat-bath
 * source of a chain with the same seed): since only the
 * parity-preserving part of M^{-1} = (2m - D)(4m^2 - D^2)^{-1} has a trace
 * and both parity blocks have the same spectrum, Tr M^{-1} = 4m Tr_e A^{-1},
 * estimated by (4m/V) Re <eta, A^{-1} eta> (an observable of the sampled
 * configurations, Sec. 2).  Host outs: the mean and, if err_out is not NULL,
 * its standard error (0 for one source).  Each source is solved to tol.
 * Errors: no gauge field, invalid arguments, NOT_CONVERGED, NONFINITE. */
stag_status stag_chiral_condensate(stag_handle h, double mass, double tol, int maxiter, int n_noise,
                                   uint64_t seed, double* mean_out, double* err_out);
/* K = (1/2) sum over links and a of mom_a^2 (host out). */
stag_status stag_kinetic_energy(stag_handle h, const void* mom, double* K_out);
/* U <- exp(i dt p) U for every link, then projection back to SU(3)
 * (Gram-Schmidt of rows 0,1; row 2 = conj(row0 x row1)). */
stag_status stag_link_update(stag_handle h, const void* mom, double dt);

/* ---- random fields (Philox4x32-10, Box-Muller) --------------------------- */

/* Gaussian momenta, each coordinate N(0,1).  Stream: key = seed, counter =
 * (draw index, field 0, traj); link 4l+mu uses draws 4(4l+mu)+q, q = 0..3. */
stag_status stag_random_momentum(stag_handle h, uint64_t seed, uint64_t traj, void* mom_out);
/* Gaussian even half vector with density exp(-xi^dag xi) (field 1; site k,
 * colour q uses draw 3k+q, real/imag parts N(0,1/2)). */
stag_status stag_random_source(stag_handle h, uint64_t seed, uint64_t traj, void* xi_even_out);
/* Raw Philox4x32-10 words: out[4i..4i+3] = philox(ctr + (i,0,0,0), key) for
 * i < n (ctr word 0 wraps mod 2^32).  ctr, key: host arrays. */
stag_status stag_philox(const uint32_t ctr[4], const uint32_t key[2], size_t n, uint32_t* out_dev,
                        void* hip_stream);

/* ---- one RHMC trajectory (Sec. 3.1) -------------------------------------- */

/* ---- learned force model (optional stand-in for the pseudofermion force) -- */

/* A gauge-covariant force model tied to lattice h: per link, an MLP
 * (16 -> 64 -> 64 -> 8, SiLU; bf16 matrix-core products, FP32 accumulation)
 * maps gauge-invariant inputs (Re/Im tr of U S_j for the link's six plaquette
 * staples S_j, site parity, staggered sign, and the cosine of the auxiliary
 * force G with the staple sum) to coefficients c_j, and
 * F_a = sum_{j<6} c_j Im tr(T_a U S_j) + c_6 G_a (G = 0 without one).
 * capacity = number of (gauge field, force) training pairs the device dataset
 * can hold. */
typedef struct stag_surrogate* stag_surrogate_handle;
stag_status stag_surrogate_create(stag_surrogate_handle* out, stag_handle h, int capacity, uint64_t seed);
stag_status stag_surrogate_destroy(stag_surrogate_handle s);
const char* stag_surrogate_last_error(stag_surrogate_handle s);
/* Number of FP32 parameters: W1[64][16], b1[64], W2[64][64], b2[64], W3[8][64], b3[8]. */
int stag_surrogate_param_count(void);
/* Read (get_out) and/or replace (set_in, resets the optimiser) the parameters; host arrays. */
stag_status stag_surrogate_params(stag_surrogate_handle s, float* get_out, const float* set_in);
/* Auxiliary force field of the model (device, internal momentum layout, read
 * by later add_pair / eval / force calls) or NULL for none: the seventh
 * channel, weighted per link like the six staple forces. */
stag_status stag_surrogate_set_aux(stag_surrogate_handle s, const void* aux_force);
/* Training pairs stored so far, and the dataset capacity (0 for a NULL handle). */
int stag_surrogate_pair_count(stag_surrogate_handle s);
int stag_surrogate_capacity(stag_surrogate_handle s);
/* Store one training pair: the features of h's current gauge field and the
 * given target force (internal momentum layout, e.g. from stag_fermion_force). */
stag_status stag_surrogate_add_pair(stag_surrogate_handle s, const void* force);
/* Adam (lr) over all stored pairs, one step per pair and epoch; loss_out =
 * mean over the last epoch of (1/links) sum |F_model - F_target|^2. */
stag_status stag_surrogate_train(stag_surrogate_handle s, int epochs, double lr, double* loss_out);
/* Loss of the model on h's current gauge field against a target force; with
 * grad_out (host, param_count floats) also its gradient. */
stag_status stag_surrogate_eval(stag_surrogate_handle s, const void* force, double* loss_out, float* grad_out);
/* Model force on h's current gauge field: mom = F (dt == 0) or mom += dt F. */
stag_status stag_surrogate_force(stag_surrogate_handle s, void* mom, double dt);

typedef struct {
    double beta, mass, tau;
    int n_steps;                  /* leapfrog steps, dt = tau / n_steps */
    stag_rational r_md;           /* force: approximates x^(-1/2) */
    stag_rational r_action;       /* action: approximates x^(-1/2) */
    stag_rational r_heatbath;     /* heat bath: approximates x^(+1/4) */
    double tol_md, tol_action;
    int maxiter;
    uint64_t seed, traj_index;    /* random stream of this trajectory */
    const void* inject_mom;       /* NULL or internal momentum used instead of the RNG */
    const void* inject_xi;        /* NULL or internal even vector used instead of the RNG */
    double inject_u;              /* Metropolis uniform in [0,1), or < 0 to draw it */
    int no_fermions;              /* 1: pure gauge trajectory (tests) */
    stag_surrogate_handle surrogate;  /* NULL, or a model standing in for the pseudofermion force
                                         (kicks k = 0..n_steps; see exact_every, coarse_force) */
    int exact_every;              /* >= 1; with n_steps % exact_every == 0 the set of exact kicks is
                                     symmetric under k -> n_steps - k, keeping leapfrog reversible.
                                     The accept/reject step always uses the exact rational action. */
    int coarse_force;             /* 1: two-time-scale leapfrog (needs n_steps % exact_every == 0).  The
                                     kicks k % exact_every == 0 carry exact_every times the impulse of
                                     the exact force minus the model's; the model alone acts on every
                                     kick.  Without a model this is the ablation (exact force on the
                                     outer scale only).  0 with a model: the model replaces the exact
                                     force on the non-exact kicks. */
    int record_pairs;             /* 1, with a model and exact_every == 1: every pseudofermion force of
                                     the trajectory is also stored as a training pair of the model,
                                     until its dataset is full */
    int inner_iters;              /* > 0, with a model: wherever the model is evaluated (and for every
                                     recorded pair) its auxiliary force is the pseudofermion force of
                                     a multi-shift solve of r_md stopped after inner_iters iterations;
                                     the model's auxiliary field is left NULL afterwards */
    int md_link_format;           /* 0: the MD force solves in FP64.  STAG_LINKS_F32_18 or
                                     STAG_LINKS_F16_12: FP32 Krylov vectors with links in that format
                                     (FP64 solutions and reductions), to tol_md on the recursive
                                     residual, no refinement.  The force stays a deterministic
                                     function of the links, so the algorithm stays exact; heat bath
                                     and actions are always FP64. */
    double spectrum_lo, spectrum_hi; /* both 0: no check.  Otherwise the interval the rational tables
                                     were made for: the trajectory first checks it against the
                                     spectrum of A on its starting links (stag_check_spectrum) and
                                     returns STAG_ERR_SPECTRUM, with nothing changed, if it does not
                                     cover it */
    int judge_model;              /* 1, with a model: at every exact kick the model's force is also
                                     evaluated on the same links and compared with the exact force
                                     (info->model_force_err); the exact kick then adds dt * F from a
                                     separate force field, which changes its rounding, not the method */
} stag_hmc_params;

typedef struct {
    double dH;
    double K_old, Sg_old, Sf_old;
    double K_new, Sg_new, Sf_new;
    double plaquette;             /* of the configuration kept */
    int accepted;
    int cg_iters_total;
    int n_solves;
    double seconds;
    double model_force_err;       /* mean of |F_model - F| / |F| over the exact kicks (judge_model),
                                     -1 when not judged */
    int used_model;               /* 1 when a model stood in for the force on some kicks */
} stag_traj_info;

/* Heat bath, leapfrog integration and Metropolis test on the handle's gauge
 * field; on rejection the field is restored.  info may be NULL.  Errors:
 * invalid parameters (nothing done), NOT_CONVERGED / NONFINITE from a solve,
 * model failures: on every error after the heat bath the gauge field is
 * restored to its state at the call and the model's auxiliary field is
 * detached, so the handle still holds the chain's configuration. */
stag_status stag_md_trajectory(stag_handle h, const stag_hmc_params* p, stag_traj_info* info);

/* A chain of n_traj trajectories (indices p->traj_index, +1, ...) where the
 * exact force is the fallback of the model and its judge: trajectories that
 * use the model (p->surrogate with its schedule) are judged (judge_model), and
 * after one whose judged force error exceeds max_model_err, or once the last
 * `window` model trajectories accepted less than min_acceptance on average,
 * the next exact_trajectories trajectories run with the exact force on every
 * kick before the model is tried again.  Decisions use completed
 * trajectories only, never a trajectory in progress: every trajectory is an
 * exact, reversible RHMC update (its Metropolis test takes the exact action
 * whichever force drove it), while the choice between the two integrators
 * depends on the chain's history, as in any adaptive scheme.  The fallback
 * trajectories run with exact_every 1 and without coarse_force,
 * record_pairs or inner_iters; without a model (p->surrogate NULL) every
 * trajectory runs with p's own schedule.  infos: host [n_traj]; n_done (may be NULL):
 * the trajectories completed (all of them unless an error stops the chain,
 * whose status is returned).  STAG_ERR_INVALID_ARG for window < 1,
 * exact_trajectories < 1, max_model_err <= 0 or min_acceptance outside
 * [0, 1]. */
typedef struct {
    int window;
    double min_acceptance;
    double max_model_err;
    int exact_trajectories;
} stag_chain_policy;
stag_status stag_md_chain(stag_handle h, const stag_hmc_params* p, int n_traj, const stag_chain_policy* policy,
                          stag_traj_info* infos, int* n_done);

/* ---- batched form: many lattices x right-hand sides x poles ---------------- */

typedef struct stag_batch* stag_batch_handle;

#define STAG_BATCH_MAX_RHS 4

/* A batch of n_inst independent lattices (dims: host int[n_inst][4], each
 * extent even and >= 2) with nrhs right-hand sides each (1..4).  Every
 * multi-shift kernel launch covers all tiles of all lattices, and the Dslash
 * applies each link it loads to all nrhs vectors of its lattice. */
stag_status stag_batch_create(stag_batch_handle* out, int n_inst, const int* dims, int nrhs, void* hip_stream);
stag_status stag_batch_destroy(stag_batch_handle b);
const char* stag_batch_last_error(stag_batch_handle b);
/* Bytes of one packed canonical batch vector: for lattice i (in order) and
 * right-hand side j, the canonical even half vector complex128 [Vh_i][3]. */
size_t stag_batch_vec_bytes(stag_batch_handle b);
/* Canonical gauge field (device, complex128 [V_i][4][3][3]) of lattice inst. */
stag_status stag_batch_set_gauge(stag_batch_handle b, int inst, const double* U_canon);

typedef struct {
    int precision;        /* 0: FP64 links and Krylov vectors; 1: FP32 links and Krylov
                             vectors (FP64 solutions and reductions) to tol_sloppy, then
                             FP64 CG refinement of every pole to tol */
    double tol;           /* per system and pole: |b - (A_i + pole) x| <= tol |b| */
    double tol_sloppy;    /* precision 1 only */
    int maxiter;
    int use_graph;        /* 1: replay chunks of iterations from a captured hipGraph */
} stag_batch_opts;

typedef struct {
    int iters;            /* multi-shift iterations until the last system stopped */
    int refine_iters;     /* precision 1: CG iterations of the refinement (sum over poles) */
    double seconds;       /* wall time of the call */
    double* latency;      /* NULL or host [n_inst*nrhs]: seconds from the start of the solve
                             to the stop of each system (device wall clock) */
    double* true_resid;   /* NULL or host [n_inst*nrhs*n_poles]: FP64 |b-(A+pole)x|/|b| */
    int* iters_sys;       /* NULL or host [n_inst*nrhs]: multi-shift iterations per system */
    int* iters_per_pole;  /* NULL or host [n_inst*nrhs*n_poles]: multi-shift iteration at which
                             each pole of each system stopped */
} stag_batch_info;

/* Solve (A_i + pole_k) x = b for every lattice i (mass masses[i], host
 * array), right-hand side and pole of r.  b: one packed canonical batch
 * vector; x: n_poles packed canonical batch vectors one after the other (pole
 * k at byte offset k * stag_batch_vec_bytes).  Both device pointers. */
stag_status stag_batch_solve(stag_batch_handle b, const double* masses, const stag_rational* r, const void* b_canon,
                             void* x_canon, const stag_batch_opts* opts, stag_batch_info* info);
/* Shift-update window of the batched multi-shift solver: 1, 2, 4 or 8
 * iterations (default 8); results do not depend on it.  Tuning. */
stag_status stag_batch_set_shift_window(stag_batch_handle b, int lag);
/* Autotune the Dslash work split for this batch: times the batched operator
 * for 1, 2, 4 and 8 threads per site (precision 0 or 1) and keeps the
 * fastest.  us_out: NULL or host [4] microseconds per application. */
stag_status stag_batch_tune(stag_batch_handle b, int precision, double* us_out);
/* Autotuner with a persisted cache: the batched operator is timed (precision
 * 0 or 1, 10 applications each) for every work split -- 1, 2 or 4 threads per
 * site (tiles of 256, 128, 64 sites) with plain or non-temporal link loads,
 * and 8 lanes per site (one hop per lane) -- and the fastest is kept.
 * cache_path (NULL or "" for none): a text file of lines
 * "key threads_per_site link_nt microseconds", key = device architecture,
 * precision, right-hand sides and the multiset of lattice shapes; a batch
 * whose key is in the file takes its entry without timing, a tuned one is
 * appended.  us_out: NULL or host [7] microseconds in the candidate order
 * (tps 1, 2, 4 plain; 1, 2, 4 non-temporal; 8), -1 when read from the cache.
 * choice_out: NULL or host [3] = {threads per site, link_nt, from cache}.
 * Results of the solver do not depend on the choice. */
stag_status stag_batch_autotune(stag_batch_handle b, int precision, const char* cache_path, double* us_out,
                                int* choice_out);
/* Link format of the batched operators: STAG_LINKS_F64_18 (default) reads
 * all 18 reals of a link; STAG_LINKS_F64_12 reads rows 0 and 1 (12 reals) and
 * rebuilds row 2 = conj(row 0 x row 1), exact to rounding for SU(3) links
 * (the FP32 operator of the mixed precision then does the same with its FP32
 * copy).  The stored links are unchanged; the key of stag_batch_autotune's
 * cache includes the format.  STAG_ERR_INVALID_ARG for any other format. */
stag_status stag_batch_set_link_format(stag_batch_handle b, int format);
/* Set the Dslash work split directly: 1, 2 or 4 threads per site share the
 * four directions of a site through LDS; 8 lanes per site take one hop each
 * and combine by lane exchanges.  Results agree to rounding.  Tuning. */
stag_status stag_batch_set_tps(stag_batch_handle b, int tps);

/* ---- measurement and tuning (not part of the method) ---------------------- */

/* Record a pair of hipEvents around each Dslash and shift-update launch of the
 * following solves on h (at most max_launches launches in one solve); 0 turns
 * recording off.  Resets the accumulated times. */
stag_status stag_profile_enable(stag_handle h, int max_launches);
/* Accumulated kernel milliseconds and launch counts since stag_profile_enable:
 * index 0 = D_oe (odd <- even), 1 = D_eo with the fused CG epilogue,
 * 2 = fused multi-shift vector update.  Host arrays of length 3, may be NULL.
 * While recording is on, stag_dslash also times its launch (waiting for it)
 * and books it under 0 (D_oe) or 1 (plain D_eo). */
stag_status stag_profile_read(stag_handle h, double ms[3], long counts[3]);
/* The individual recorded launch durations of one kind (index as above), in
 * microseconds and in launch order: *n_out receives the number recorded, the
 * first min(cap, *n_out) go to us_out (host array).  STAG_ERR_INVALID_ARG for
 * a kind outside [0, 2], cap < 0, n_out NULL, or us_out NULL with cap > 0. */
stag_status stag_profile_samples(stag_handle h, int kind, float* us_out, int cap, int* n_out);
/* The fused iteration of multi-shift solves (shift-update window >= 2; FP64,
 * and the FP32 phase of the precision form and of FP32 MD force solves):
 * the base system's update of step j-1 is folded into the D_oe launch of
 * iteration j, which forms p_j = (r_{j-1} - alpha Ap_{j-1}) + beta p_{j-1}
 * where it reads it, and the shifted systems are updated by one flush launch
 * per window -- two launches per iteration instead of three, and one memory
 * round trip before the arithmetic of each.  mode 1 (default): on lattices
 * whose Dslash grid (Vh / 64 blocks) is at most 512 blocks, where iterations
 * are latency-bound; 2: at every size; 0: never (the three-launch loop).
 * The two loops solve the same systems to the same tolerance; their reduction
 * trees differ, so results agree to rounding, not bitwise.  Returns
 * STAG_ERR_INVALID_ARG for a mode outside 0..2. */
stag_status stag_set_fused_iteration(stag_handle h, int mode);
/* How every FP64 operator application of h loads the links (and long links):
 * mode 1 (default) with non-temporal loads when the FP64 field(s) exceed
 * 512 MB -- they cannot stay in the 256 MB Infinity Cache between Dslash
 * launches, and streaming them past it keeps the shared vectors cached --
 * and plain loads otherwise; 0 always plain, 2 always non-temporal.  Results
 * are bitwise the same in every mode.  STAG_ERR_INVALID_ARG for other modes. */
stag_status stag_set_link_streaming(stag_handle h, int mode);
/* Solvers replay each chunk of iterations from a hipGraph captured on first
 * use (kernel nodes only; up to 8 cached per handle, keyed by every launch
 * argument) unless profiling or reliable updates need per-launch work.  on = 0
 * launches every kernel individually.  Results are identical either way. */
stag_status stag_set_graphs(stag_handle h, int on);
/* Multi-shift solver: the shifted solutions and directions are updated once
 * per window of `lag` iterations (1..8, default 8), each read and written once
 * per window; the results do not depend on the window.  Measurement/tuning. */
stag_status stag_set_shift_window(stag_handle h, int lag);
/* Dslash work split: tps = threads cooperating on one output site (1, 2 or 4);
 * chunk = solver iterations enqueued between two convergence polls (>= 1). */
stag_status stag_tune(stag_handle h, int tps, int chunk);

#ifdef __cplusplus
}
#endif
#endif /* STAG_H */
