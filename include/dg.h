/*
 * dg.h -- C ABI of the gfx950 DG ideal-MHD library (libdgmhd.so).
 *
 * The library advances the modal discontinuous-Galerkin discretisation of
 * ideal MHD of Guillet et al., "High-order magnetohydrodynamics for
 * astrophysics with an adaptive mesh refinement discontinuous Galerkin
 * scheme" (MNRAS 2019):
 *   - state: per-cell modal weights w_l^K (Sec. 3.1, eq. u-exp) on the
 *     Legendre basis (Sec. 3.2) or, for the magnetic field under the Powell
 *     scheme, the locally divergence-free basis (Sec. 3.3, App. A);
 *   - right-hand side: the weak form eq. wdot with (d+1)-point Gauss-Legendre
 *     quadrature (Sec. 3.5), HLLD face fluxes with the Alfven-weighted face
 *     normal field (Sec. 4.1.2, eq. bxface-average-alfven), Powell face terms
 *     (Sec. 4.1.3, eq. powell-src-face, eq. powellq-average) or GLM cleaning
 *     (Sec. 4.1.5);
 *   - time step: eq. cfl, the Powell cap eq. powell_dt, c_h and c_p of
 *     Sec. 4.1.5; SSP-RK3 stages (Sec. 3.6);
 *   - limiters after every stage: TVB characteristic slope limiter
 *     (Sec. 4.2.1-4.2.2, eq. tvb-limiter), LDF slope fix (Sec. 4.2.4) and the
 *     positivity limiter (Sec. 4.3, eq. wtilde, eq. tau_rho, eq. tau_press).
 *
 * Conventions shared with every caller:
 *   Variables v = (rho, m1, m2, m3, E, B1, B2, B3, psi); Heaviside-Lorentz
 *   units; ideal gas with adiabatic index gamma.
 *   Legendre modes: l_k normalised by l_k(1) = 1 (mode 0 = cell mean,
 *   mass M = prod 2/(2k+1)); modes of total degree <= d ordered by total
 *   degree, then k1 descending, then k2 descending.  Mode index v*n(d) + l.
 *   Powell: the 5 hydro variables (and B3 in 2-D) on the Legendre basis,
 *   then N_div LDF weights generated as in App. A: curls of the Legendre
 *   products of degree <= d+1 placed in the x, then y, then z component,
 *   stably sorted by degree, Gram-Schmidt orthogonalised, not normalised.
 *   State array: [nmodes][ld], cells fastest, ld a multiple of 64 (see
 *   dg_layout); FP64 if precision == DG_FP64, FP32 otherwise.
 *   Uniform grids: cell index i + n0 (j + n1 k); octree meshes: the caller's
 *   leaf order.
 *
 * Ownership: the caller owns every state / output array (device memory) and
 * the stream.  The handle owns its tables, workspaces and face lists and
 * frees them in dg_destroy.
 *
 * Errors: every call returns DG_OK or a negative code.  DG_EINVAL and
 * DG_EUNSUPPORTED are detected before any device work and leave all arrays
 * untouched.  dg_last_error(h) returns a message for the last failure.  No
 * C++ exception crosses this interface.
 *
 * Concurrency: all device work is ordered on the stream given to dg_init.
 * Calls that return host values (dg_dt, dg_limit with stats, dg_step with a
 * time pointer, dg_proj_points) synchronise that stream.  A handle must not
 * be used from two threads at once.
 */
#ifndef DGMHD_DG_H
#define DGMHD_DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_handle_s* dg_handle;

enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (null pointer, size, unknown enum) */
  DG_EUNSUPPORTED = -2,  /* valid but not built (e.g. degree > 3) */
  DG_EHIP = -3,          /* a HIP runtime call failed */
  DG_ENOMEM = -4,        /* device allocation failed */
  DG_ENONFINITE = -5,    /* a non-finite value appeared in the state */
  DG_ECH = -6            /* warning: GLM with fixed c_h below twice the largest signal
                            speed (Sec. 4.1.5); the call completed and its outputs are valid */
};
enum { DG_GLM = 0, DG_POWELL = 1 };
enum { DG_FP64 = 0, DG_FP32 = 1 };
enum { DG_LIM_TVB = 1, DG_LIM_CHAR = 2, DG_LIM_POS = 4, DG_LIM_LEARNED = 8 };
enum { DG_MESH_UNIFORM = 0, DG_MESH_OCTREE = 1 };
enum { DG_POWELL_Q_MEAN = 0, DG_POWELL_Q_INTERP = 1 };

/* Scheme parameters (Sec. 3.6, 4.1, 4.2, 4.3; defaults of the paper in
 * brackets).  rk_stages selects the SSP Runge-Kutta scheme of Sec. 3.6 (order
 * 1 to 4): 1 forward Euler, 2 SSP-RK2, 3 SSP-RK3 (Shu-Osher), 5 the
 * five-stage fourth-order SSP scheme of Spiteri & Ruuth (in the survey the
 * paper cites, Gottlieb 2005); other values DG_EUNSUPPORTED.  cfl_glm is C' of Sec. 4.1.5
 * (0 selects min(2 cfl, 0.9)); glm_cr is c_r = c_p^2 / c_h [0.18];
 * glm_ch_fixed > 0 fixes c_h (required on octree meshes).  tvb_Mtilde [5],
 * tvb_beta [2], tvb_eps [1e-8]; eps_rho = eps_p [1e-12]; powell_eta [0.2].
 * mlp_lo / mlp_hi bound the band of learned-indicator outputs that falls
 * back to the plain TVB detector.  powell_q (Powell scheme only) selects the
 * state q-dagger of the face term eq. powell-src-face: DG_POWELL_Q_MEAN, q of
 * the cell average (eq. powellq-average, the paper's default), or
 * DG_POWELL_Q_INTERP, q integrated along the straight path in primitive
 * variables from the cell's trace to the HLLD interface state
 * (eq. powellq-interp). */
typedef struct {
  int32_t dim, degree, divb, precision, rk_stages, limiter, powell_q;
  double gamma, cfl, cfl_glm, glm_cr, glm_ch_fixed;
  double tvb_Mtilde, tvb_beta, tvb_eps, eps_rho, eps_p, powell_eta;
  double mlp_lo, mlp_hi;
} dg_params;

/* Mesh on the periodic box [0, box]^dim.  kind == DG_MESH_UNIFORM: n[0..dim)
 * cells per axis, cubic cells (box[a]/n[a] equal), at most 2^31 - 1 cells
 * (DG_EINVAL beyond).  kind == DG_MESH_OCTREE:
 * n[] is the level-0 grid, and leaf c has refinement level level[c] >= 0 and
 * integer coordinates ijk[3c..3c+2] on the grid of that level (host arrays,
 * copied by dg_init).  Leaves must tile the box and be 2:1 balanced across
 * faces. */
typedef struct {
  int32_t kind;
  int32_t n[3];
  double box[3];
  int64_t nleaves;
  const int8_t* level; /* [host] */
  const int32_t* ijk;  /* [host] */
} dg_mesh;

/* Limiter statistics of one dg_limit call.  n_floor counts the cell-average
 * floors that fired (density and pressure separately); injected_mass and
 * injected_energy are what they added, summed over cells in a fixed order
 * (bitwise reproducible); n_ch_violation counts the time-step evaluations of
 * the call whose fixed c_h was below twice the largest signal speed. */
typedef struct {
  int64_t n_tvb_triggered, n_mlp_flagged, n_fallback, n_pos_scaled, n_floor, n_ch_violation;
  double injected_mass, injected_energy, max_signal, ch;
} dg_limit_stats;

/* Create a handle: builds the tables (Gauss-Legendre rules, Legendre and LDF
 * bases, face tables), the face lists and the workspaces on the current HIP
 * device.  hip_stream: a hipStream_t (NULL = default stream). */
int dg_init(const dg_params* p /*[host]*/, const dg_mesh* m /*[host]*/, void* hip_stream,
            dg_handle* out /*[host]*/);

/* Sizes of the state array: nmodes rows of ld elements, ncells of them used. */
int dg_layout(dg_handle h, int64_t* nmodes, int64_t* ncells, int64_t* ld);

/* Reference coordinates of the (d+3)^dim projection points used by
 * dg_project (Sec. 5.2.1 rule), point-major: xi[p*dim + a]; synchronous. */
int dg_proj_points(dg_handle h, double* xi /*[host] or NULL*/, int64_t* npts /*[host]*/);

/* L2 projection of pointwise primitive values onto the modal state
 * (w_l = M_l^-1 sum_q w_q u(x_q) . phi_l(xi_q)).  prim: device FP64 array
 * [9][ncell][npts] holding (rho, v1, v2, v3, p, B1, B2, B3, psi) at the
 * points of dg_proj_points for cells cell0 .. cell0+ncell-1; writes those
 * columns of w.  Async. */
int dg_project(dg_handle h, const double* prim, int64_t cell0, int64_t ncell, void* w);

/* Conserved state at the points of dg_proj_points (the (d+3)^dim Gauss
 * rule with which eq. lp_norm measures errors) for cells cell0 ..
 * cell0+ncell-1: out is a device FP64 array [nvar][npts][ncell] (nvar = 9
 * for GLM, 8 for Powell; variables rho, m1, m2, m3, E, B1, B2, B3, psi),
 * evaluated in FP64 from the weights of w (of either precision).  DG_EINVAL
 * for a null pointer or a cell range outside the grid.  Async. */
int dg_nodal(dg_handle h, const void* w, int64_t cell0, int64_t ncell, double* out);

/* Dynamic refinement (Sec. 4.4; GLM handles, Legendre basis; DG_EUNSUPPORTED
 * for Powell).  fields: bit v set monitors conserved variable v (0 rho,
 * 1-3 m, 4 E, 5-7 B, 8 psi); the paper refines on rho and B (0xE1).
 *
 * dg_amr_indicator: S[cell] (device FP64, ncells) = the largest smoothness
 * indicator S_alpha(u) = sum_{k=1}^{d} 2^(2k-1) int (d^k u/dxi_alpha^k)^2 over
 * the monitored fields and the directions.  Async. */
int dg_amr_indicator(dg_handle h, const void* w, uint32_t fields, double* S);

/* dg_amr_plan: one regrid decision for the state w.  A leaf is split when its
 * indicator exceeds 2 s_tilde and its level is below max_level; a complete
 * group of 2^dim sibling leaves none of which is split merges into its parent
 * when the parent's polynomial (the L2 restriction of the children) has an
 * indicator below s_tilde / 2.  A merge that would leave a face neighbour two
 * levels finer is dropped; other 2:1 violations are removed by refinement.
 * The handle keeps the plan (new leaves in Morton order and the transfer
 * map); *n_new (host) receives the number of new leaves.  A uniform grid's
 * leaves are its level-0 cells.  Synchronous. */
int dg_amr_plan(dg_handle h, const void* w, uint32_t fields, double s_tilde, int32_t max_level, int64_t* n_new);

/* dg_amr_leaves: the planned leaves, level[n_new] and ijk[n_new][3] (host,
 * caller-allocated), the input of a new handle's dg_mesh (DG_MESH_OCTREE,
 * same base grid). */
int dg_amr_leaves(dg_handle h, int8_t* level /*[host]*/, int32_t* ijk /*[host]*/);

/* dg_amr_transfer: weights of the new leaves from the old state w_old: kept
 * leaves copied, split leaves prolongated (L2 projection of the parent's
 * polynomial onto each child, through every level of a split), merged groups
 * restricted (L2 projection of the children onto the parent); exact for the
 * polynomial space and conservative.  h_new must have been created from
 * dg_amr_leaves of h_old's plan with the same dimension, degree, scheme and
 * precision (DG_EINVAL otherwise).  Waits for h_old's stream, runs on
 * h_new's; synchronous. */
int dg_amr_transfer(dg_handle h_old, const void* w_old, dg_handle h_new, void* w_new);

/* Time step of the state w (eq. cfl; Powell cap eq. powell_dt; GLM c_h and
 * kappa = c_h^2 / c_p^2 of Sec. 4.1.5).  Synchronous; outputs on the host.
 * DG_ENONFINITE if the state's signal speed is not finite; DG_ECH (outputs
 * valid) if a fixed c_h is below twice the largest signal speed. */
int dg_dt(dg_handle h, const void* w, double* dt, double* ch, double* kappa);

/* dwdt = M^-1 R(w): the semi-discrete right-hand side of eq. wdot including
 * the Powell face terms or the GLM flux and damping source (c_h, kappa
 * given).  w and dwdt: [nmodes][ld] device arrays (distinct).  Async. */
int dg_rhs(dg_handle h, const void* w, void* dwdt, double ch, double kappa);

/* The same right-hand side as dg_rhs (same kernels, same result) for
 * callers that cannot allocate device memory at call time: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Its
 * workspace (face fluxes, Powell normal-field jumps, device scalars) lives in
 * one 32 MiB device array of the library per device, whose address is
 * resolved at dg_init; the call allocates nothing.  DG_EINVAL (no device
 * work) if the mesh needs more than 32 MiB of workspace (3-D degree 3 FP64:
 * about 9,700 cells; 2-D degree 1 FP64: about 116,000 cells) or if the
 * current device is not the one the handle was created on.  All calls on one
 * device share that array: calls that overlap on one device (two streams,
 * two threads) race and must be ordered by the caller.  Async. */
int dg_rhs_noalloc(dg_handle h, const void* w, void* dwdt, double ch, double kappa);

/* Apply the limiters selected in dg_params.limiter to w in place (slope
 * limiter first, then positivity).  stats == NULL: async; otherwise the
 * stream is synchronised, stats filled, the limited state scanned for
 * non-finite weights (DG_ENONFINITE, state left as computed) and DG_ECH
 * returned (state valid) if the c_h check of the call failed. */
int dg_limit(dg_handle h, void* w, dg_limit_stats* stats /*[host] or NULL*/);

/* Advance w by nsteps steps of the selected SSP-RK scheme (Sec. 3.6); dt, c_h and kappa are
 * computed on the device from the state at the start of each step and the
 * selected limiters run after every stage (Sec. 4.3: before any state is
 * evaluated at quadrature points again).  Limiting the initial state is the
 * caller's dg_limit call.  t (host, may be NULL) is advanced by the sum of
 * the steps' dt; a non-NULL t synchronises and checks the call: DG_ENONFINITE
 * if a non-finite value met a time-step reduction or is left in the final
 * state (state left as computed), else DG_ECH (state valid) if a fixed c_h
 * was below twice the largest signal speed at some step. */
int dg_step(dg_handle h, void* w, int32_t nsteps, double* t /*[host] in/out*/);

/* Learned troubled-cell indicator (GLM on uniform grids).  The network maps
 * 256 features of a cell (its 9 x 20 modal weights and its 6 face
 * neighbours' mean differences, each divided by s_v = |mean_v| + sigma_v,
 * zero padded) through 256 -> 64 -> 64 -> 64 -> 1 (GELU, sigmoid) to the
 * probability that the plain TVB detector (Sec. 4.2) fires.  With
 * DG_LIM_LEARNED set, dg_limit / dg_step skip the slope limiter on cells with
 * probability < mlp_lo, use the plain detector on the band [mlp_lo, mlp_hi)
 * ("fallback") and count cells >= mlp_hi as flagged.  Matrix products run on
 * BF16 matrix cores with FP32 accumulation; masters and Adam state are FP32.
 *
 * Parameters (public FP32 layout, 24833 values): for each layer W[in][out]
 * row-major then b[out], layers 256x64, 64x64, 64x64, 64x1. */

/* Feature scales from a state (normally the initial one): sigma_v = RMS over
 * cells of the cell means of variable v, floored at 1e-2 of the largest;
 * kept in the handle and copied to sigma (host, 9, may be NULL).  Sync. */
int dg_mlp_scale(dg_handle h, const void* w, double* sigma /*[host] or NULL*/);
/* Install parameters (params == NULL: W ~ U(+-1/sqrt(in)) from seed, b = 0)
 * and feature scales (sigma == NULL keeps those of dg_mlp_scale).  Sync. */
int dg_mlp_set(dg_handle h, const float* params /*[host] or NULL*/, const double* sigma /*[host] 9 or NULL*/,
               uint64_t seed);
/* Copy the current parameters to params (host, 24833 floats).  Synchronous. */
int dg_mlp_get(dg_handle h, float* params /*[host]*/);
/* Features of every cell of w into X (device BF16 [ncells][256]).  Async. */
int dg_mlp_features(dg_handle h, const void* w, void* X);
/* Plain TVB detector decisions of every cell of w into y (device FP32, 1/0),
 * c_h from the time-step rule of w; w is not modified.  Async. */
int dg_mlp_labels(dg_handle h, const void* w, float* y);
/* Record (features, label) pairs of the pre-limiter state of every later
 * dg_limit call and of every stage of later dg_step calls: positives kept with probability q_pos, negatives with
 * q_neg (counter-based hash of cell, stage and seed), rows appended to X
 * (device BF16 [cap][256]) and y (device FP32 [cap]) through the device
 * counter (uint64, caller-cleared; it may exceed cap: rows beyond cap are
 * dropped).  X == NULL stops recording. */
int dg_mlp_record(dg_handle h, void* X, float* y, unsigned long long* counter, int64_t cap, double q_pos,
                  double q_neg, uint64_t seed);
/* Network output for nrows feature rows (device X BF16 [nrows][256]) into
 * prob (device FP32 [nrows]).  Async. */
int dg_mlp_forward(dg_handle h, const void* X, int64_t nrows, float* prob);
/* Mean binary cross-entropy loss and its gradient w.r.t. the parameters
 * (public layout, host) for one batch of nrows rows (device X, y).  Sync. */
int dg_mlp_grad(dg_handle h, const void* X, const float* y, int64_t nrows, float* grads /*[host]*/,
                float* loss /*[host] or NULL*/);
/* Adam training (beta 0.9 / 0.999, eps 1e-8) for `epochs` passes over nrows
 * rows in shuffled mini-batches of `batch`; per-epoch mean losses to
 * losses (host, may be NULL).  Synchronous. */
int dg_mlp_train(dg_handle h, const void* X, const float* y, int64_t nrows, int32_t batch, int32_t epochs, float lr,
                 uint64_t seed, float* losses /*[host]*/);

/* Measurement hook: launch one kernel of the step `reps` times back to back
 * on the handle's stream between two HIP events and return the mean time per
 * launch in ms.  which: 0 face flux kernel, 1 cell (volume + surface + stage
 * update) kernel in the step's mix of forms (rep i: the first stage's form
 * if i % 3 == 0, else the later stages'), 2 time-step reduction, 3 limiter
 * sequence.  Reads w; writes
 * only the handle's workspaces.  Synchronous. */
int dg_time_kernel(dg_handle h, const void* w, int32_t which, int32_t reps, double* ms /*[host]*/);

/* Autotuner of the kernel schedule.  A schedule is cell variant + 16 x face
 * variant.  Cell variants: 0-3 LDS-tiled kernels (cells per block x threads
 * per block: 16x256, 32x256, 32x512, 64x512); GLM: 4-7 matrix-core kernel (4
 * or 2 waves of 16 cells per block, 6-7 with batched operand loads), 8-9
 * batched and persistent with the tables in LDS; Powell: 6 the persistent
 * matrix-core kernel with the LDF basis (tables in LDS; the plain one where
 * they do not fit), 8-9 the plain one with 4 or 2 waves per block (4, 5 and
 * 7 are not built).  Face variants: 0 LDS-staged; 1-3 matrix-core (GLM; 1 for
 * Powell; they also select the matrix-core max-signal-speed reduction of the
 * time step): 1 four waves per block, 2 one wave per block, 3 one wave per
 * block with the right traces in LDS and one face point solved at a time
 * (two waves per SIMD); on octree grids 1-3 run the matrix-core sub-face
 * kernel.  The matrix-core face kernels hand the cell kernels face moments
 * (the projections of the face values on the polynomials of degree <= d in
 * the face coordinates, the only part of a face flux the weak form uses) on
 * GLM grids (uniform and octree) and for the 3-D Powell scheme with the
 * cell-mean q-dagger; the LDS kernels hand over face-point values; so a
 * schedule pairs cell 0-3 with face 0 or a matrix-core cell variant with a
 * matrix-core face variant (2-D Powell: any pair).  *variant >= 0 forces that
 * schedule (DG_EINVAL if it is not built for this configuration or pairs the
 * two layouts); *variant < 0 times every built cell variant and every face
 * variant on the state w (read only; the handle's workspaces are written)
 * and keeps the fastest valid pair.  Before any call the schedule is 6 + 16
 * (GLM) or 8 + 16 (Powell).  cache_path (may be NULL): a JSON file of earlier
 * choices keyed by precision, dimension, degree, divergence scheme, the
 * Powell q-dagger form, cell count and, on octrees, the leaves per level and
 * the face count; an entry found there is used without timing and new
 * choices are appended.  On return *variant holds the schedule in use.
 * Synchronous. */
int dg_autotune(dg_handle h, const void* w, const char* cache_path, int32_t* variant /*[host] in/out*/);

const char* dg_last_error(dg_handle h);
void dg_destroy(dg_handle h);

#ifdef __cplusplus
}
#endif

#endif /* DGMHD_DG_H */
