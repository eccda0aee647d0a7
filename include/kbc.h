/*
 * kbc.h -- C ABI of libkbc, the MI355X (gfx950) implementation of the D2Q9
 * lattice Boltzmann stream-and-collide step with the entropic multi-relaxation
 * (KBC) collision of Boesch, Chikatamarla and Karlin, "Entropic
 * Multi-Relaxation Models for Simulation of Fluid Turbulence"
 * (arXiv:1507.02509), and the LBGK baseline.
 *
 * Model (paper sections cited per entry point):
 *   f_i(x + v_i, t + 1) = f_i' = (1 - beta) f_i(x, t) + beta f_i^mirr(x, t)
 *                                                               eq. (Egeneral)
 *   LBGK: f^mirr = 2 feq - f                                    eq. (LBGKmirr)
 *   KBC:  f^mirr = k + [2 s^eq - s] + [gamma h^eq + (1 - gamma) h]
 *                                                            eq. (ksh-mirror)
 *         with the moment groups of Table kbc_moment_grouping and
 *         gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>      eq. (result21)
 *   feq: second-order polynomial equilibrium                       eq. (Eq)
 *   nu = cs2 (1/(2 beta) - 1/2), cs2 = 1/3                   eq. (viscosity)
 *
 * Lattice conventions:
 *   velocity order i = 0..8: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *   (-1,-1) (1,-1); weights W = 4/9, 1/9 (x4), 1/36 (x4); periodic in x and y
 *   (a slab of a domain split in y takes its rows beyond y = 0 .. ny - 1 from
 *   halo buffers instead: lbm_set_halo).
 *
 * Storage (device memory owned by the caller, e.g. torch tensors):
 *   a population buffer holds, for every lattice row y, the nine population
 *   rows of `pitch` elements one after another ([ny][9][pitch], x fastest):
 *   element (i, y, x) at offset (9 * y + i) * pitch + x.  The stored value
 *   is the deviation g_i = f_i - W_i rho0 in the form's storage type:
 *     LBM_F16DEV_F32: binary16 holding g_i * 2^s_i (s = 1 for i = 0, 3 for the
 *                     axis velocities, 5 for the diagonals), FP32 arithmetic;
 *     LBM_F32DEV_F32: binary32 g_i, FP32 arithmetic;
 *     LBM_F64:        binary64 g_i, FP64 arithmetic.
 *   The step is a fused pull: each node gathers buf_i(x - v_i), collides and
 *   writes buf'_i(x).  Hence the buffer after n steps holds the post-collision
 *   state of step n-1 at its source node, and the pre-collision state the
 *   paper calls f(x, t = n) is f_i(x) = buf_i(x - v_i) + W_i rho0.  Every entry
 *   point that reads or writes "the state" uses f(x, t = n) in that sense.
 *
 * Macroscopic fields (rho, u_x, u_y, gamma, gradients) are dense FP64 device
 * arrays [ny][nx], x fastest.
 *
 * Calls are stream-ordered on params.stream (a hipStream_t; NULL = the null
 * stream) and return LBM_OK (0) or a negative LBM_E* code; lbm_last_error()
 * then holds a message for the calling thread.  Argument checks run before
 * any HIP call.  No entry point synchronises the stream unless it says so.
 */
#ifndef KBC_H
#define KBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,        /* invalid argument */
    LBM_EHIP = -2,          /* a HIP runtime call failed */
    LBM_ENOMEM = -3,        /* device or host allocation failed */
    LBM_ENONFINITE = -4,    /* not returned by the library: the code of a non-finite state
                               that a caller finds with lbm_diagnostics (the Python
                               binding's checked run raises it) */
    LBM_EUNSUPPORTED = -5,  /* valid but not implemented combination */
    LBM_ESYNC = -6          /* a persistent ensemble launch gave up waiting at its grid
                               barrier (lbm_ensemble_check): the members' states are invalid */
};

/* collision: LBGK eq. (LBGKmirr) or KBC eq. (ksh-mirror) */
typedef enum { LBM_LBGK = 0, LBM_KBC = 1 } lbm_collision;
/* moment grouping of Table kbc_moment_grouping */
typedef enum { LBM_KBC_A = 0, LBM_KBC_B = 1, LBM_KBC_C = 2, LBM_KBC_D = 3 } lbm_variant;
/* storage / arithmetic form (see "Storage" above) */
typedef enum { LBM_F16DEV_F32 = 0, LBM_F32DEV_F32 = 1, LBM_F64 = 2 } lbm_form;
/* stabiliser: gamma* of eq. (result21) with the denominator guard, a fixed
 * value (gamma_fixed; 2 gives LBGK, 1/beta the regularised model), or the
 * root of eq. (result1) by Newton iteration from gamma* (guarded nodes keep
 * gamma = 2; the iteration stops when a logarithm's argument would leave
 * (0, inf), after a step below 1e-15 (FP64) or 5e-7 (FP32 arithmetic)
 * relative, after a step that is not at most half the previous one (rounding
 * noise reached), or after 100 / 20 steps).  LBM_GAMMA_EXACT runs in the step,
 * moments, diagnostics, the ensemble and the adjoint (which differentiates the
 * root by the implicit function theorem, holding gamma where the iteration
 * stopped without a root). */
typedef enum { LBM_GAMMA_ESTIMATE = 0, LBM_GAMMA_FIXED = 1, LBM_GAMMA_EXACT = 2 } lbm_gamma_mode;
/* initial populations: equilibrium eq. (Eq); Grad's approximation eq. (Grad)
 * with Pi = Pi^eq + Pi^(1) (eqs. Peq, P1AC) and velocity gradients from
 * second-order central differences, or from the caller */
typedef enum { LBM_INIT_EQ = 0, LBM_INIT_GRAD_CD = 1, LBM_INIT_GRAD_GIVEN = 2 } lbm_init_mode;

typedef struct {
    int32_t nx, ny;        /* lattice size, each in [3, 2^28] (see "Size limits") */
    double beta;           /* relaxation parameter, 0 < beta <= 1 */
    double rho0;           /* reference density of the deviation storage (> 0, usually 1) */
    int32_t collision;     /* lbm_collision */
    int32_t variant;       /* lbm_variant (ignored for LBGK) */
    int32_t form;          /* lbm_form */
    int32_t gamma_mode;    /* lbm_gamma_mode */
    double gamma_guard;    /* gamma = 2 where <dh|dh> <= gamma_guard * <ds|ds> (>= 0; default 1e-12) */
    double gamma_fixed;    /* stabiliser for LBM_GAMMA_FIXED */
    void* stream;          /* hipStream_t all work is ordered on */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Diagnostics of the state f(x, t = n) (section "Decaying Two-Dimensional
 * Turbulence" statistics): totals, spatial means and standard deviations of
 * e = |u|^2/2, z = omega^2/2 and p = |grad omega|^2/2 (omega and its gradient
 * by second-order central differences), mean entropy per node eq. (S), mean
 * and standard deviation of gamma, node counts with a non-finite population or
 * a non-positive equilibrium population.  Sums are accumulated in FP64. */
typedef struct {
    double mass, jx, jy;
    double E, E_std, Z, Z_std, P, P_std;
    double S, gamma, gamma_std;
    double n_nonfinite, n_feq_nonpos;
    double rho_std;
    double reserved;
} lbm_diag;

/* Size limits.  Each side is at most 2^28 nodes, so that a node's byte
 * offset within a population row is a 32-bit value.  A kernel launch holds at
 * most 2^32 - 1 work-items (the grid size of a dispatch is 32-bit); a call
 * whose launch would need more returns LBM_EUNSUPPORTED without making that
 * launch (every launch of lbm_step has the same grid, so it enqueues
 * nothing; lbm_adjoint_rollout may have enqueued earlier, smaller ones).
 * Work-items per node: 1 / rows-per-thread for the single step (1/4 with the
 * FP16 default 256 x 4 tile, 1 with the FP32 and FP64 defaults), 4 / rows for
 * the fused step (1/4 with 16-row tiles, 1/2 with FP64's 8), 1 / (rows per
 * thread) for the adjoint step (1/2 for FP32 and FP16 lattices of at least
 * 8192 tiles of 128 x 4 nodes, else 1), plus 1 for the forward step that
 * lbm_adjoint_rollout combines with it, and 1 for lbm_adjoint_init.  So every
 * lattice whose buffers fit the device's memory steps in the default
 * configuration (the largest: about 2^32 nodes in FP16, two 77 GB population
 * buffers).  Offsets of rows within buffers are 64-bit everywhere. */

/* Smallest legal pitch (elements) for nx in form f: nx rounded up to 64.
 * Returns 0 for invalid arguments (nx outside [1, 2^28], unknown form). */
size_t lbm_required_pitch(int32_t nx, int32_t form);

/* Bytes of one population buffer: 9 * ny * pitch * sizeof(storage type). */
size_t lbm_buffer_bytes(int32_t nx, int32_t ny, int32_t form);

/* Create a context over two caller-owned population buffers (buf_a, buf_b,
 * each lbm_buffer_bytes; they must not overlap; pitch_elems >= the required
 * pitch and a multiple of 64) and write the initial state into buf_a, per
 * `mode` from rho (NULL: uniform rho0), ux, uy and, for LBM_INIT_GRAD_GIVEN,
 * grad[4][ny][nx] = (d_x u_x, d_y u_x, d_x u_y, d_y u_y) (section
 * "Green-Taylor Vortex Flow", eq. (Grad); central differences as in the
 * turbulence section).  The macroscopic inputs are read before the call's
 * work completes on the stream; keep them alive until then.  *out receives
 * the context; the caller frees it with lbm_free. */
int lbm_init(lbm_ctx** out, const lbm_params* p, void* buf_a, void* buf_b, size_t pitch_elems,
             const double* rho, const double* ux, const double* uy, const double* grad,
             int32_t mode);

/* Advance nsteps >= 0 time steps of eq. (Egeneral).  By default every pair of
 * steps is one launch (two fused pull-stream + collide steps, the first step's
 * result kept in LDS; see lbm_set_fusion) and an odd remainder one single-step
 * launch; each launch reads one buffer and writes the other.  Enqueues only;
 * does no value checks (see lbm_diagnostics).  A slab (lbm_set_halo) takes
 * at most one launch's steps per call. */
int lbm_step(lbm_ctx* c, int32_t nsteps);

/* Density, velocity and (optionally) the stabiliser gamma the next collision
 * would use, of f(x, t = n).  Each output is a dense FP64 device array
 * [ny][nx] or NULL. */
int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* gamma);

/* Export / import f(x, t = n) as full FP64 populations [9][ny][nx] (device). */
int lbm_get_populations(lbm_ctx* c, double* f);
int lbm_set_populations(lbm_ctx* c, const double* f);

/* Diagnostics of f(x, t = n) into *out (host).  Synchronises the stream. */
int lbm_diagnostics(lbm_ctx* c, lbm_diag* out);

/* Steps taken since lbm_init (or the last lbm_set_step). */
int64_t lbm_step_count(const lbm_ctx* c);
int lbm_set_step(lbm_ctx* c, int64_t n);

/* Shell-summed spectra of f(x, t = n) on a square lattice (N x N), section
 * "Decaying Two-Dimensional Turbulence": with u_hat the unnormalised discrete
 * Fourier transform of each velocity component and integer wavevectors k,
 * E_k[s] = sum over round(|k|) = s of (|ux_hat|^2 + |uy_hat|^2) / (2 N^4)
 * (so sum_s E_k[s] = E = <|u|^2> / 2 when kmax covers every shell) and
 * Z_k[s] = the same sum weighted by (2 pi |k| / N)^2 (enstrophy with the
 * exact derivative, so it differs from the diagnostics' central-difference
 * Z at high k).  E_k and Z_k are device arrays of kmax + 1 doubles (either may
 * be NULL); shells above kmax are dropped.  Shell sums use atomic adds:
 * repeatable to rounding, not bit for bit.  Allocates 2 N^2 + 4 N (N/2 + 1)
 * doubles of scratch and an FFT plan on first use (kept until lbm_free).
 * LBM_EUNSUPPORTED for non-square lattices. */
int lbm_spectra(lbm_ctx* c, int32_t kmax, double* E_k, double* Z_k);

/* Device pointer of the buffer holding the current state and of the other one. */
void* lbm_state_buffer(const lbm_ctx* c);
void* lbm_work_buffer(const lbm_ctx* c);

/* Workgroup tile of the step kernel: `width` in {64, 128, 256} nodes by
 * (256 / width) * rows_per_thread rows, rows_per_thread in {1, 2, 4}
 * (default per form: 256 x 4 for FP16, 256 x 1 for FP32, 128 x 2 for FP64);
 * flags: LBM_TILE_NONTEMPORAL writes the new state with non-temporal stores
 * (by default on, except for lattices whose two buffers together take between
 * 40 MB (80 MB for FP16) and 256 MiB: the last-level cache then holds the new
 * state for the next step).  The flag applies to the fused launch too.  A
 * tuning knob only: results are bitwise identical for every setting. */
#define LBM_TILE_NONTEMPORAL 1
int lbm_set_tile(lbm_ctx* c, int32_t width, int32_t rows_per_thread, int32_t flags);
/* The current tile and flags (any pointer may be NULL); LBM_EINVAL for a
 * NULL ctx. */
int lbm_get_tile(const lbm_ctx* c, int32_t* width, int32_t* rows_per_thread, int32_t* flags);

/* Time steps per kernel launch in lbm_step: 1, or 2 (temporal blocking: each
 * workgroup runs the first step on its 64 x `rows` tile plus a one-node ring,
 * keeps that state in LDS and runs the second step from it, so a pair of
 * steps reads and writes the state once).  `rows` in {8, 16, 24, 32} sets the
 * fused tile height (0 keeps the current one; 32 is LBM_EUNSUPPORTED for
 * FP64, whose tile would not fit the LDS of a CU).  Defaults: 2 steps with 16
 * rows for FP32 and FP16 (8 rows when the lattice has fewer than 1792 tiles
 * of 16 rows), 8 rows for FP64.  Odd
 * remainders run as single steps.  Results are bitwise identical for every
 * setting; the non-temporal flag of lbm_set_tile applies to the fused launch
 * too.  LBM_EINVAL for other values.  lbm_get_fusion returns the steps per
 * launch and stores the fused tile height in *rows when rows is not NULL
 * (-1 for a NULL ctx). */
int lbm_set_fusion(lbm_ctx* c, int32_t steps_per_launch, int32_t rows);
int lbm_get_fusion(const lbm_ctx* c, int32_t* rows);

/* Slab mode: the context's lattice is one slab of a larger domain split in y
 * (one slab per GPU), periodic in x only.  The step's pull (eq. Egeneral:
 * population i arrives from x - v_i) then reads the two rows on each side of
 * the slab from the neighbouring slabs instead of wrapping onto itself.
 * `lo` holds rows -2 and -1, `hi` rows ny and ny + 1, of the state at the
 * current time, each laid out [2][9][pitch] exactly like the state ([row][population]
 * [x], storage form, the context's pitch): device memory owned by the caller,
 * read by every following lbm_step until the next lbm_set_halo.  Both NULL
 * returns the context to periodic rows (the default); one NULL is
 * LBM_EINVAL.  While a halo is set:
 *   - lbm_step(c, n) takes n <= steps per launch (lbm_set_fusion): one
 *     launch, since the halo holds the neighbours' rows at one time only
 *     (two rows: enough for two fused steps); the caller refreshes the halo
 *     between calls.  Larger n is LBM_EINVAL.
 *   - fused tiles are 8 or 16 rows (LBM_EUNSUPPORTED otherwise) and graph
 *     replay is off (lbm_set_graph with chunk > 0 is LBM_EINVAL);
 *   - the context cannot join an ensemble (and lbm_set_halo is LBM_EINVAL
 *     while it is in one).
 * Only lbm_step reads the halo: moments, diagnostics, spectra and the
 * adjoint still treat the slab as periodic in y.  Results equal, bit for bit,
 * the rows of the whole domain stepped as one periodic lattice. */
int lbm_set_halo(lbm_ctx* c, const void* lo, const void* hi);

/* The rows a neighbouring slab needs as its halo, from the current state:
 * rows 0 and 1 into lo_rows (the halo `hi` of the slab below, in -y) and rows
 * ny - 2 and ny - 1 into hi_rows (the halo `lo` of the slab above), each
 * [2][9][pitch] in the storage form.  Two device-to-device copies enqueued on
 * params.stream; both pointers are device memory the caller owns (in a
 * multi-GPU run, the send buffers of the halo exchange). */
int lbm_get_edge_rows(lbm_ctx* c, void* lo_rows, void* hi_rows);

/* HIP graph replay for launch-bound (small) lattices.  With chunk >= 2,
 * lbm_step runs every whole chunk of `chunk` steps as one hipGraphLaunch on
 * params.stream and the remainder as direct launches.  The graph of a chunk
 * is captured on first use, once for each of the two buffers that can hold
 * the start state: the same kernel launches lbm_step makes directly are
 * recorded on a private stream of the context (created then, default
 * priority; nothing runs during the capture) and instantiated.  The graphs
 * hold kernel nodes only, so results are bitwise identical to direct
 * launches.  chunk = 0 (the default) launches every kernel directly.
 * Measured on MI355X, replays do not beat direct launches from one stream
 * (64^2 to 1024^2, 2000 steps: within -5 % to +4 %): a small lattice's step
 * is bound by the latency of its few workgroups, not by launch submission.
 * lbm_set_fusion, lbm_set_tile and lbm_set_beta (with a new value) discard
 * the captured graphs, synchronising the stream first; lbm_free releases them
 * and the private stream.  Errors: LBM_EINVAL for chunk 1, < 0 or > 2^20;
 * LBM_EHIP if capture, instantiation or launch fails (the step counter and
 * state then stand after the last whole chunk that was launched).
 * lbm_get_graph returns the chunk (-1 for a NULL ctx). */
int lbm_set_graph(lbm_ctx* c, int32_t chunk);
int lbm_get_graph(const lbm_ctx* c);

/* Replace beta (e.g. between rollouts); other parameters are fixed per ctx.
 * An ensemble holding the context picks the new value up at its next
 * lbm_ensemble_step. */
int lbm_set_beta(lbm_ctx* c, double beta);

/* Release the context and the scratch memory it allocated (never the
 * caller's buffers).  Synchronises the stream.  NULL is accepted.
 * LBM_EINVAL (and nothing is released) while the context is a member of a
 * live ensemble: free the ensemble first. */
int lbm_free(lbm_ctx* c);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

/* ------------------------------------------------------------------ adjoint
 * Gradients of a loss of the final state with respect to the initial
 * velocity and beta (discrete adjoint of eq. (Egeneral) with the collision of
 * this context, gamma(f) of eq. (result21) differentiated; constant where the
 * guard selects gamma = 2).  An adjoint buffer holds dL/df for every node and
 * velocity, [ny][9][pitch] in the form's arithmetic type (float for the two
 * deviation forms, double for LBM_F64), NOT shifted: element (i, y, x) is
 * dL/df_i(x, y).  `state` arguments are population buffers in this context's
 * layout holding f(x, t = n) (e.g. checkpoints copied from lbm_state_buffer).
 * Derivatives of beta are added (+=) to the device double *dbeta when it is
 * not NULL, in a fixed summation order (bitwise reproducible). */

/* How the adjoint step treats the stabiliser: LBM_ADJ_GAMMA_FULL (default)
 * differentiates gamma(f) of eq. (result21); LBM_ADJ_GAMMA_FROZEN holds it at
 * the forward value (derivative of the map with gamma a per-node constant).
 * The exact derivative of gamma* carries factors 1 / <dh|dh>, large where dh
 * is small but above the guard, so over long turbulent rollouts the full
 * adjoint can grow far beyond the finite-difference slope of the loss. */
#define LBM_ADJ_GAMMA_FULL 0
#define LBM_ADJ_GAMMA_FROZEN 1
int lbm_set_adjoint_gamma(lbm_ctx* c, int32_t mode);

/* Bytes of one adjoint buffer. */
size_t lbm_adjoint_bytes(int32_t nx, int32_t ny, int32_t form);

/* One forward step from population buffer src into dst (neither is the
 * context's own state unless the caller passes it); used to recompute states
 * between checkpoints. */
int lbm_step_buffers(lbm_ctx* c, const void* src, void* dst);

/* lam = dL/df for a loss of the moments of `state`: given dL/drho, dL/du_x,
 * dL/du_y (dense FP64 [ny][nx] device arrays, each nullable = 0),
 * lam_i(x) = dL/drho + (dL/du_x (v_xi - u_x) + dL/du_y (v_yi - u_y)) / rho. */
int lbm_adjoint_seed(lbm_ctx* c, const void* state, const double* dL_drho, const double* dL_dux,
                     const double* dL_duy, void* lam);

/* One adjoint step: with state = f^n and lam_in = dL/df^{n+1}, writes
 * lam_out = dL/df^n and adds the step's dL/dbeta to *dbeta. */
int lbm_adjoint_step(lbm_ctx* c, const void* state, const void* lam_in, void* lam_out, double* dbeta);

/* lbm_adjoint_step of a slab of a domain split in y (see lbm_set_halo): the
 * adjoint step reads the state f^n at x - v_i and the incoming adjoint at
 * x + v_i, so rows -1 and ny of both come from the neighbouring slabs.
 * state_lo / state_hi: rows -2, -1 and ny, ny + 1 of `state`, [2][9][pitch]
 * in the storage form (the layout of lbm_set_halo; the step reads rows -1
 * and ny); lam_lo / lam_hi: the same rows of lam_in, [2][9][pitch] of the
 * adjoint type.  Device memory owned by the caller, read during this call's
 * work only.  lambda^n equals, bit for bit, the rows of the whole domain's
 * adjoint step; *dbeta receives this slab's share of dL/dbeta (the whole
 * domain's is the sum over slabs, equal up to summation order). */
int lbm_adjoint_step_slab(lbm_ctx* c, const void* state, const void* state_lo, const void* state_hi,
                          const void* lam_in, const void* lam_lo, const void* lam_hi, void* lam_out, double* dbeta);

/* lbm_adjoint_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results, bit for bit, but the step's
 * per-workgroup dL/dbeta partials live in a fixed device array of
 * LBM_NOALLOC_SCRATCH_DOUBLES doubles (8 MiB; one per GPU the library runs
 * on, held until the process ends) instead of scratch the context allocates,
 * and the call allocates nothing (no hipMalloc, hipFree or allocating
 * library call).  Limit: the step needs adjoint partials plus one slice of
 * doubles, about one per 512 nodes for FP32/FP16 lattices of at least 8192
 * tiles of 128 x 4 (so up to about 5.3e8 nodes, e.g. 16384 x 32768) and one
 * per 256 nodes otherwise (FP64 up to just under 16384 x 16384); larger
 * lattices return LBM_EINVAL before any launch.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind: nothing in it needs to
 * start at zero (a call writes every value before reading it), but calls
 * that overlap on one GPU (two streams, two host threads) race on it.  The
 * context's device must be current (LBM_EINVAL otherwise); the array's
 * address is looked up on the first call on each device. */
#define LBM_NOALLOC_SCRATCH_DOUBLES (1 << 20)
int lbm_adjoint_step_noalloc(lbm_ctx* c, const void* state, const void* lam_in, void* lam_out, double* dbeta);

/* One checkpoint segment of the backward pass: from state0 = f^s, recompute
 * f^{s+1} .. f^{s+k-1} into slots[0 .. k-2] (population buffers of this
 * context's layout), then run k adjoint steps from lam_in = dL/df^{s+k} down
 * to dL/df^s, adding the steps' dL/dbeta to *dbeta.  The two adjoint buffers
 * are used in turn; *which receives 0 if dL/df^s ended in lam_in and 1 if in
 * lam_out. */
int lbm_adjoint_segment(lbm_ctx* c, const void* state0, void* const* slots, int32_t k, void* lam_in,
                        void* lam_out, double* dbeta, int32_t* which);

/* The whole backward pass of a checkpointed rollout of nsteps steps.
 * ckpts[j] = f^{j seglen} for j = 0 .. ceil(nsteps / seglen) - 1 (population
 * buffers of this context's layout).  Segments run from last to first, their
 * states f^{s+1} .. f^{s+k-1} held in one of two slot sets (slots_a, slots_b:
 * seglen - 1 distinct buffers each, alternating between segments).  Each
 * launch runs one adjoint step of segment j and, in the same grid, one
 * forward step recomputing a state of segment j - 1 into the other set, so
 * the recomputation costs no launches of its own and the two fill the chip
 * together on small lattices.  The result is bitwise that of calling
 * lbm_adjoint_segment for every segment in turn.  lam_in holds dL/df^{nsteps}
 * on entry; *which receives 0 if dL/df^0 ended in lam_in, 1 if in lam_out;
 * the steps' dL/dbeta are added to *dbeta (nullable).  Stream-ordered on the
 * context's stream; owns no buffer. */
int lbm_adjoint_rollout(lbm_ctx* c, const void* const* ckpts, int32_t nsteps, int32_t seglen,
                        void* const* slots_a, void* const* slots_b, void* lam_in, void* lam_out, double* dbeta,
                        int32_t* which);

/* Adjoint of lbm_init for modes LBM_INIT_EQ and LBM_INIT_GRAD_CD: from
 * lam0 = dL/df^0 and the initial fields (rho nullable = rho0), writes
 * dL/du_x, dL/du_y (dense FP64 [ny][nx]) and adds dL/dbeta of the initial
 * state (through Pi^(1), eq. P1AC) to *dbeta. */
int lbm_adjoint_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t mode,
                     const void* lam0, double* grad_ux, double* grad_uy, double* dbeta);

/* ----------------------------------------------------------------- ensemble
 * Many independent lattices (e.g. of different sizes and beta) advanced
 * together.  An ensemble borrows member contexts created with lbm_init (same
 * form, collision, variant, stabiliser mode and stream)
 * and steps all of them; each member keeps its own buffers, parameters and
 * entry points (moments, populations, diagnostics).  Stepping is bitwise
 * identical to calling lbm_step on every member.  A member cannot be freed
 * while the ensemble lives (lbm_free returns LBM_EINVAL); a member's new beta
 * (lbm_set_beta) is taken up at the next lbm_ensemble_step, which then
 * rebuilds the member table (synchronising the stream). */
typedef struct lbm_ens lbm_ens;

int lbm_ensemble_create(lbm_ens** out, lbm_ctx* const* members, int32_t count);

/* Tile of the ensemble kernel: 128 x 4 (width 128, 2 rows per thread),
 * 256 x 1 or 256 x 2; flags as for lbm_set_tile (the default store kind
 * follows the same rule, applied to all members' buffers together).
 * Synchronises the stream. */
int lbm_ensemble_set_tile(lbm_ens* e, int32_t width, int32_t rows_per_thread, int32_t flags);

/* Steps per launch of lbm_ensemble_step: 1, or 2 (the fused two-step tile of
 * lbm_set_fusion for every member, 64 x `rows` tiles, rows in {8, 16}; 0
 * keeps the current height).  Defaults: 2 steps with 16 rows for FP32 and
 * FP16, 8 rows for FP64.  Bitwise identical either way; the
 * non-temporal flag of lbm_ensemble_set_tile applies to both.
 * lbm_ensemble_get_fusion returns the steps per launch and stores the rows in
 * *rows when not NULL (-1 for a NULL ensemble).  set_fusion with new rows
 * synchronises the stream. */
int lbm_ensemble_set_fusion(lbm_ens* e, int32_t steps_per_launch, int32_t rows);
int lbm_ensemble_get_fusion(const lbm_ens* e, int32_t* rows);

/* Advance every member nsteps of eq. (Egeneral).
 *   persistent = 0: one launch per step, or per pair of steps with
 *     lbm_ensemble_set_fusion(2), over all members' tiles;
 *   persistent = 1: ONE launch for all the steps (pairs of fused steps, or
 *     single steps with fusion 1; an odd step left over by the pairs runs as
 *     one more single-step launch): lbm_ensemble_blocks() workgroups, all
 *     resident at once, each taking tiles of its band of the tile range as it
 *     asks for them (a device-memory counter per band), with a grid barrier
 *     (device-memory arrival counters) between steps.
 *     Every barrier wait is bounded by the spin limit
 *     (lbm_ensemble_set_spin_limit): a workgroup that polls the counter that
 *     many times marks the launch as failed and every wait of the launch then
 *     ends at once, so the launch always terminates; lbm_ensemble_check
 *     reports it (LBM_ESYNC).  Runs of more than (2^32 - 1) / blocks barriers
 *     are split into several launches.
 * Both modes run the single-lattice tile code on the same tiles: bitwise
 * identical to lbm_step on every member.  All members must hold their
 * current state in the same buffer index (true when they have been stepped
 * equally since lbm_init).  Enqueues only (the persistent mode first resets
 * the barrier state with a one-workgroup kernel on the same stream). */
int lbm_ensemble_step(lbm_ens* e, int32_t nsteps, int32_t persistent);

/* Grid size of the persistent launch for the current fusion and tiles: CU
 * count x workgroups per CU, the smaller of the runtime's occupancy figure
 * and the kernel's own limits (8 four-wave workgroups, the CU's LDS over the
 * kernel's LDS, 512 registers over the kernel's register count), rounded
 * down to a multiple of 8.  Negative on error. */
int lbm_ensemble_blocks(const lbm_ens* e);

/* Polls of the barrier counter after which a waiting workgroup of a
 * persistent launch gives up (default LBM_ENSEMBLE_SPIN_DEFAULT, a few
 * seconds; every poll is a device-scope load followed by a short sleep; at
 * most LBM_ENSEMBLE_SPIN_MAX, else LBM_EINVAL).  0 gives up at the first poll
 * that finds the barrier still closed: a host-side way to exercise the
 * failure path. */
#define LBM_ENSEMBLE_SPIN_DEFAULT (1u << 22)
#define LBM_ENSEMBLE_SPIN_MAX (1u << 26)
int lbm_ensemble_set_spin_limit(lbm_ens* e, uint32_t polls);

/* Synchronises the stream and reports whether any persistent launch since
 * the last check gave up at a barrier: LBM_OK, or LBM_ESYNC (the members'
 * states are then invalid: re-initialise them).  Clears the flag. */
int lbm_ensemble_check(lbm_ens* e);

/* Release the ensemble (never the members).  Synchronises the stream. */
int lbm_ensemble_free(lbm_ens* e);

/* Streaming copy dst[i] = src[i] of n 4-byte words on `stream`, one word per
 * lane: the bandwidth and profiler-counter reference measured beside the step
 * (the same access granularity as the step kernel). */
int lbm_copy_probe(void* dst, const void* src, size_t n_words, void* stream);

#ifdef __cplusplus
}
#endif

#endif
