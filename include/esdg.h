/*
 * esdg.h -- C ABI of the MI355X (gfx950) entropy-stable DGSEM solver for the
 * two-dimensional shallow water equations on curvilinear quadrilateral
 * meshes with wet/dry fronts (Wintermeyer, Winters, Gassner, Warburton,
 * "An entropy stable discontinuous Galerkin method for the shallow water
 * equations on curvilinear meshes with wet/dry fronts accelerated by GPUs",
 * arXiv:1804.02221).
 *
 * The library evaluates the semi-discrete operator of Lemma 1 extended by
 * the artificial-viscosity terms of Theorem 1,
 *     J W_t = -(L_xi + L_eta) + S + L^v_xi + L^v_eta,
 * applies the positivity-preserving limiter (eq. PosPres) and advances the
 * solution with a low-storage Runge-Kutta method (section 2.2) or SSPRK(3,3)
 * (eq. RKSSP) at a step chosen from a CFL bound, a viscous bound and the
 * mean-positivity bounds of Lemma 2 (eq. CFLConstraints).  Everything runs
 * in hand-written HIP kernels on one GPU; the host code only validates
 * arguments, owns device buffers and launches kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Polynomial degree N in [2, 8]; (N+1)^2 Legendre-Gauss-Lobatto nodes per
 *    element (section 2.2).  Nodal arrays are structure-of-arrays
 *    [K][(N+1)^2] float64, node p = i*(N+1) + j, i the xi-index, j the
 *    eta-index (the coalesced order of the paper's GPU section, version 4).
 *  - Local sides 0..3 are the paper's s = 1..4: eta=-1, xi=+1, eta=+1, xi=-1
 *    (Lemma 2).  Face node k runs along increasing xi (sides 0, 2) or
 *    increasing eta (sides 1, 3): side 0 -> (k,0), 1 -> (N,k), 2 -> (k,N),
 *    3 -> (0,k).
 *  - Face map: nbr_elem[e*4+s], nbr_side[e*4+s] name the element and local
 *    side sharing side s of element e; flip[e*4+s] = 1 when the neighbour's
 *    face-node order is reversed (its node N-k meets node k).  The mesh must
 *    be conforming.  nbr_elem[e*4+s] = -1 makes side s a solid (reflecting)
 *    wall: the interface flux takes as outside state the element's own trace
 *    with the normal velocity reversed (the same height and bathymetry), the
 *    artificial viscosity sees no jump there (U* = u, F^{v,*} = F^v), and the
 *    Lemma 2 bound uses the same mirror state (nbr_side/flip are ignored).
 *  - mem = 0: the pointer is host memory; mem = 1: device memory of the
 *    context's GPU (e.g. a torch tensor's data_ptr()).  The library copies
 *    in and out and never keeps a caller pointer.  Device-pointer transfers
 *    are asynchronous on the context stream; host-pointer transfers return
 *    after the data has arrived.
 *  - The ABI is float64 everywhere.  A precision-32 context converts on
 *    upload/download and computes in float32 (the bathymetry is taken in
 *    float64; its derivatives and face values are rounded); its volume,
 *    interface and viscous terms are formed from jumps to the own node (the
 *    two-point sums less the own flux), and each element's metric terms are
 *    stored relative to those of its middle node, so that its right-hand
 *    side is limited by the FP32 rounding of the stored state rather than
 *    by cancellation in the flux differencing.
 *  - Return value: ESDG_OK or a negative esdg_status; esdg_last_error()
 *    describes the last failure of a context.  No entry point throws.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef ESDG_H
#define ESDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esdg_ctx esdg_ctx;

typedef enum {
    ESDG_OK = 0,
    ESDG_EINVAL = -1,      /* bad argument, or call out of order            */
    ESDG_ENOMEM = -2,      /* device allocation failed                      */
    ESDG_EHIP = -3,        /* HIP runtime error                             */
    ESDG_EMESH = -4,       /* face map inconsistent or J <= 0 at a node     */
    ESDG_ENEGMEAN = -5,    /* limiter met a negative element mean (Lemma 2
                              violated); the state is still finite          */
    ESDG_EDTPOS = -6,      /* no admissible time step (all bounds infinite
                              or not positive)                              */
    ESDG_ENONFINITE = -7   /* a stage wrote a non-finite value (NaN or
                              infinity) into the state; checked once per
                              esdg_step / esdg_ensemble_step call            */
} esdg_status;

/* Run-time parameters.  esdg_default_params() fills the defaults. */
typedef struct {
    double g;          /* gravitational constant (9.81)                       */
    double h_tol;      /* dry cut-off: velocities are zero where h <= h_tol
                          in every flux; the limiter zeroes hu, hv where
                          h < h_tol (section 6.1; default 1e-4)             */
    double eps0;       /* artificial-viscosity amplitude (appendix A)        */
    double sigma_min;  /* indicator thresholds (appendix A); the paper gives
                          no values: default s0 -+ 1, s0 = -4 log10(N)      */
    double sigma_max;
    double cfl;        /* advective CFL number (0.5)                          */
    double cfl_visc;   /* safety factor of the viscous bound (0.5)            */
    int surface_flux;  /* 0: entropy stable (appendix B), 1: entropy
                          conservative (eq. surfaceFluxes)                   */
    int av_on;         /* artificial viscosity (Theorem 1)                    */
    int limiter_on;    /* positivity limiter after every stage (eq. PosPres),
                          and the Lemma 2 bound enters the adaptive step     */
    int integrator;    /* 0: LSRK(5,4) 2N-storage, 1: SSPRK(3,3)              */
    int max_dt_retries;/* redo a step (fixed or adaptive) from W^n with
                          dt/2, at most this many times, when it meets a
                          negative element mean or exceeds twice the smaller
                          of the CFL and viscous bounds of the state it
                          produced (each step then synchronises with the
                          host)                                             */
} esdg_params;

/* Fill *p with the defaults for degree N (N selects sigma_min/sigma_max). */
void esdg_default_params(esdg_params *p, int N);

/* Create a context on HIP device `device`; precision 64 or 32. */
int esdg_create(esdg_ctx **out, int device, int precision);
/* Free every device buffer of the context; ctx may be NULL. */
int esdg_destroy(esdg_ctx *ctx);
/* Launch and copy on `hip_stream` (a hipStream_t; NULL = default stream). */
int esdg_set_stream(esdg_ctx *ctx, void *hip_stream);
int esdg_set_params(esdg_ctx *ctx, const esdg_params *p);
int esdg_get_params(const esdg_ctx *ctx, esdg_params *p);

/*
 * Upload the mesh: nodal coordinates x, y [K][(N+1)^2] and the face map
 * (int32 [K][4], int8 [K][4], int8 [K][4]).  The metric terms x_xi, x_eta,
 * y_xi, y_eta are computed on the device by the LGL derivative matrix and
 * J = x_xi y_eta - x_eta y_xi (eqs. JacobianDef, NablaRelation).
 * ESDG_EMESH if the map is not symmetric or J <= 0 anywhere.  Replaces any
 * previous mesh, bathymetry and state.
 */
int esdg_upload_mesh(esdg_ctx *ctx, int N, int64_t K, const double *x, const double *y,
                     const int32_t *nbr_elem, const int8_t *nbr_side, const int8_t *flip,
                     int mem);

/*
 * Nodal bathymetry b [K][(N+1)^2].  Builds the split-form derivatives of
 * eq. SourceDisc (read with D in place of the printed 2D, and with the
 * chain-rule sign of b_y) and the face traces used by the interface flux.
 * b may jump across faces: the interface penalty S^{.,*} of eq. SourceDisc
 * (whose form the paper leaves to its earlier work) is taken as the one
 * Lemma 1.2 and 1.3 fix, -(1/w_0) J^surf {h} [[b]] n at every face node
 * (entering the source as (g/2) S^{.,*}); it vanishes where b is continuous
 * and at walls.  Lemma 2's positivity bound assumes a continuous b.
 */
int esdg_set_bathymetry(esdg_ctx *ctx, const double *b, int mem);

/* Conservative state h, hu, hv [K][(N+1)^2].  Resets the time to 0. */
int esdg_set_state(esdg_ctx *ctx, const double *h, const double *hu, const double *hv, int mem);
int esdg_get_state(esdg_ctx *ctx, double *h, double *hu, double *hv, int mem);

/*
 * R = dW/dt at the current state: R = -(1/J)(L_xi + L_eta - S - L^v), the
 * split-form flux-differencing volume term with the entropy-conservative
 * two-point fluxes (eqs. fluxDiffFormF, Fmij, volumeFluxes), the rotated
 * ES (or EC) interface flux (appendix B), the bathymetry source and, with
 * av_on, the BR1 viscous terms with the element viscosity of appendix A.
 * Outputs [K][(N+1)^2] each.
 */
int esdg_rhs(esdg_ctx *ctx, double *rh, double *rhu, double *rhv, int mem);

/* Positivity limiter in place (eq. PosPres, Jacobian-weighted means, theta
 * = 1 when the minimum is >= 0) followed by the h_tol velocity cut-off.
 * *n_limited (may be NULL) receives the number of scaled elements.
 * ESDG_ENEGMEAN if an element mean is negative (that element is set to its
 * mean). */
int esdg_limit(esdg_ctx *ctx, int64_t *n_limited);

/*
 * Time-step bounds at the current state: out[0] = dt (min of the CFL,
 * viscous and, when limiter_on, Lemma 2 bounds), out[1] = CFL bound,
 * out[2] = viscous bound (+inf without AV), out[3] = Lemma 2 bound
 * (eq. CFLConstraints with w_0 = 2/(N(N+1)) and a = J/J^surf).
 */
int esdg_compute_dt(esdg_ctx *ctx, double out[4]);

/*
 * Advance nsteps steps.  dt > 0: fixed step; dt <= 0: adaptive step from
 * esdg_compute_dt's bounds, evaluated on the device at the start of every
 * step (no host synchronisation unless max_dt_retries > 0).  With
 * limiter_on the limiter follows every stage.  *t_out (may be NULL)
 * receives the accumulated time.  Returns after the last step completed.
 * Status, checked once at the end of the call (the steps are not stopped
 * early): ESDG_ENONFINITE if any stage wrote a NaN or an infinity (a NaN
 * state also leaves no admissible adaptive step; ENONFINITE is reported
 * first), else ESDG_EDTPOS, else ESDG_ENEGMEAN (after max_dt_retries
 * halvings of a step).  The kernels run to completion on non-finite
 * values; the state then holds them.
 * With max_dt_retries > 0 a step is also checked after the fact (section 6:
 * the CFL step is adjusted when a smaller one proves necessary): a negative
 * element mean in the limiter, or a step (fixed or adaptive) larger than
 * twice the smaller of the CFL and viscous bounds of the state it produced
 * (its wave speeds or viscosity grew that much within the step), restarts
 * the step from W^n with half its size.  Out of retries the step is kept;
 * only a negative mean is then reported.
 */
int esdg_step(esdg_ctx *ctx, int nsteps, double dt, double *t_out);

/*
 * Graph replay of esdg_step (enable = 1, the default; an ensemble replays
 * per degree group).  Once the launch sequence of a step is fixed -- kernel
 * timing off, max_dt_retries = 0, the current state's viscosity and (for an
 * adaptive step) its time-step bounds already on the device -- each step
 * is launched as one HIP graph captured from the same launches: one graph
 * per start state buffer, kept until the parameters, the stage variant, the
 * fixed step or the mesh change.  Results are bitwise those of the eager
 * launches.  enable = 0 launches every kernel separately and frees the
 * graphs.  If graph capture fails the context falls back to eager launches
 * for good.
 */
int esdg_set_graphs(esdg_ctx *ctx, int enable);

/* Accumulated simulation time, and its reset. */
int esdg_get_time(esdg_ctx *ctx, double *t);
int esdg_set_time(esdg_ctx *ctx, double t);

/*
 * out[8] = total mass sum J w_i w_j h, momentum x, momentum y, total energy
 * (the entropy, eq. entropyFunction), its semi-discrete rate
 * sum J w_i w_j q . R (eq. entropyVariables), min h, max h, number of dry
 * nodes (h <= h_tol).
 */
int esdg_diagnostics(esdg_ctx *ctx, double out[8]);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as esdg_diagnostics, bitwise (the same kernels, and the partial
 * sums added in the same order), with the per-workgroup partial sums held
 * in a fixed device array of the library instead of the context's buffer,
 * and their final sum taken on the device.  The array holds 65536 partial
 * rows (4 MiB on each GPU the library runs on, kept until the process
 * ends); a mesh needing more -- more than 65536 * T nodes, T = 64 threads
 * per workgroup at N = 2, 3, 7 and 256 at N = 4, 5, 6, 8, i.e. 4,194,304
 * resp. 16,777,216 nodes -- returns ESDG_EINVAL with the limit in
 * esdg_last_error.  The call allocates nothing and returns after out[]
 * has arrived.  Every call on one GPU uses that GPU's one array: calls that
 * overlap in time on the same GPU (from several host threads or contexts)
 * race and must be serialised by the caller.
 */
int esdg_diagnostics_noalloc(esdg_ctx *ctx, double out[8]);

/* Activity of the hot path's non-smooth parts: *limited (may be NULL) =
 * element-stages the positivity limiter scaled during the last esdg_step
 * call (eq. PosPres); *viscous (may be NULL) = elements of the current state
 * with a positive viscosity (appendix A; 0 with av_on = 0). */
int esdg_step_stats(esdg_ctx *ctx, int64_t *limited, int64_t *viscous);

/* Element viscosities eps [K] of the current state (appendix A). */
int esdg_get_eps(esdg_ctx *ctx, double *eps, int mem);

/* Device-computed metric terms and Jacobian, [K][(N+1)^2] each. */
int esdg_get_geometry(esdg_ctx *ctx, double *xxi, double *xeta, double *yxi, double *yeta,
                      double *J, int mem);

/*
 * Kernel timing: with enable = 1, esdg_step and esdg_rhs record HIP events
 * around every launch of the stage kernel (the fused volume + interface +
 * source + update + limiter kernel), the viscosity kernels and the
 * time-step pass on the context stream (the events are recorded by the
 * kernel dispatch itself).
 * esdg_profile_read returns the summed event time in milliseconds and the
 * number of timed launches since the last reset, and resets the counters.
 */
int esdg_profile(esdg_ctx *ctx, int enable);
int esdg_profile_read(esdg_ctx *ctx, double *stage_ms, int64_t *stage_launches,
                      double *av_ms, int64_t *av_launches);
/* The same for the reverse stage kernel of esdg_rhs_vjp and
 * esdg_adjoint_backward: summed milliseconds and launches since the last
 * read, then reset. */
int esdg_profile_read_adjoint(esdg_ctx *ctx, double *ms, int64_t *launches);
/* Per kernel class, summed event milliseconds ms[k] and launches[k] since
 * the last read (all classes then reset): k = 0 stage kernel, 1 indicator
 * (viscosity of a state no stage produced), 2 viscous face fluxes (BR1,
 * Theorem 1), 3 viscous divergence (eq. ViscTermsDisc), 4 time-step pass
 * (eq. CFLConstraints and the CFL/viscous bounds), 5 adjoint reverse stage.
 * esdg_profile_read's av figures are classes 1-3. */
int esdg_profile_read_kernels(esdg_ctx *ctx, double ms[6], int64_t launches[6]);

/*
 * Autotuner of the stage kernel (the paper tunes its elements per block per
 * degree and GPU, appendix C).  Every degree has ESDG_STAGE_VARIANTS
 * compiled variants: 0 the default tile (one 64-lane wave where whole
 * elements fill it -- N = 2, 3, 7 -- else 256 threads) with its register
 * budget and partner-loop unroll; 1 the alternative workgroup size (256
 * resp. 128 threads); 2 the default tile with one wave per SIMD less in its
 * register budget; 3 the default tile with the other partner-loop unroll;
 * 4 the default tile with bank-conflict-free staging rows: padded by one
 * node (the paper's LDS padding, more LDS per tile), at N = 7 XOR-swizzled
 * columns instead (no more LDS).
 * esdg_autotune times reps launches of each on the context's mesh and
 * current state, twice, in the form the integrator uses (an interior
 * LSRK(5,4) stage, which reads the LSRK register, or an SSPRK(3,3) stage).
 * Trial stages write only a scratch state buffer: the state, the LSRK
 * register and the time are unchanged, and esdg_profile does not count
 * them.  esdg_autotune keeps
 * the fastest for all later launches and returns the
 * choice and the mean launch times in ms, ms[0..ESDG_STAGE_VARIANTS-1]
 * (either output may be NULL).  esdg_set_stage_variant sets the choice
 * directly.  Results do not depend on the choice (the same arithmetic per
 * element in the same order).
 */
#define ESDG_STAGE_VARIANTS 5
int esdg_autotune(esdg_ctx *ctx, int reps, int *choice, double ms[ESDG_STAGE_VARIANTS]);
int esdg_set_stage_variant(esdg_ctx *ctx, int variant);

/* Empirical LDS roofline (the paper's shared-memory roofline): 16-byte LDS
 * reads per second on device `device` in the volume term's access pattern
 * (one 8 x 8 element per 64-lane wave read along its lines), measured with
 * HIP events over a dedicated kernel.  Allocates and frees a small buffer. */
int esdg_lds_bandwidth(int device, double *bytes_per_s);

/* Last error message of ctx (never NULL). */
const char *esdg_last_error(const esdg_ctx *ctx);

/* ABI version (major*100 + minor). */
int esdg_abi_version(void);

/* ------------------------------------------------------------------------
 * Ensembles (batched instances)
 * ------------------------------------------------------------------------
 * Many independent problems -- each with its own mesh, degree, bathymetry,
 * initial state, time step and time -- advanced together.  The instances of
 * one degree form one context whose mesh is the disjoint union of their
 * meshes, so that every kernel launch covers all of them (small meshes that
 * would not fill the GPU alone share the launch); each instance keeps its
 * own adaptive step (the same bounds as esdg_compute_dt, reduced per
 * instance) and its own time.  Different degrees run on separate streams.
 * The arithmetic of every instance is that of a single-instance context.
 *
 * esdg_ensemble_add copies the instance (host pointers only; arrays as in
 * esdg_upload_mesh, esdg_set_bathymetry and esdg_set_state) and returns
 * its id (0, 1, ...).  Instances of one degree must have identical
 * parameters.  With max_dt_retries > 0 every instance takes the step check
 * of esdg_step on its own: an instance whose step met a negative element
 * mean or exceeds twice the CFL / viscous bound of its result redoes it with
 * half its step; the degree group's step is relaunched from W^n for the
 * instances to redo only (the others keep their step's results, the same
 * bit for bit; each degree group then waits for its step's checks, one host
 * synchronisation per round of redos).
 * esdg_ensemble_build uploads everything (done by the first step or query
 * if not called); no instance can be added afterwards.
 * esdg_ensemble_step advances every instance by nsteps adaptive steps and
 * returns when they are done (ESDG_ENEGMEAN / ESDG_EDTPOS if any instance
 * kept a step that met a negative element mean -- with retries, after them
 * -- / had no admissible step; with retries ESDG_ENONFINITE and ESDG_EDTPOS
 * end the call at the step where they occur).
 * esdg_ensemble_get_state / _get_time return one instance's state (mem:
 * 0 host, 1 device destination) and time.
 */
typedef struct esdg_ensemble esdg_ensemble;

int esdg_ensemble_create(esdg_ensemble **out, int device, int precision);
int esdg_ensemble_destroy(esdg_ensemble *en);
int esdg_ensemble_add(esdg_ensemble *en, const esdg_params *p, int N, int64_t K, const double *x,
                      const double *y, const int32_t *nbr_elem, const int8_t *nbr_side,
                      const int8_t *flip, const double *b, const double *h, const double *hu,
                      const double *hv, int *id);
int esdg_ensemble_build(esdg_ensemble *en);
int esdg_ensemble_step(esdg_ensemble *en, int nsteps);
/* Graph replay of every degree group's steps (esdg_set_graphs; on by
 * default).  Builds the ensemble if needed. */
int esdg_ensemble_set_graphs(esdg_ensemble *en, int enable);
int esdg_ensemble_size(const esdg_ensemble *en, int *n);
int esdg_ensemble_get_state(esdg_ensemble *en, int id, double *h, double *hu, double *hv, int mem);
int esdg_ensemble_get_time(esdg_ensemble *en, int id, double *t);
/* The degrees of the ensemble (n of them, in N[0..n-1] when N != NULL) and
 * the autotuner per degree (choices[g] for degree N[g], may be NULL). */
int esdg_ensemble_degrees(const esdg_ensemble *en, int *n, int *N);
int esdg_ensemble_autotune(esdg_ensemble *en, int reps, int *choices);
const char *esdg_ensemble_last_error(const esdg_ensemble *en);

/* ------------------------------------------------------------------------
 * Discrete adjoint (float64 contexts, inviscid operator: av_on = 0)
 * ------------------------------------------------------------------------
 * Reverse mode of the semi-discrete operator R of esdg_rhs (volume term of
 * eqs. fluxDiffFormF, Fmij and volumeFluxes, interface flux of appendix B,
 * source of eq. SourceDisc) and of LSRK(5,4) and SSPRK(3,3) steps (eq.
 * RKSSP), for gradients with respect to the nodal bathymetry.  The
 * artificial viscosity is frozen at zero (av_on must be 0: ESDG_EINVAL
 * otherwise).  Solid walls are covered: their outside state is a linear
 * mirror of the own trace, and the reverse mode runs through it.  The
 * limiter must not act: on a wet state (h >= h_tol everywhere, so theta = 1
 * and no velocity is cut off) it is the identity and so is its derivative.
 * |x| is differentiated as sign(x) with sign(0) = 0.
 */

/* gh, ghu, ghv = (dR/dW)^T lam and gb = (dR/db)^T lam at the current state
 * and bathymetry, lam = (lh, lhu, lhv).  Arrays [K][(N+1)^2] (mem: 0 host,
 * 1 device). */
int esdg_rhs_vjp(esdg_ctx *ctx, const double *lh, const double *lhu, const double *lhv, double *gh,
                 double *ghu, double *ghv, double *gb, int mem);

/* Gauges: ng >= 1 points, gauge g at reference point (xi[g], eta[g]) in
 * [-1,1]^2 of element elem[g] (host arrays).  A gauge reads the water surface
 * H = h + b interpolated with the LGL Lagrange basis.  Replaces earlier
 * gauges; a new mesh clears them.  esdg_gauge_values returns H at the gauges
 * for the current state (ng values; mem as above). */
int esdg_set_gauges(esdg_ctx *ctx, int ng, const int32_t *elem, const double *xi, const double *eta);
int esdg_gauge_values(esdg_ctx *ctx, double *H, int mem);

/*
 * Forward sweep of the gauge-misfit loss
 *     L = 1/2 sum_{n=1..nsteps} sum_g (H_g(t_n) - target[n-1][g])^2 dt
 * over nsteps steps of fixed size dt from the current state, LSRK(5,4) or
 * SSPRK(3,3) as the parameters' integrator selects.  target is [nsteps][ng]
 * (mem: 0 host, 1 device);
 * *loss (may be NULL) receives L and H (may be NULL) the gauge values
 * [nsteps][ng].  The state is advanced as by esdg_step; the states at steps
 * 0, every, 2 every, ... are kept on the device for esdg_adjoint_backward
 * (ceil(nsteps/every) states, plus S every + 1 stage states during the
 * backward sweep, S = 5 stages per LSRK step, 3 per SSPRK step).
 * ESDG_EINVAL if the limiter acted in any stage.
 */
int esdg_adjoint_forward(esdg_ctx *ctx, int nsteps, double dt, int every, const double *target, int mem,
                         double *loss, double *H);

/*
 * Reverse sweep of the last esdg_adjoint_forward: gb = seed * dL/db (the
 * initial state held fixed) and, when not NULL, g{h,hu,hv}0 = seed * dL/dW(0).
 * Each segment between checkpoints is recomputed from its checkpoint, then
 * its stages are reversed.  Leaves the current state alone.  ESDG_EINVAL if
 * no forward sweep is recorded or the bathymetry or the parameters changed
 * since.  (For an
 * initial state set through the surface, h(0) = H0 - b, the total gradient
 * is gb - gh0.)
 */
int esdg_adjoint_backward(esdg_ctx *ctx, double seed, double *gb, double *gh0, double *ghu0,
                          double *ghv0, int mem);

#ifdef __cplusplus
}
#endif

#endif /* ESDG_H */
