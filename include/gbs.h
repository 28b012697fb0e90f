/*
 * gbs.h — C ABI of the MI355X (gfx950) extrapolated Gragg–Bulirsch–Stoer
 * time stepper for method-of-lines wave problems.
 *
 * Method (Ellison & Fornberg, "A parallel-in-time approach for wave-type
 * PDEs"): for y' = f(t, y) and a macro step H, each of k sequences with an
 * even step count N_j and substep h_j = H / N_j runs
 *     y_1 = y_0 + h f(t_0, y_0)                        forward Euler
 *     y_{n+1} = y_{n-1} + 2 h f(t_0 + n h, y_n)        leap-frog, n = 1..N_j
 *     y*_j = (y_{N-1} + 2 y_N + y_{N+1}) / 4           averaging
 * (Sect. 2.1, eq. GBS) and the step returns y_out = sum_j c_j y*_j
 * (Sect. 3.2) with weights c that satisfy the order constraints of eq.
 * (vander) and, when k > p/2, free weights chosen for the stability domain
 * (Sect. 3.7, eqs. order_constraints and cdep_computation).  f(t_0, y_0) is
 * the same for every sequence (Sect. 3.6): the streaming variants evaluate
 * it once per macro step and share it; the temporally blocked variants
 * evaluate it again in each sequence's first pass, which Sect. 3.6 allows
 * (they count 1 + sum_j N_j evaluations per point like the others, but
 * perform k + sum_j N_j).
 *
 * Conventions for every entry point:
 *  - Return value: GBS_OK (0) or a negative status; gbs_last_error() then
 *    returns a message for the calling thread.  No C++ exception crosses the
 *    ABI.
 *  - "host" pointers are read during the call only (copied where kept);
 *    "device" pointers are HIP device memory owned by the caller.  The
 *    library allocates no device memory: every scratch buffer lives in the
 *    caller's workspace.
 *  - Device work is enqueued on the plan's HIP stream and the call returns
 *    without synchronising; a fault in device code surfaces at the caller's
 *    next synchronisation.
 *  - A plan is not thread-safe; calls on one plan must not overlap.
 *
 * Data layout: a state is a contiguous array [R][F][Z][Y][X] (x fastest) of
 * the plan's dtype, R independent right-hand sides, F fields:
 *   GBS_ADVECT1D    F = 1 (u),                          grid X
 *   GBS_ACOUSTIC2D  F = 3 (p, v_x, v_y),                grid Y x X
 *   GBS_ACOUSTIC3D  F = 4 (p, v_x, v_y, v_z),           grid Z x Y x X
 * on the periodic unit box with spacing 1/n per axis.  The operators are the
 * periodic centred first-derivative stencils of order 4 or 8, or, for
 * GBS_ADVECT1D only, the Fourier (spectral) derivative of the paper's own
 * experiment (Sect. 4.1; fd_order = GBS_FD_SPECTRAL): the derivative of the
 * trigonometric interpolant on the n points, mode k multiplied by 2 pi i k
 * for |k| < n/2 and the mode n/2 of an even n by 0, applied on the device as
 * the equivalent centred sum over all n points (n^2 work per evaluation,
 * 4 <= n <= 8192):
 *   advection  u_t = -u_x
 *   acoustic   p_t = -c^2 div v + sum_s w_s r(t) delta_s,   v_t = -grad p
 * with r the Ricker wavelet of the plan's sources (if any).
 */
#ifndef GBS_H
#define GBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GBS_OK = 0,
  GBS_EINVAL = -1,      /* null pointer, bad size, shape or enum value          */
  GBS_ESTEPS = -2,      /* step count odd, non-positive, duplicated; k < p/2    */
  GBS_EORDER = -3,      /* order p odd or <= 0; p = 2 (mod 4) for a wave plan   */
  GBS_ESINGULAR = -4,   /* order-constraint system singular                      */
  GBS_EUNSTABLE = -5,   /* H exceeds ISB(R) / spectral radius of the operator    */
  GBS_EDEVICE = -6,     /* a HIP call failed                                     */
  GBS_ENOMEM = -7,      /* workspace too small                                   */
  GBS_EUNSUPPORTED = -8 /* combination not built (operator, order, dtype)        */
};

enum { GBS_ADVECT1D = 1, GBS_ACOUSTIC2D = 2, GBS_ACOUSTIC3D = 3 };
/* fd_order value of the Fourier derivative (GBS_ADVECT1D only) */
enum { GBS_FD_SPECTRAL = 0 };
enum { GBS_F32 = 1, GBS_F64 = 2 };
/* plan flags */
enum { GBS_FLAG_NO_STABILITY_CHECK = 1 };

typedef struct gbs_problem {
  int32_t op;           /* GBS_ADVECT1D / GBS_ACOUSTIC2D / GBS_ACOUSTIC3D            */
  int32_t fd_order;     /* 4 or 8, or GBS_FD_SPECTRAL with GBS_ADVECT1D              */
  int64_t n[3];         /* points along x, y, z (unused axes: 1)                     */
  int32_t n_rhs;        /* R >= 1 independent states sharing the coefficient field   */
  int32_t dtype;        /* GBS_F64, or GBS_F32 (stepping in FP32; the averaging and  */
                        /* the weighted combination are always accumulated in FP64)  */
  double c2;            /* constant c^2 (acoustic) when c2_field is NULL             */
  const void* c2_field; /* device, [Z][Y][X] in dtype, or NULL                       */
  double c_max;         /* max |c| over the grid; required with c2_field (stability) */
  int32_t flags;        /* GBS_FLAG_*                                                */
  int32_t reserved;
} gbs_problem;

typedef struct gbs_scheme {
  int32_t p;              /* order of the extrapolated step (even)            */
  int32_t k;              /* number of sequences, 1 <= k <= GBS_MAX_SEQ        */
  const int32_t* steps;   /* host [k]: even, distinct step counts N_j          */
  const double* weights;  /* host [k]: c_j, usually from gbs_weights()         */
} gbs_scheme;

#define GBS_MAX_SEQ 16
#define GBS_MAX_SRC 16
#define GBS_MAX_REC 1024

typedef struct gbs_plan gbs_plan;

/*
 * gbs_weights — order-constraint weights (Sect. 3.2 eq. vander; Sect. 3.7
 * eqs. order_constraints and cdep_computation).
 *   p         order (even, > 0); the system has p/2 rows k = 0..p/2-1 with
 *             entries n_i^(-2k) (the H^(2k) row scale cancels) and b = e_1.
 *   m         number of step counts; m >= p/2.
 *   steps     host [m] step counts (even, distinct, > 0).
 *   n_free    m - p/2 (or 0 when m = p/2).
 *   free_idx  host [n_free] positions in steps of the free weights, or NULL.
 *   c_free_num, c_free_den  host [n_free] the free weights as exact
 *             fractions num/den (den > 0), or NULL when n_free = 0.
 *   c_out     host [m] out: every weight rounded to the nearest double (ties
 *             to even) after an exact rational solve for the dependent ones.
 *   isb_out   host out, nullable: imaginary stability boundary of the exact
 *             R(xi) = sum c_i P_i(xi) (App. A/B), found from the exact
 *             polynomial |R(iy)|^2 - 1 with its zero at the origin divided
 *             out (0 when |R| > 1 next to the origin, e.g. p = 2 mod 4).
 * Host-only: needs no GPU.
 */
int gbs_weights(int32_t p, int32_t m, const int32_t* steps, int32_t n_free,
                const int32_t* free_idx, const int64_t* c_free_num,
                const int64_t* c_free_den, double* c_out, double* isb_out);

/*
 * gbs_isb — imaginary stability boundary of sum_j c_j P_{N_j} for the given
 * FP64 weights taken at their exact binary values (App. A; Sect. 2.2).
 * Host-only.
 */
int gbs_isb(int32_t k, const int32_t* steps, const double* weights, double* isb_out);

/*
 * gbs_plan_workspace_bytes — device workspace needed by a plan: a 512-byte
 * source table, a 16 KiB receiver table, one FP64 accumulator state plus,
 * per sequence, two levels
 * in the plan's dtype
 * (four for GBS_ACOUSTIC2D, whose temporally blocked passes read one pair
 * and write the other), each 256-byte aligned.
 */
int gbs_plan_workspace_bytes(const gbs_problem* prob, const gbs_scheme* sch, size_t* bytes);

/*
 * gbs_plan_create — validate and build a plan.
 *   prob, sch  host, copied.
 *   H          macro step (> 0).  Unless GBS_FLAG_NO_STABILITY_CHECK is set,
 *              H * rho must not exceed the ISB of the scheme, with rho =
 *              c_max * sigma * sqrt(sum_axes n_a^2), sigma = max_theta of the
 *              stencil's symbol (App. A: the operator's eigenvalues must lie
 *              in the stability domain) -> GBS_EUNSTABLE.  The ISB is that of
 *              the exact order-p scheme the FP64 weights round (the weights
 *              beyond the first p/2 as given, the first p/2 re-solved from
 *              the order constraints), when that moves no weight by more
 *              than 1e-12 of sum |c|; otherwise that of the given weights.
 *   workspace  device, at least gbs_plan_workspace_bytes(); owned by the
 *              caller, must outlive the plan, and must not be shared by
 *              plans whose calls overlap.
 *   hip_stream hipStream_t to enqueue on (NULL: the null stream).
 */
int gbs_plan_create(gbs_plan** out, const gbs_problem* prob, const gbs_scheme* sch,
                    double H, void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * gbs_plan_set_stream — enqueue the plan's later work on another
 * hipStream_t (NULL: the null stream).  The new stream first waits for the
 * work already enqueued on the old one (an event), so the plan's workspace
 * is never used by two streams at once; the caller orders its own buffers.
 * Errors: GBS_EINVAL (null plan), GBS_EDEVICE (event calls failed; the plan
 * keeps the old stream).
 */
int gbs_plan_set_stream(gbs_plan* plan, void* hip_stream);

/*
 * gbs_plan_set_sources — point sources on the pressure equation of an
 * acoustic plan: f_p[rhs[s]][flat_index[s]] += weight[s] * r(t), with the
 * Ricker wavelet r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - delay))^2,
 * evaluated on the host in FP64 at every substep time t_0 + n h_j.
 *   n_src <= GBS_MAX_SRC (0 removes the sources); arrays host [n_src];
 *   flat_index is the index within one field ([Z][Y][X], x fastest).
 *   The table is copied into the workspace; the call synchronises the
 *   plan's stream.
 */
int gbs_plan_set_sources(gbs_plan* plan, int32_t n_src, const int32_t* rhs,
                         const int64_t* flat_index, const double* weight, double f0,
                         double delay);

/*
 * gbs_step — n_macro extrapolated macro steps starting at time t0
 * (macro step i starts at t0 + i*H).
 *   y_in   device state at t0.
 *   y_out  device state at t0 + n_macro*H; may alias y_in.
 */
int gbs_step(gbs_plan* plan, double t0, int32_t n_macro, const void* y_in, void* y_out);

/*
 * gbs_rk4_step — n_steps classical fourth-order Runge-Kutta steps of size h
 * from t0 (step i starts at t0 + i*h) with the plan's operator, coefficient,
 * sources and dtype: the comparison method of Sect. 3.8 and App. A, on the
 * same stencil code (one streaming launch per stage; the stage sum
 * k1 + 2 k2 + 2 k3 + k4 in FP64).  y_in / y_out as for gbs_step (may alias).
 * Unless GBS_FLAG_NO_STABILITY_CHECK is set, h * rho must not exceed RK4's
 * imaginary stability boundary 2 sqrt 2 -> GBS_EUNSTABLE.  Uses the plan's
 * workspace (calls on one plan must not overlap).
 */
int gbs_rk4_step(gbs_plan* plan, double t0, int32_t n_steps, double h, const void* y_in,
                 void* y_out);

/*
 * gbs_plan_set_variant — choose the leap-frog kernel (all variants compute
 * the same values in the same order; they differ in work layout only):
 *   GBS_VARIANT_AUTO        library's choice (default): 2-D acoustic
 *                           GBS_VARIANT_TEMPORAL_S5, 3-D acoustic
 *                           GBS_VARIANT_TILE3D, 1-D GBS_VARIANT_FLAT
 *   GBS_VARIANT_FLAT        one grid point per thread (every operator)
 *   GBS_VARIANT_MARCH8/16   2-D acoustic: each thread marches 8 / 16 rows,
 *                           y-stencil rows kept in registers; 3-D acoustic:
 *                           each thread marches 64 / 128 planes, z-stencil
 *                           planes kept in registers
 *   GBS_VARIANT_MARCH8/16_NT  as above with non-temporal level stores
 *   GBS_VARIANT_TEMPORAL    2-D acoustic only: temporally blocked passes of
 *                           up to 7 (FD4) / 3 (FD8) evaluations of f per
 *                           launch, levels kept in registers; f(t_0, y_0) is
 *                           evaluated once per sequence
 *   GBS_VARIANT_TEMPORAL4   the same with at most 4 evaluations per pass
 *   GBS_VARIANT_TEMPORAL_S5/S6  at most 5 / 6 evaluations per pass, the
 *                           levels of one row step evaluated independently
 *                           (one more row of time skew between levels)
 *   GBS_VARIANT_PLAIN       the unfused reference form: one streaming launch
 *                           per sequence per leap-frog step (every operator)
 *   GBS_VARIANT_TEMPORAL_WG4/WG8  as GBS_VARIANT_TEMPORAL, with 4 / 8
 *                           wavefronts of a workgroup sharing their edge
 *                           columns through LDS (halo recomputed only at
 *                           the workgroup's edges)
 *   GBS_VARIANT_TILE3D      3-D acoustic only: z-marching sweeps in which a
 *                           1024-thread block stages each plane's 64 x 16
 *                           tile and its x/y halo in LDS once
 * The temporally blocked variants agree with the streaming ones to
 * rounding (the combination is summed in the same order, the products may
 * be contracted differently).
 * gbs_plan_get_variant returns the variant AUTO resolves to.
 * gbs_plan_set_band sets the rows per band of the temporally blocked
 * passes; 0 (the default) lets the library choose per launch from the
 * launch's wavefront count and the GPU's resident wavefronts (taller bands
 * for launches with few sequences).
 */
enum {
  GBS_VARIANT_AUTO = 0,
  GBS_VARIANT_FLAT = 1,
  GBS_VARIANT_MARCH8 = 2,
  GBS_VARIANT_MARCH16 = 3,
  GBS_VARIANT_MARCH8_NT = 4,
  GBS_VARIANT_MARCH16_NT = 5,
  GBS_VARIANT_TEMPORAL = 6,
  GBS_VARIANT_TEMPORAL4 = 7,
  GBS_VARIANT_TEMPORAL_S5 = 8,
  GBS_VARIANT_TEMPORAL_S6 = 9,
  GBS_VARIANT_PLAIN = 10,
  GBS_VARIANT_TEMPORAL_WG4 = 11,
  GBS_VARIANT_TEMPORAL_WG8 = 12,
  GBS_VARIANT_TILE3D = 13
};
int gbs_plan_set_variant(gbs_plan* plan, int32_t variant);
int gbs_plan_set_band(gbs_plan* plan, int32_t rows);
/*
 * gbs_plan_set_wave_order — order of the temporally blocked passes'
 * workgroups (a tuning knob; results do not change): 0 (default) one grid
 * row per sequence; 1 and 2 put the sequences of one group of 4 strips next
 * to each other on one XCD (workgroups reach the 8 XCDs round-robin), so
 * that first passes reading the same y_0 rows share an L2, with the groups
 * round-robin over the XCDs (1) or contiguous per XCD (2).  Errors:
 * GBS_EINVAL for a null plan or another value.
 */
int gbs_plan_set_wave_order(gbs_plan* plan, int32_t order);
/*
 * gbs_plan_set_form — how the temporally blocked passes organise a macro
 * step (flags; results agree to rounding):
 *   GBS_FORM_SHARED_F0      f(t_0, y_0) evaluated once per macro step by a
 *                           kernel of its own and shared by the first passes
 *                           of all sequences (Sect. 3.6), which then start
 *                           from (y_0, y_0 + h_j F_0); without it every first
 *                           pass evaluates f(t_0, y_0) itself
 *   GBS_FORM_FUSED_COMBINE  when the largest-N sequence's final pass is alone
 *                           in the last launch (and the plan runs on one
 *                           lane), that pass also forms y_out = sum_j c_j y*_j
 *                           instead of a separate combination kernel
 *   GBS_FORM_ALIGNED_FIRST  the first passes (one launch, every sequence
 *                           reading y_0) share one strip geometry, that of
 *                           the widest halo among them, and the workgroups
 *                           of the sequences for one group of strips are
 *                           adjacent on one XCD (wave order 2 unless another
 *                           is set), so that y_0 is read from HBM about once
 *                           rather than once per sequence; the sequences
 *                           with fewer evaluations recompute a wider halo
 * Default: 0 (neither: on the 2-D workload both measured slower, the shared
 * F_0 doubling the first passes' reads and the fused tail running one
 * sequence's wavefronts alone).  Errors: GBS_EINVAL (null plan, unknown
 * flags).
 */
enum { GBS_FORM_SHARED_F0 = 1, GBS_FORM_FUSED_COMBINE = 2, GBS_FORM_ALIGNED_FIRST = 4 };
int gbs_plan_set_form(gbs_plan* plan, int32_t form);
int gbs_plan_get_variant(const gbs_plan* plan, int32_t* variant);

/*
 * gbs_plan_set_lanes — lanes (1..4, default 1): the temporally blocked
 * passes of one macro step are spread over this many HIP streams — the
 * plan's stream and lanes - 1 streams the plan creates (default priority) —
 * with the sequences folded in pairs by ascending N (longest with shortest,
 * Sect. 3.6) and pair i on lane i mod lanes; the lanes start after all
 * earlier work on the plan's stream and are joined back into it before the
 * combination, so callers see every result ordered on the plan's stream.
 * Lanes let a launch with few sequences share the GPU with another lane's
 * launch instead of ending in a partly filled wave of wavefronts.  Other
 * variants ignore it.
 */
int gbs_plan_set_lanes(gbs_plan* plan, int32_t lanes);

/*
 * gbs_plan_autotune — the project's own tuner: times every temporally
 * blocked variant (those built for the plan's stencil order) at 32, 64, 96
 * and 128 rows per band and with the per-launch choice (0), on 1, 2 and 3
 * lanes (or, if *lanes_io > 0 on entry, on that many only), macro_steps
 * macro steps each from y_in into y_out (device buffers of one state, may be
 * the same; y_out is overwritten), on the plan's stream, and keeps the
 * fastest.  Operators other than the 2-D acoustic one have a single form:
 * the call returns it unchanged.  variant_out, band_out and lanes_io (host,
 * on return the lanes chosen) are nullable.  Synchronises the plan's stream.
 */
int gbs_plan_autotune(gbs_plan* plan, const void* y_in, void* y_out, int32_t macro_steps,
                      int32_t* variant_out, int32_t* band_out, int32_t* lanes_io);

/*
 * gbs_plan_set_timing — enabled != 0: every kernel launch is bracketed by HIP
 * events on the plan's stream, and gbs_plan_get_timing() returns the summed
 * duration (ms) and the launch count of the stepping kernel (streaming
 * leap-frog sweeps, or temporally blocked passes) and of the auxiliary
 * kernel (the shared first evaluation, or the final combination) since the
 * last reset (the read synchronises the stream and resets).  enabled > 1
 * also creates the events for that many macro steps up front.  enabled = 0
 * turns timing off.
 */
int gbs_plan_set_timing(gbs_plan* plan, int32_t enabled);
int gbs_plan_get_timing(gbs_plan* plan, double* step_ms, int64_t* step_launches,
                        double* aux_ms, int64_t* aux_launches);

/*
 * gbs_plan_get_adjoint_timing — with timing enabled, the summed duration
 * (ms) and the count of the temporally blocked adjoint's pass launches
 * (adj_pass2d; timed when the plan runs on one lane) since the last read,
 * and their algorithmic HBM bytes: per launch, y_N, y_{N-1} and ybar read by
 * a first pass or the two Z levels (Y and Psi) by a later one, the two Z
 * levels written (or lambda_0 + lambda_1 and h lambda_1 in FP64 by a final
 * pass), the FP64 gradient row sums written or updated, and c^2 once.  The
 * read synchronises the plan's stream and resets.  Outputs are nullable.
 */
int gbs_plan_get_adjoint_timing(gbs_plan* plan, double* pass_ms, int64_t* pass_launches,
                                double* pass_bytes);

/*
 * gbs_plan_algorithmic_bytes — HBM bytes one macro step must move with the
 * plan's current variant, per kernel class (stepping kernel / auxiliary
 * kernel, as in gbs_plan_get_timing), and the launches of each per macro
 * step: every state a launch reads counted once per launch (y0, shared by
 * the first passes of all sequences, and the c^2 field, shared by all
 * sequences and right-hand sides), every level, y* or accumulator it writes
 * once over the grid; halo re-reads and redundant edge work are not
 * counted.  For measurement only.
 */
int gbs_plan_algorithmic_bytes(const gbs_plan* plan, double* step_bytes, int64_t* step_launches,
                               double* aux_bytes, int64_t* aux_launches);

/* Updates (grid point x RHS x f-evaluation) one macro step performs. */
int gbs_plan_updates_per_macro_step(const gbs_plan* plan, double* updates);

int gbs_plan_destroy(gbs_plan* plan);

/*
 * Receivers and the adjoint (acoustic plans).  The paper defines only the
 * forward step (Sect. 2.1, eq. GBS; Sect. 3.2); the adjoint below is the
 * exact transpose of that discrete step for f(t, y) = A y + s(t):
 * each sequence's recurrence run backwards (leap-frog, averaging, forward
 * Euler, the shared first evaluation), plus the gradient with respect to
 * the coefficient field c^2.
 *
 * gbs_plan_set_receivers — n_rec <= GBS_MAX_REC receivers of the pressure:
 *   rhs[r], flat_index[r] (within one field) host arrays, copied into the
 *   workspace (synchronises the plan's stream).
 * gbs_step_record — as gbs_step, and after every macro step m writes
 *   traces[m][r] = p[rhs_r][flat_index_r] of the new state (device array
 *   [n_macro][n_rec] in the plan's dtype).
 * gbs_plan_adjoint_workspace_bytes — scratch for gbs_adjoint_step, the
 *   larger of the two forms' needs: streaming, the forward levels of one
 *   sequence (N_max of them), two adjoint levels and two FP64 accumulator
 *   states; temporally blocked (2-D, FD4), per sequence two pairs of
 *   (forward level, adjoint level) states, two FP64 states and one FP64
 *   gradient field per right-hand side, plus two FP64 states.
 * gbs_adjoint_step — one macro step backwards (the transpose of the
 *   discrete step; the paper defines the forward step only, Sect. 2.1 and
 *   3.2).  y_in: forward state at t0 (start of the macro step); ybar
 *   (device, in/out): on entry the adjoint of the state at t0 + H, on return
 *   the adjoint of the state at t0; trace_bar (device [n_rec], nullable):
 *   adjoint of the traces recorded at t0 + H, added to ybar's pressure at
 *   the receivers first; grad_c2 (device FP64 [Z][Y][X], nullable, needs a
 *   c^2 field): dL/dc^2 of this macro step is added to it.  The forward
 *   levels are recomputed from y_in (with the plan's sources): the 2-D FD4
 *   operator with a temporally blocked variant (the default) regenerates
 *   them by running the leap-frog backwards from the last two levels, which
 *   blocked forward passes leave in the plan's workspace (so calls on one
 *   plan must not overlap, as for gbs_step); every other case stores the
 *   levels of one sequence at a time in the adjoint workspace.
 */
int gbs_plan_set_receivers(gbs_plan* plan, int32_t n_rec, const int32_t* rhs,
                           const int64_t* flat_index);
int gbs_step_record(gbs_plan* plan, double t0, int32_t n_macro, const void* y_in, void* y_out,
                    void* traces);
int gbs_plan_adjoint_workspace_bytes(const gbs_plan* plan, size_t* bytes);
int gbs_adjoint_step(gbs_plan* plan, double t0, const void* y_in, void* ybar,
                     const void* trace_bar, double* grad_c2, void* adj_workspace,
                     size_t adj_workspace_bytes);

/*
 * Kept forward levels for the temporally blocked adjoint (2-D FD4 operator
 * with a temporally blocked variant; GBS_EUNSUPPORTED otherwise, checked
 * before any device work).  Trades memory for the forward passes that
 * gbs_adjoint_step runs to rebuild (y_{N_j - 1}, y_{N_j}) of every sequence:
 *
 * gbs_step_keep_pairs — as gbs_step (n_macro >= 1), and the final pass of
 *   every sequence also writes its last two leap-frog levels into `pairs`
 *   (device, caller-owned, in the plan's dtype), laid out
 *   [n_macro][k][2][R][F][Y][X]: macro step m, sequence j in the order of
 *   the scheme's steps[], then y_{N_j - 1} and y_{N_j}, each a whole state
 *   (2 k R F n_x n_y elements per macro step).
 * gbs_adjoint_step_pairs — as gbs_adjoint_step for the macro step starting
 *   at (t0, y_in), with `pairs` (device, read only) the [k][2][state] block
 *   that gbs_step_keep_pairs wrote for that macro step from the same y_in,
 *   t0 and plan settings; the result equals gbs_adjoint_step's.
 */
int gbs_step_keep_pairs(gbs_plan* plan, double t0, int32_t n_macro, const void* y_in,
                        void* y_out, void* pairs);
int gbs_adjoint_step_pairs(gbs_plan* plan, double t0, const void* y_in, const void* pairs,
                           void* ybar, const void* trace_bar, double* grad_c2,
                           void* adj_workspace, size_t adj_workspace_bytes);

/*
 * Batches of independent 2-D acoustic instances (GBS_ACOUSTIC2D, n_rhs = 1,
 * no sources), each with its own grid size, coefficient (constant c^2 or a
 * c^2 field) and macro step H[i], one common scheme, dtype and stencil
 * order.  The instances' sequences (Sect. 3.2) are advanced by the
 * temporally blocked passes: one launch per pass round covers every
 * (instance, sequence) pair, one more launch forms every instance's
 * combination; the per-launch work lists live in the workspace.
 *
 * gbs_batch_workspace_bytes — workspace for the item tables plus four
 *   levels per (instance, sequence).
 * gbs_batch_plan_create — validates every instance as gbs_plan_create does
 *   (stability check per instance with its own H and c_max); probs and H are
 *   host arrays [n_inst], copied; workspace as for gbs_plan_create.
 * gbs_batch_step — n_macro macro steps of every instance, in place: y is a
 *   host array [n_inst] of device state pointers ([1][3][ny][nx] each).
 *   The item tables are rebuilt and uploaded (synchronising the plan's
 *   stream) when the pointers differ from the previous call.
 * gbs_batch_set_variant — kernel variant (GBS_VARIANT_TEMPORAL*, 0 keeps
 *   the current one) and rows per band (0 keeps the current one).
 * gbs_batch_set_graph — enabled != 0: one macro step is captured once in a
 *   hipGraph on a stream the plan owns and replayed n_macro times, ordered
 *   after and before the caller's stream by events.
 * gbs_batch_autotune — times every candidate variant and band on the given
 *   states (which are advanced: pass copies) and keeps the fastest;
 *   variant_out and band_out are nullable.
 */
typedef struct gbs_batch_plan gbs_batch_plan;
int gbs_batch_workspace_bytes(int32_t n_inst, const gbs_problem* probs, const gbs_scheme* sch,
                              size_t* bytes);
int gbs_batch_plan_create(gbs_batch_plan** out, int32_t n_inst, const gbs_problem* probs,
                          const gbs_scheme* sch, const double* H, void* workspace,
                          size_t workspace_bytes, void* hip_stream);
int gbs_batch_set_variant(gbs_batch_plan* plan, int32_t variant, int32_t band);
int gbs_batch_set_graph(gbs_batch_plan* plan, int32_t enabled);
/* gbs_batch_set_stream — as gbs_plan_set_stream, for a batch plan. */
int gbs_batch_set_stream(gbs_batch_plan* plan, void* hip_stream);
int gbs_batch_step(gbs_batch_plan* plan, int32_t n_macro, void* const* y);
int gbs_batch_autotune(gbs_batch_plan* plan, void* const* y, int32_t macro_steps,
                       int32_t* variant_out, int32_t* band_out);
int gbs_batch_updates_per_macro_step(const gbs_batch_plan* plan, double* updates);
int gbs_batch_plan_destroy(gbs_batch_plan* plan);

/*
 * gbs_step_scratch — gbs_step without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): n_macro macro steps of the problem and
 * scheme (as for gbs_plan_create, without sources or receivers) from y_in
 * at t0 into y_out (device, caller-owned; may alias), enqueued on hip_stream.
 * The workspace is a static device array of the library, GBS_SCRATCH_BYTES
 * per GPU, held from the first call on a GPU until the process ends; its
 * address is looked up once per device.  Every call on one GPU uses the same
 * array and leaves its contents behind: calls that overlap on one GPU (other
 * threads, other streams without ordering) race.  Nothing in the array needs
 * clearing (every level is written before it is read).
 * Errors: those of gbs_plan_create and gbs_step; GBS_ENOMEM when the
 * problem's workspace (gbs_plan_workspace_bytes) exceeds GBS_SCRATCH_BYTES;
 * GBS_EUNSUPPORTED for the Fourier derivative.
 */
#define GBS_SCRATCH_BYTES ((size_t)64 << 20)
int gbs_step_scratch(const gbs_problem* prob, const gbs_scheme* sch, double H, double t0,
                     int32_t n_macro, const void* y_in, void* y_out, void* hip_stream);

/* Message for the last non-zero status returned on this thread. */
const char* gbs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GBS_H */
