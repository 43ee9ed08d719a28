/*
 * swe_dg.h -- C ABI of the MI355X (gfx950) quadrature-free discontinuous
 * Galerkin solver for the 2D shallow water equations.
 *
 * Method: Faghih-Naini, Aizinger, Kuckuk, Angersbach, Koestler,
 * "p-adaptive discontinuous Galerkin method for the shallow water equations on
 * heterogeneous computing architectures" (2023).
 *   - equations (mass), (momentum) and the compact form (compact_qf_1),
 *     (compact_qf_2), (def_A_h_qf): state c = (xi, U, V), velocity u from u H = q;
 *   - semi-discrete form (variational_disc_1), (variational_disc_2) with the
 *     Lax-Friedrichs flux and penalty (eq:lambda);
 *   - modal expansions (c_h), (c_h_tilde) in a hierarchical orthonormal basis,
 *     K(p) = 1, 3, 6, 10 for p = 0..3;
 *   - order separation into a base part (order <= b on every element) and a
 *     correction (Sec. "Algorithmic adaptation: order separation",
 *     eq. (mass_basis)), constant-part penalty and friction, and the truncated
 *     depth expansion K(p,i,j) in u H = q;
 *   - two-stage SSP Runge-Kutta time stepping.
 *
 * Conventions
 *   - Host pointers passed in are borrowed for the duration of the call only;
 *     the library copies what it keeps.  Output pointers are written in full.
 *   - Device memory belongs to the context and is freed by swe_destroy.
 *   - Host coefficient arrays use the layout [element][component][mode]:
 *     component 0 = xi (elevation, m), 1 = U, 2 = V (m^2/s), K(p_max) modes
 *     in the physical orthonormal basis phi_ei (int phi_ei phi_ej = delta_ij),
 *     elements in the caller's order; modes above K(p_e) are zero.
 *   - Every call returns a swe_status; nothing aborts or throws across the
 *     ABI.  On failure swe_last_error() describes the cause.  After
 *     SWE_ESTATE the context refuses swe_step until swe_set_state.
 *   - A context is used by one host thread at a time; distinct contexts are
 *     independent.
 */
#ifndef SWE_DG_H
#define SWE_DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swe_ctx swe_ctx;

typedef enum {
    SWE_OK = 0,
    SWE_EINVAL = -1,        /* invalid argument, mesh or call order */
    SWE_ENOMEM = -2,        /* device or host allocation failed */
    SWE_EDEVICE = -3,       /* HIP runtime error */
    SWE_ESTATE = -4,        /* non-finite value or non-positive mean depth detected */
    SWE_EUNSUPPORTED = -5   /* valid request this build does not implement */
} swe_status;

enum { SWE_FP64 = 0,        /* state and all arithmetic in FP64 */
       SWE_FP32_WB = 1 };   /* FP32 state and bulk arithmetic; bathymetry terms
                               (well-balancing) and the mass reduction in FP64 */

enum { SWE_FRICTION_NONE = 0,
       SWE_FRICTION_LINEAR = 1,     /* r = -kappa q, kappa = friction_coef (1/s) */
       SWE_FRICTION_QUADRATIC = 2   /* r = -C_f |u_mean| u, C_f = friction_coef;
                                       u_mean = constant part of u (Sec. order separation) */
};

typedef struct {
    int precision;          /* SWE_FP64 or SWE_FP32_WB */
    int p_base, p_max;      /* 0 <= p_base <= p_max <= 3; every element order lies in [p_base, p_max] */
    double g;               /* gravitational acceleration (m/s^2), > 0 */
    double f_coriolis;      /* Coriolis parameter (1/s) */
    int friction;           /* SWE_FRICTION_* */
    double friction_coef;
    int adapt;              /* 0: static order map; 1: orders re-chosen every step by the indicator */
    double adapt_tau;       /* indicator threshold (m) when adapt = 1 */
    int separate;           /* 0: one full-order kernel per stage; 1: base and correction
                               kernels on two streams (the order separation of the
                               paper); 2: order-partitioned: elements of order p_base
                               with neighbours of order p_base in the base kernel, every
                               other element's full stage in a kernel of its order, on
                               parallel branches (same results, fewer dependent kernels);
                               not available with SWE_FP32_WB and p_max = 3 (SWE_EINVAL) */
    void *stream_base;      /* hipStream_t for the base work, or NULL for a library-owned stream */
    void *stream_corr;      /* hipStream_t for the correction work, or NULL */
    int step_graph;         /* how swe_step enqueues a step: 1 (default) one replayed HIP
                               graph per step (forcing clock on the device) for separated and
                               partitioned steps, plain launches for a fused step; 2 always
                               the graph; 0 always kernel-by-kernel launches */
    int hetero;             /* 1: heterogeneous stages (the paper's CPU + GPU co-execution,
                               Sec. "Performance results"): with separate = 1 and a static
                               order map, the GPU runs the base pass over every element while
                               the host's cores compute the listed elements' correction (the
                               same element code, on host copies of the state that listed
                               elements and their neighbours need, copied down and back each
                               stage); the GPU joins both in the epilogue.  Steps are
                               enqueued stage by stage and swe_step returns once the host part
                               of its last stage is done.  0 (default): every stage on the GPU */
    int host_threads;       /* host threads of the heterogeneous correction; 0: every usable core */
    double h_min;           /* minimum depth control (m) after every RK stage of swe_step (the
                               paper lists such a kernel, Sec. "Performance results", without a
                               formula; this reading): an element whose total depth is below
                               h_min at a vertex or an edge midpoint has its depth's deviation
                               from the element mean scaled by theta = (mean - h_min) /
                               (mean - lowest), or 0 when the mean is below h_min, keeping the
                               mean (the mass); its momentum's deviation is scaled alike and its
                               velocity solved again.  Order-0 elements are left alone.  0
                               (default): off.  Not available in batches (swe_batch_admit
                               refuses such a member) */
} swe_config;

/* Fill *cfg with defaults: FP64, p_base = p_max = 1, g = 9.81, no Coriolis,
 * no friction, static orders, unseparated, library-owned streams. */
void swe_config_default(swe_config *cfg);

/* Create a context on the current HIP device.  Fails with SWE_EINVAL for
 * out-of-range fields and SWE_EDEVICE if no device is usable. */
swe_status swe_create(const swe_config *cfg, swe_ctx **out);

/* Upload the triangulation (domain partition of Sec. "Quadrature-free DG
 * formulation").  vxy[nv][2] vertex coordinates (m); tri[ne][3] vertex ids of
 * counter-clockwise triangles; edge_tag[ne][3] (may be NULL) tags local edge k
 * (opposite vertex k): -1 interior/unspecified, 0 land (q.n = 0), 1 open sea
 * (xi = xi_hat).  Boundary edges tagged -1 are land.  Interior connectivity
 * is found from shared vertex pairs.  SWE_EINVAL for a non-positive area, an
 * out-of-range vertex id or an edge shared by more than two triangles.
 * Resets bathymetry (to 0), orders (to p_max, or p_base if separated), state
 * (to rest) and time (to 0). */
swe_status swe_set_mesh(swe_ctx *ctx, int64_t nv, const double *vxy, int64_t ne,
                        const int32_t *tri, const int8_t *edge_tag);

/* Bathymetry h_b at the vertices (m, depth below the datum); h_b is the
 * continuous piecewise-linear interpolant (reading of eqs. (mass)-(momentum)). */
swe_status swe_set_bathymetry(swe_ctx *ctx, const double *hb_vertex);

/* Per-element polynomial order p[ne] in [p_base, p_max].  Modes above the new
 * K(p_e) are dropped from the state (the L2 projection, the basis being
 * hierarchical and orthonormal); new modes start at zero.  In a separated,
 * non-adaptive context (a static order map) the library also renumbers its
 * device storage of the elements (elements without a correction first, then
 * those with one, by order) so that each order's list is contiguous; this
 * costs host time linear in ne and a rebuild of the step graphs, keeps the
 * source term of swe_set_source, and changes nothing at the interface (every
 * array in and out stays in the caller's element order). */
swe_status swe_set_order(swe_ctx *ctx, const int8_t *p);
swe_status swe_get_order(swe_ctx *ctx, int8_t *p_out);

/* Open-sea forcing xi_hat(t) = sum_i amp[i] sin(omega[i] t + phase[i]), ncon <= 16. */
swe_status swe_set_open_boundary(swe_ctx *ctx, int ncon, const double *amp,
                                 const double *omega, const double *phase);

/* State at time t0 from host coefficients coef[ne][3][K(p_max)] (physical
 * orthonormal basis, caller's element order).  Modes above each element's
 * current order are ignored; the current order is the one set by
 * swe_set_order or, in an adaptive context, the one the last order update on
 * the device chose (read back by this call, as by swe_get_order). */
swe_status swe_set_state(swe_ctx *ctx, double t0, const double *coef);

/* Input preparation: xy_out[ne][SWE_NQP][2] receives the physical points of
 * the projection rule; swe_set_state_points then L2-projects point values
 * vals[ne][SWE_NQP][3] of (xi, U, V) onto each element's space. */
#define SWE_NQP 36
swe_status swe_project_points(swe_ctx *ctx, double *xy_out);
swe_status swe_set_state_points(swe_ctx *ctx, double t0, const double *vals);

/* Optional extra right-hand side s[ne][3][K(p_max)] (coefficients of
 * (s, phi_ei), e.g. a manufactured-solution source); NULL clears it. */
swe_status swe_set_source(swe_ctx *ctx, const double *coef);

/* Advance nsteps SSP-RK2 steps of size dt (s).  Work is enqueued on the
 * context's streams; errors detected on the device surface at swe_sync.
 * With a step graph (see step_graph; at most 4 forcing constituents), one
 * step is a graph of kernel nodes (base and correction branches joined
 * where the scheme joins them) replayed nsteps times; stage times and the
 * open-sea elevation are computed on the device from t0 + k dt. */
swe_status swe_step(swe_ctx *ctx, int64_t nsteps, double dt);

/* Wait for queued work; returns SWE_ESTATE if a stage produced a non-finite
 * value or a non-positive element-mean depth. */
swe_status swe_sync(swe_ctx *ctx);

/* Current state coef_out[ne][3][K(p_max)] and time (synchronises). */
swe_status swe_get_state(swe_ctx *ctx, double *coef_out, double *t_out);

/* Total volume above the datum, sum_e int_e xi, reduced on the device in FP64
 * in a fixed order (deterministic). */
swe_status swe_mass(swe_ctx *ctx, double *out);

/* swe_mass for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same deterministic FP64 reduction over the current state, enqueued on the
 * context's base stream without allocating, copying, filling memory or
 * synchronising; the result (one double, the same bits as swe_mass) is
 * written to the device pointer d_out once the stream reaches it.  The
 * reduction's partial sums live in one fixed device array of 16384 doubles
 * per GPU (128 KiB, held until the process ends), so the mesh may have at
 * most 4,194,304 elements (SWE_EINVAL beyond, before anything is enqueued).
 * Calls that overlap on one GPU (other contexts' streams included) share
 * that array and race; serialise them.  SWE_EINVAL for a context resident in
 * a batch. */
swe_status swe_mass_noalloc(swe_ctx *ctx, double *d_out);

/* Test hooks: the semi-discrete right-hand side L(c, t) of (variational_disc_1)
 * (the time derivative of the coefficients) and the velocity coefficients
 * u_out[ne][2][K] of (variational_disc_2) for the given host state.  They do
 * not change the context's state. */
swe_status swe_rhs(swe_ctx *ctx, double t, const double *coef, double *rhs_out);
swe_status swe_usolve(swe_ctx *ctx, const double *coef, double *u_out);

/* Same as swe_rhs but split as the method's order separation defines it:
 * base_out receives the part with every basis index <= K(p_base), corr_out
 * the remainder; base + corr = full right-hand side. */
swe_status swe_rhs_split(swe_ctx *ctx, double t, const double *coef, double *base_out,
                         double *corr_out);

/* Indicator of the order adaptation, I[ne] (m), for the host state. */
swe_status swe_indicator(swe_ctx *ctx, double t, const double *coef, double *I_out);

/* Last error message of the context (never NULL; empty if none). */
const char *swe_last_error(const swe_ctx *ctx);

/* Upper bound of the device bytes a batch-ready context (uniform order
 * p_max, not separated, not adaptive) with ne elements holds on its own
 * after swe_set_mesh (state, velocity, geometry, order map, scratch, edge
 * items), and of what it takes resident in an empty batch (its share of the
 * pools plus the arrays it keeps); the vertex count is bounded by that of a
 * triangulated polygon with a few holes. */
int64_t swe_footprint_bytes(int64_t ne, int p_max, int precision);

/* Free everything the context holds; NULL is accepted. */
void swe_destroy(swe_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent instances advanced together.  Every resident
 * instance of one order is covered by one launch per RK stage (one tile per block);
 * each instance keeps its own time, step size, forcing and step budget on
 * the device, so one step graph (built from kernel nodes, no stream capture,
 * and replayed) serves any resident set.  Other host threads may create and
 * fill contexts while a batch runs.
 * Members are ordinary contexts (precision equal to the batch's, the fused
 * scheme separate = 0, no extra source) prepared with swe_set_mesh /
 * swe_set_bathymetry / swe_set_open_boundary (at most 4 constituents) /
 * swe_set_order / swe_set_state: one uniform order, a static per-element
 * order map, or orders the indicator re-chooses before every step (adapt).
 * A member lives in the pool of its p_max; a member with per-element orders
 * is stepped by the element-gather kernel with each element's modes masked
 * by its order (its order class then uses that kernel for every member),
 * and an indicator-driven member's order update runs over all such members
 * of the class in one launch before the stages.  While resident, a member refuses
 * swe_step, swe_set_* and the test hooks; swe_get_state and swe_mass wait
 * for the batch.  The budget given at creation bounds the device memory the
 * batch holds: its per-order pools (capacity doubling while the budget
 * allows, exact growth otherwise; old and new arrays are counted together
 * while a pool grows), tile lists, vertex pool, and the arrays a member
 * keeps while resident (vertex and neighbour ids, vertices, flag).  A
 * member's state buffers are released at admission (the pool holds its
 * state) and re-created when it is retired; swe_get_state and swe_mass of a
 * resident member re-create them for the call only.  A pool whose order has
 * no member left is released.
 * ------------------------------------------------------------------------ */
typedef struct swe_batch swe_batch;

/* cfg supplies the precision and the streams (stream_base, or NULL for a
 * library-owned stream); physics comes from each member.  max_instances
 * bounds the resident set (slots 0 .. max_instances-1). */
swe_status swe_batch_create(const swe_config *cfg, int64_t hbm_budget_bytes, int max_instances,
                            swe_batch **out);

/* Make ctx resident for nsteps steps of size dt from its current state and
 * time.  SWE_ENOMEM if the pool growth it needs would take the batch beyond
 * its budget (nothing changes then) or no slot is free; SWE_EINVAL if ctx
 * does not qualify.  *slot receives the slot. */
swe_status swe_batch_admit(swe_batch *b, swe_ctx *ctx, int64_t nsteps, double dt, int32_t *slot);

/* Enqueue nsteps steps of every resident instance (each stops at its own
 * budget).  Asynchronous. */
swe_status swe_batch_tick(swe_batch *b, int64_t nsteps);

/* Wait for queued steps. */
swe_status swe_batch_sync(swe_batch *b);

/* Steps left, current time and failure flag (non-finite value or
 * non-positive mean depth) of the instance in slot; synchronises. */
swe_status swe_batch_query(swe_batch *b, int32_t slot, int64_t *steps_left, double *t, int *failed);

/* Resident slots that are done (step budget used up) or failed, in slot
 * order: slots[0 .. *n-1] (at most max entries), failed[k] = 1 if slots[k]
 * was flagged.  One synchronising read for the whole batch. */
swe_status swe_batch_poll(swe_batch *b, int32_t *slots, int32_t *failed, int max, int *n);

/* Release the slot; the member context keeps its state and gets back its
 * time (and the failed state if flagged) and can be used on its own again. */
swe_status swe_batch_retire(swe_batch *b, int32_t slot);

/* Time the candidates on the resident set and keep the fastest per order:
 * the element-gather kernel with tiles of 64, 128 or 256 elements and, for
 * orders 1 to 3, the kernel that computes each edge flux inside a
 * 256-element tile once and shares it through LDS; reps timed launches
 * each. */
swe_status swe_batch_tune(swe_batch *b, int reps);

/* Choose the kernel of order p by hand instead of swe_batch_tune: the gather
 * kernel with tile = 64, 128 or 256 elements (shared = 0), or the shared-flux
 * kernel (shared = 1, tile = 256; SWE_EUNSUPPORTED for order 0).  Takes effect from the next tick.  If a resident member
 * of the order has no edge items, the order keeps the gather kernel. */
swe_status swe_batch_set_tile(swe_batch *b, int p, int tile, int shared);

/* Tile size, grid and kernel (*shared = 1: shared edge fluxes) of an order;
 * any pointer may be NULL. */
swe_status swe_batch_tile_config(const swe_batch *b, int p, int *tile, int *grid, int *shared);

/* Budget minus the device bytes the batch holds now. */
int64_t swe_batch_free_bytes(const swe_batch *b);
int swe_batch_resident(const swe_batch *b);
const char *swe_batch_last_error(const swe_batch *b);
void swe_batch_destroy(swe_batch *b);

/* Number of elements and stored modes per component (K(p_max)). */
int64_t swe_num_elements(const swe_ctx *ctx);
int swe_num_modes(const swe_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SWE_DG_H */
