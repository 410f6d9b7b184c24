/*
 * hj.h -- C ABI of libhj, an MI355X (gfx950) implementation of the explicit
 * time step of the level-set / Hamilton-Jacobi(-Isaacs) method of
 * arXiv 2507.11542 (LevelSetPy).
 *
 * One call of hj_solve advances V_t + H(x, grad V) = 0 (Sec. 1.1, eq. ivp;
 * Sec. 4, eq. HJEquation) from V(t0) = V0 to tf on a dense Cartesian grid:
 * upwinded one-sided derivatives per axis (Sec. 3.1 first order, Sec. 3.2 ENO2,
 * Sec. 3.3 WENO5), the Lax-Friedrichs numerical Hamiltonian with dissipation
 * alpha_i = max over the grid of |dH/dp_i| (Sec. 4, LF equation), the CFL step
 * (Sec. 4), TVD Runge-Kutta stages (Sec. 5, odeCFL3 listing) and, for a
 * backward reachable tube, V <- min(V, V0) after every step (Sec. 6.1).
 *
 * Conventions shared by every call:
 *  - Arrays are C-order (last axis fastest), contiguous, one element per grid
 *    node, element type double (HJ_FP64) or float (HJ_FP32) as chosen at
 *    hj_grid_create.  The paper stores column-major (Sec. 2.1); the layout
 *    carries no meaning beyond the index order.
 *  - Pointers named V* are DEVICE pointers owned by the caller (for example
 *    torch tensors).  Other pointers are host pointers.
 *  - hip_stream is a hipStream_t (NULL = the null stream).  Calls that take a
 *    stream only enqueue work on it and return; the caller synchronises.
 *    hj_solve reads alpha back once per solve (a short wait on the stream
 *    before the step launches are enqueued).
 *  - Every call returns HJ_OK or a negative hj_status; hj_last_error() gives a
 *    message for the calling thread.  A handle is not thread-safe; separate
 *    handles are independent.
 */
#ifndef HJ_H_
#define HJ_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hj_grid_s *hj_grid_t;

/* The enums below are 32-bit integers at the boundary.  Compiled as C++ they
 * get int32_t as their fixed underlying type, so that a caller passing a
 * value outside the listed ones (which the calls reject with HJ_E_ARG) hands
 * the library a valid value of the type, not undefined behaviour. */
#ifdef __cplusplus
#define HJ_ENUM enum : int32_t
#else
#define HJ_ENUM enum
#endif

typedef HJ_ENUM {
    HJ_OK = 0,
    HJ_E_ARG = -1,         /* invalid argument (message says which) */
    HJ_E_OOM = -2,         /* device or host allocation failed */
    HJ_E_DEVICE = -3,      /* a HIP call failed */
    HJ_E_STATE = -4,       /* call order violated (e.g. no dynamics set) */
    HJ_E_NUMERIC = -5,     /* non-finite value detected where checked */
    HJ_E_UNSUPPORTED = -6  /* valid but not built (e.g. dynamics/ndim pair) */
} hj_status;

/* HJ_FP32 stores and computes V in float; alpha, dt and t stay double. */
typedef HJ_ENUM { HJ_FP64 = 0, HJ_FP32 = 1 } hj_precision;

/* HJ_SET: the reachable set V(tf).  HJ_TUBE: the tube, V <- min(V, V0) after
 * every full step (Sec. 6.1, backward reachable tube).  HJ_TUBE_VI: the tube
 * as the variational inequality of Sec. 6.1 (its min[0, H] form): every RK
 * stage uses L = min(L, 0), so V never increases and the zero sublevel set
 * only grows; V0 is not read after the start.  HJ_TUBE_OUTPUTS: V <- min(V, V0)
 * at the output times only (hj_solve: at tf; hj_solve_outputs: at each
 * output time), free steps in between. */
typedef HJ_ENUM { HJ_SET = 0, HJ_TUBE = 1, HJ_TUBE_VI = 2, HJ_TUBE_OUTPUTS = 3 } hj_mode;

/* One-sided derivative approximations (Sec. 3): first order (Sec. 3.1, halo
 * 1), ENO2 (Sec. 3.2, halo 2), ENO3 (Sec. 3.2's third-order paragraph, halo
 * 3), WENO5 (Sec. 3.3, halo 3). */
typedef HJ_ENUM { HJ_UPWIND1 = 1, HJ_ENO2 = 2, HJ_ENO3 = 3, HJ_WENO5 = 5 } hj_space;

/* Lax-Friedrichs dissipation coefficients (Sec. 4; its dissipation routine
 * takes the one-sided derivatives).  HJ_DISS_LF (default): alpha_d = max over
 * the grid nodes of the control-set bound of |dH/dp_d|, once per solve.
 * HJ_DISS_LLF: per node, max over the node's own costate box
 * [min(p-, p+), max(p-, p+)] of |dH/dp_d|.  HJ_DISS_GLF: per node, max over
 * the grid-wide box of both one-sided derivatives of the stage input (one
 * extra reduction pass over the grid per stage).  A switching function's
 * sign set over a box comes from interval arithmetic on its ends.  The step
 * size always uses the control-set bound, which bounds both box variants. */
typedef HJ_ENUM { HJ_DISS_LF = 0, HJ_DISS_LLF = 1, HJ_DISS_GLF = 2 } hj_dissipation;

/* TVD Runge-Kutta order (Sec. 5): forward Euler, Shu-Osher RK2, RK3. */
typedef HJ_ENUM { HJ_RK1 = 1, HJ_RK2 = 2, HJ_RK3 = 3 } hj_time;

/* Compiled dynamics, sign convention V_t + H = 0, H = -opt_{u,d} p.f(x,u,d).
 * params (in order) and dimension:
 *   HJ_DYN_TRANSLATION       any ndim   b[0..ndim-1]        x' = b,         H = -b.p
 *   HJ_DYN_BALL              any ndim   s                   x' = s u, |u|<=1, H = s|p|
 *   HJ_DYN_DOUBLE_INTEGRATOR ndim 2     umax                x1' = x2, x2' = u, |u|<=umax,
 *                                                           control minimises
 *   HJ_DYN_REL_DUBINS        ndim 3     ve, vp, we, wp      (x, y, psi) relative Dubins
 *                                       pursuit-evasion; evader (|we|) maximises,
 *                                       pursuer (|wp|) minimises
 *   HJ_DYN_DUBINS4D          ndim 4     wmax, amax          (x, y, th, v) Dubins car with
 *                                       speed state, control minimises
 *   HJ_DYN_ROCKETS           ndim 3     a, g, umax          (x, z, th) rockets launch game
 *                                       of Sec. 6.1 with the vector field of eq. ham_def,
 *                                       x' = a cos th + ue x, z' = a sin th + a + up x - g,
 *                                       th' = up - ue, |ue|,|up| <= umax, evader (ue)
 *                                       maximises, pursuer (up) minimises:
 *                                       H = -a p1 cos th - p2 (a sin th + a - g)
 *                                           - umax|p1 x - p3| + umax|p2 x + p3| */
typedef HJ_ENUM {
    HJ_DYN_TRANSLATION = 0,
    HJ_DYN_BALL = 1,
    HJ_DYN_DOUBLE_INTEGRATOR = 2,
    HJ_DYN_REL_DUBINS = 3,
    HJ_DYN_DUBINS4D = 4,
    HJ_DYN_ROCKETS = 5
} hj_dyn;

/* Implicit surfaces (Sec. 2.2, Fig. 4): a shape is negative inside.  It takes
 * part along the axes of `axes` (bit d: axis d; 0 = all axes; a sphere always
 * uses all axes), with plain coordinate differences (no wrap on a periodic
 * axis).
 *   HJ_SHAPE_SPHERE, HJ_SHAPE_CYLINDER  sqrt(sum (x_d - center_d)^2) - radius
 *                                       (signed distance; a cylinder is
 *                                       infinite along the axes it leaves out)
 *   HJ_SHAPE_BOX        signed distance to the box |x_d - center_d| <= size_d
 *   HJ_SHAPE_ELLIPSOID  sum size_d (x_d - center_d)^2 - radius (the quadratic
 *                       form of the ellipsoid listing, weights e.g. 1, 4, 9)
 * Shapes combine left to right with their op (the first one's is ignored):
 * HJ_OP_UNION min(v, s), HJ_OP_INTERSECT max(v, s), HJ_OP_SUBTRACT
 * max(v, -s). */
typedef HJ_ENUM {
    HJ_SHAPE_SPHERE = 0,
    HJ_SHAPE_CYLINDER = 1,
    HJ_SHAPE_BOX = 2,
    HJ_SHAPE_ELLIPSOID = 3
} hj_shape_kind;
typedef HJ_ENUM { HJ_OP_UNION = 0, HJ_OP_INTERSECT = 1, HJ_OP_SUBTRACT = 2 } hj_shape_op;
typedef struct {
    int32_t kind;      /* hj_shape_kind */
    int32_t op;        /* hj_shape_op */
    uint32_t axes;     /* axis mask, 0 = all */
    uint32_t reserved; /* 0 */
    double center[4];
    double size[4];    /* box half-widths, ellipsoid weights */
    double radius;     /* sphere/cylinder radius, ellipsoid level */
} hj_shape;

/* Sec. 2.1 (createGrid(min, max, N, pdim)).  ndim in [1, 4]; N[i] nodes on
 * axis i in [lo[i], hi[i]]; bit i of periodic_mask makes axis i periodic.  A
 * bounded axis has both ends as nodes, dx = (hi-lo)/(N-1); a periodic axis
 * excludes hi, dx = (hi-lo)/N.  Bounded axes take linearly extrapolated ghost
 * values.  Needs N[i] >= 7 (the widest stencil), lo < hi, prod(N) < 2^31.
 * Allocates the per-axis coordinate tables on the current HIP device; the
 * handle owns them and its stage buffers until hj_grid_destroy. */
hj_status hj_grid_create(int ndim, const int64_t *N, const double *lo, const double *hi,
                         uint32_t periodic_mask, hj_precision prec, hj_grid_t *out);

/* Sec. 6.1 / eq. ham_def: choose the Hamiltonian (see hj_dyn).  params is a
 * host array of nparams doubles; HJ_E_ARG on a wrong count, HJ_E_UNSUPPORTED
 * when the dynamics needs another ndim. */
hj_status hj_set_dynamics(hj_grid_t g, hj_dyn kind, const double *params, int nparams);

/* Sec. 3-5: derivative scheme, RK order and CFL number (0 < cfl <= 1).  The
 * default is WENO5, RK3, 0.8. */
hj_status hj_set_scheme(hj_grid_t g, hj_space space, hj_time time, double cfl);

/* Sec. 4: the dissipation coefficients of later solves and steps (see
 * hj_dissipation).  HJ_E_ARG on an unknown kind. */
hj_status hj_set_dissipation(hj_grid_t g, hj_dissipation kind);

/* Sec. 5 time loop over [t0, tf] (odeCFL3): alpha is max-reduced on the GPU,
 * dt = cfl / sum_i alpha_i/dx_i, steps of min(dt, tf - t) until
 * tf - t < 100*2^-52*(tf - t0).  V0 and V_out are device arrays of prod(N)
 * elements; V_out receives V(tf) and must not overlap V0.  t0 == tf copies
 * V0.  HJ_E_ARG on NULL pointers, overlap, tf < t0 or non-finite times. */
hj_status hj_solve(hj_grid_t g, const void *V0, void *V_out, double t0, double tf,
                   hj_mode mode, void *hip_stream);

/* hj_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, checks, kernels and results as hj_solve, but the RK stage
 * buffers are taken from a static 128 MiB device array of the library (one
 * per device, held until the process ends) instead of the handle's own, and
 * the call allocates nothing.  The stage buffers of RK3 need 2 * prod(N) *
 * sizeof(element) bytes (RK1/RK2: half), so FP64 grids up to 8,388,608 nodes
 * and FP32 grids up to 16,777,216 nodes fit; larger grids get HJ_E_ARG.
 * HJ_DISS_GLF (per-stage reduction buffers) gets HJ_E_UNSUPPORTED.  The array
 * is shared by every call on a device and keeps the last call's contents:
 * calls whose work overlaps on one device (other streams, other threads)
 * race, so order them on one stream or wait between them.  Like hj_solve it
 * waits once on the stream for alpha. */
hj_status hj_solve_noalloc(hj_grid_t g, const void *V0, void *V_out, double t0, double tf,
                           hj_mode mode, void *hip_stream);

/* Sec. 2.2: V_out (device, prod(N) elements of the grid's precision) at every
 * node from the nshapes shapes (host array, 1..16 of them), evaluated in FP64
 * on the device (FP32 grids store the rounded value), so a solve's initial
 * values need no host-to-device copy.  Enqueued on hip_stream.  HJ_E_ARG on
 * NULL pointers, nshapes out of range, unknown kinds or ops, or masks naming
 * axes >= ndim. */
hj_status hj_init_shapes(hj_grid_t g, void *V_out, const hj_shape *shapes, int nshapes,
                         void *hip_stream);

/* Sec. 6.1 (the global time steps of the rockets game) with the Sec. 5 loop:
 * a solve from V0 at t0 through the output times times[0..ntimes) (host
 * array, ascending, times[0] >= t0).  Each interval [t_{k-1}, t_k] runs the
 * loop of hj_solve on its own and ends exactly at t_k.  V_outs is one device
 * array of ntimes * prod(N) elements: V(t_k) is written at offset
 * k * prod(N); it must not overlap V0.  Enqueues on hip_stream after one
 * synchronisation (alpha).  HJ_E_ARG on NULL pointers, ntimes < 1, times out
 * of order or before t0, overlap, or non-finite times. */
hj_status hj_solve_outputs(hj_grid_t g, const void *V0, void *V_outs, double t0,
                           const double *times, int ntimes, hj_mode mode, void *hip_stream);

/* Precision form of hj_solve for an HJ_FP32 grid: V0 and V_out are FP64
 * device arrays; V0 is rounded to FP32, the whole solve runs in FP32 storage
 * and arithmetic (alpha, dt and t in FP64), and the result is widened to FP64
 * with the tube comparison of Sec. 6.1 taken again in FP64 where the zero
 * level set lies: V_out = min(V32, V0) on the band |V32| <= band (HJ_TUBE),
 * V32 elsewhere.  band < 0 selects 3 max(dx).  The handle keeps two FP32
 * working arrays.  Modes HJ_SET, HJ_TUBE and HJ_TUBE_VI (no FP64 minimum
 * for the last).  HJ_E_ARG on an FP64 grid or the argument errors of
 * hj_solve. */
hj_status hj_solve_mixed(hj_grid_t g, const double *V0, double *V_out, double t0, double tf,
                         hj_mode mode, double band, void *hip_stream);

/* The FP64 end of hj_solve_mixed on its own, for FP32 results computed some
 * other way (hj_solve, hj_step, a batch): V_out = min(double(V32), V0) on the
 * band |V32| <= band when mode is HJ_TUBE (the tube comparison of Sec. 6.1,
 * taken in FP64 where the zero level set lies), double(V32) elsewhere and
 * for HJ_SET and HJ_TUBE_VI.  V32 is the grid's FP32 array, V0 and V_out
 * FP64 arrays of the grid's node count (device, C order); V_out must not
 * overlap either.  band < 0 selects 3 max(dx).  hj_solve_mixed equals
 * hj_solve on float(V0) followed by this call, bit for bit.  HJ_E_ARG on an
 * FP64 grid, NULL pointers, overlap or another mode. */
hj_status hj_tube_finish(hj_grid_t g, const float *V32, const double *V0, double *V_out,
                         hj_mode mode, double band, void *hip_stream);

/* One full TVD-RK step in place on V (device), of size min(dt, tf - *t),
 * then the tube update against V0 when mode is HJ_TUBE (V0 may be NULL for
 * HJ_SET and HJ_TUBE_VI; HJ_TUBE_OUTPUTS is not a per-step mode: HJ_E_ARG).  *t advances by the step (FP64, host); *dt_used receives it
 * (may be NULL).  alpha is reduced on the first call and cached.  Resuming a
 * solve from (V, t) is a sequence of hj_step calls. */
hj_status hj_step(hj_grid_t g, void *V, const void *V0, double *t, double tf,
                  hj_mode mode, double *dt_used, void *hip_stream);

/* Sec. 4: L(V) = -Hhat(p-, p+) at every node (the semi-discrete right-hand
 * side of one stage) into L_out (device, same element type).  Runs the alpha
 * reduction first if no alpha is cached. */
hj_status hj_rhs(hj_grid_t g, const void *V, void *L_out, void *hip_stream);

/* Sec. 4 dissipation and CFL bound: runs the GPU max-reduction of |dH/dp_i|
 * over all nodes (synchronising the stream), caches it, and returns alpha
 * (ndim doubles), dt and the step count for [t0, tf].  Any output may be NULL. */
hj_status hj_get_schedule(hj_grid_t g, double t0, double tf, double *alpha, double *dt,
                          int64_t *n_steps, void *hip_stream);

/* Sec. 4 dissipation and CFL bound, and the length of the last solve:
 * alpha (ndim doubles) of the current dynamics (reduced on the GPU on the
 * null stream, with a synchronisation, if the handle has none cached), the
 * CFL step dt, and the number of RK steps of the handle's last hj_solve or
 * hj_solve_outputs (0 before the first; the steps of hj_solve_mixed count,
 * hj_step does not).  Any output may be NULL.  HJ_E_STATE before
 * hj_set_dynamics. */
hj_status hj_get_info(hj_grid_t g, double *alpha, double *dt, int64_t *n_steps);

/* ------------------------------------------------------------------------
 * Batched solves.  n independent grids that share ndim, dynamics kind,
 * derivative scheme (ENO2, ENO3 or WENO5), RK order (2 or 3), precision and device
 * advance together: one fused launch per RK-stage round covers the tiles of
 * every instance still running, so instances of any size and step count run
 * side by side, and each keeps its own alpha, dt and FP64 time t on the device
 * (Sec. 5 time loop per instance).  The round launches are captured once in a
 * hipGraph and replayed; the instance tables live in device memory and are
 * uploaded before each replay.  Results equal the instances' hj_solve results
 * bit for bit (same per-node arithmetic, same FP64 step sizes). */
typedef struct hj_batch_s *hj_batch_t;

/* New batch engine on the current device. */
hj_status hj_batch_create(hj_batch_t *out);

/* Launch shape.  workgroups == 0 (the default) selects flat launches: every
 * round launch has one 256-thread workgroup per 256-node tile of the round
 * (one node per thread), and tile_nodes is ignored.  workgroups in
 * [1, 65536] selects strided launches: that many workgroups per round stride
 * over the round's tiles, each tile up to tile_nodes nodes (a multiple of
 * 256 in [256, 2^22]; an instance's tiles shrink, in steps of 256, so that
 * it has at least 512 of them when it can).  tile_nodes is checked in both
 * cases.  use_graph != 0 (default) replays a captured hipGraph instead of
 * launching directly: the handle keeps up to 16 graphs, each captured for one
 * kernel variant, RK order, launch shape and round count (flat launches: with each
 * round's workgroup count rounded up to one of 8 sizes per power of two) and
 * replayed by any batch that fits it, and captures a new one when none does.
 * HJ_E_ARG out of range. */
hj_status hj_batch_config(hj_batch_t b, int tile_nodes, int workgroups, int use_graph);

/* Solve instance i from V0s[i] over [t0[i], tf[i]] in modes[i] into Vouts[i]
 * (device arrays of grid i's size and precision; V_out must not overlap any
 * V0 or other V_out).  The grids' dynamics and schemes must be set.  Runs one
 * alpha reduction per instance (one synchronisation for all), then enqueues
 * the uploads and the launch on hip_stream and returns.  A second call waits
 * for the previous one of the same handle to finish before it reuses the
 * tables.  Modes HJ_SET, HJ_TUBE and HJ_TUBE_VI; dissipation HJ_DISS_LF or
 * HJ_DISS_LLF per instance.  HJ_E_ARG on mismatched or invalid instances,
 * HJ_E_UNSUPPORTED for first-order schemes, RK1 or HJ_DISS_GLF. */
hj_status hj_solve_batch(hj_batch_t b, int n, const hj_grid_t *gs, const void *const *V0s,
                         void *const *Vouts, const double *t0, const double *tf,
                         const hj_mode *modes, void *hip_stream);

/* Resumable batched stepping (the continuous-batching form): instance i
 * advances Vs[i] in place by up to max_steps TVD-RK steps (all remaining
 * steps if max_steps <= 0) from the time t[i] toward tf[i]; the step sequence
 * and termination rule are those of a solve started at t0[i], so any split
 * into calls gives the hj_solve result bit for bit.  On return t[i] holds the
 * time reached (computed on the host in FP64 exactly as the device
 * accumulates it), steps_taken[i] (may be NULL) the number of steps taken
 * and finished[i] (may be NULL) is 1 when tf[i] is reached.
 * V0s[i] is read for HJ_TUBE instances (may be NULL for HJ_SET ones; V0s may
 * be NULL when no instance is a tube).  alpha is reduced on an instance's
 * first call and cached in its grid.  Enqueues on hip_stream and returns. */
hj_status hj_step_batch(hj_batch_t b, int n, const hj_grid_t *gs, const void *const *V0s,
                        void *const *Vs, const double *t0, double *t, const double *tf,
                        const hj_mode *modes, int max_steps, int *steps_taken, int *finished,
                        void *hip_stream);

/* Waits for the last hj_solve_batch or hj_step_batch on hip_stream.  t_final (n doubles, may
 * be NULL) receives each instance's device-accumulated final time, items
 * (may be NULL) the number of tiles over all rounds.  The grids passed to
 * hj_solve_batch must stay alive until this returns. */
hj_status hj_batch_wait(hj_batch_t b, void *hip_stream, double *t_final, int64_t *items);

/* Frees the engine (waits for its last batch).  NULL is accepted. */
hj_status hj_batch_destroy(hj_batch_t b);

/* Optional check of solve results: with HJ_CHECK_FINITE set, hj_solve,
 * hj_solve_outputs, hj_solve_mixed and hj_solve_noalloc scan their result on
 * the device for NaN or infinite values after the last stage, wait for the
 * stream, and return HJ_E_NUMERIC if any is found (the result is written
 * either way).  Off by default: a solve then returns after enqueueing.
 * hj_step and batches are not checked.  Enabling it allocates a device flag
 * (hj_solve_noalloc stays allocation-free once it is enabled).  HJ_E_ARG on
 * unknown flags. */
enum { HJ_CHECK_FINITE = 1 };
hj_status hj_set_check(hj_grid_t g, int flags);

/* Caller-owned stage buffers: A and B are device arrays of prod(N) elements
 * of the grid's element type, not overlapping each other or any V passed to
 * this grid's solves; the handle uses them instead of allocating its own
 * (freeing any it had) and never frees them.  For callers that keep device
 * memory in their own pool (a serving loop). */
hj_status hj_grid_set_workspace(hj_grid_t g, void *A, void *B);

/* Frees the handle, its tables and stage buffers (after the device is idle
 * for this handle's work).  NULL is accepted. */
hj_status hj_grid_destroy(hj_grid_t g);

/* Message of the last failed call on this thread ("" if none). */
const char *hj_last_error(void);

/* Library version string. */
const char *hj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HJ_H_ */
