/*
 * lbm.h - C ABI of the MI355X (gfx950) Cole-Hopf fourth-order MRT lattice
 * Boltzmann solver (Chen, Liu, Chai & Shi, arXiv:2309.02825).
 *
 * The library advances the transformed diffusion equation theta_t = nu lap theta
 * (Sec. II, Cole-Hopf transformation of the coupled Burgers equations) with the
 * D1Q3 / D2Q9 / D3Q19 / D4Q33 natural-moment MRT-LB model of Sec. III.A, using the
 * relaxation rates and weights of Theorem 2 (Sec. III.D) that make the scheme
 * and the velocity u = -2 nu grad(theta)/theta fourth-order accurate.  All
 * arithmetic is IEEE double precision on the GPU.  Boundaries are periodic;
 * a 1-D solver can instead span a closed interval whose end nodes carry a
 * given theta (LB_FLAG_BOUNDED, Example 1 of Sec. IV).
 *
 * Conventions shared by every entry point
 *   - Every function returns lb_status: LB_OK (0) or a negative error code.
 *     No C++ exception crosses the ABI.  lb_last_error() returns a message
 *     for the last failure on the calling thread.
 *   - Device memory is owned by the caller (plain device pointers, e.g. from
 *     torch tensors).  A solver borrows the pointers given to it and must be
 *     destroyed before they are freed.  The library owns only its host-side
 *     solver object and a few small device tables (parameters, reduction
 *     partials), allocated at creation (lb_adjoint_segment grows a table
 *     of per-launch partials on demand) and freed by lb_destroy.
 *   - Work is enqueued asynchronously on the HIP stream given at creation
 *     (NULL = the default stream); the host returns before the GPU finishes.
 *   - One solver or batch object must not be used from two host threads at
 *     once (it keeps its buffer roles and tables); separate objects are
 *     independent and may run on different threads and streams.
 *   - Grid: n[a] nodes along x_a (x_0 fastest); unused dimensions must be 1.
 *     Node index k = x0 + n0*(x1 + n1*(x2 + n2*x3)), V = n0*n1*n2*n3 nodes,
 *     node spacing dx, time step dt, lattice speed c = dx/dt, eps = nu*dt/dx^2.
 *   - Dense fields: theta is V doubles; a vector field (grad theta, u) is
 *     d planes of V doubles (component a = along x_a) back to back.
 *   - State buffers hold the q populations of every node in a chunked
 *     structure-of-arrays order: node indices are grouped in chunks of
 *     C = lb_state_chunk() = 4096 consecutive nodes, and inside a chunk the
 *     q populations follow one another as runs of C doubles, so population i
 *     of node k is element ((k / C) * q + i) * C + k % C.  V is rounded up to
 *     whole chunks (lb_state_elements); slots of nodes >= V are never read.
 *     Storage layout of a state ("stream-shifted"): the slot of population i
 *     at node k holds f_i(k + e_i), the pre-collision population of node
 *     k + e_i at the current time (the value node k sent along e_i after its
 *     last collision), so the distribution at node x is f_i(x) = buf_i(x - e_i).
 *   - Distribution-shaped adjoint buffers (lambda) use the same chunked order
 *     with canonical node positions: the slot of population i at node k is
 *     d L / d f_i(node k) for the pre-collision f.  lb_layout_from_dense and
 *     lb_layout_to_dense convert such buffers to and from q x V arrays.
 *   - Velocity order (Sec. III.A): D1Q3 (0, +1, -1); D2Q9 (0,0) (1,0) (0,1)
 *     (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1); D3Q19 rest, +x, +y, +z, -x,
 *     -y, -z, then the xy, xz, yz edges each as (+,+) (-,+) (-,-) (+,-);
 *     D4Q33 (general rule of Sec. III.A for d > 3) rest, +x_0..+x_3,
 *     -x_0..-x_3, then for every axis pair a < b in lexicographic order
 *     (e_a, e_b) = (+,+) (-,+) (-,-) (+,-).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_ERR_INVALID_ARG = -1, /* bad dimension/size/spacing, NULL pointer, ... */
    LB_ERR_UNSTABLE = -2,    /* eps above the lattice's stability limit (von Neumann
                                spectral radius > 1): D2Q9 0.48, D3Q19 1/4 and
                                D4Q33 1/6 (w1 >= 0); D1Q3 has none */
    LB_ERR_NONFINITE = -3,   /* a non-finite or non-positive theta was found */
    LB_ERR_OOM = -4,         /* the library could not allocate its small tables */
    LB_ERR_HIP = -5,         /* a HIP runtime call failed */
    LB_ERR_STATE = -6        /* call out of order (e.g. lb_step before lb_init) */
} lb_status;

typedef struct lb_solver lb_solver; /* opaque, library-owned host object */
typedef struct lb_batch lb_batch;   /* opaque, library-owned host object */

typedef struct {
    int32_t dim;     /* 1, 2, 3 or 4 */
    int32_t flags;   /* 0 (periodic) or LB_FLAG_BOUNDED */
    int64_t n[4];    /* nodes per axis, >= 1; n[a] = 1 for a >= dim */
    double dx;       /* node spacing, > 0 */
    double dt;       /* time step, > 0 */
    double nu;       /* viscosity of the Burgers equations (Sec. II), > 0 */
} lb_config;

/* lb_config.flags: the n[0] nodes x_j = j dx, j = 0..n[0]-1, of a 1-D grid
 * span a closed interval with both end nodes on the boundary, where theta is
 * prescribed (Example 1 of Sec. IV: the Burgers velocity vanishes there and
 * theta follows from the exact solution).  After each push the one population
 * that would enter an end node from outside takes the value that makes
 * sum_i f_i equal that node's boundary theta.  Requires dim = 1 and
 * n[0] >= 2.  Such a solver steps with lb_step_bounded; lb_step,
 * lb_step_buffers, lb_macro_buffer, lb_theta_from_velocity and the adjoint
 * calls return LB_ERR_STATE, and the batched form rejects the flag. */
#define LB_FLAG_BOUNDED 1

/* Relaxation rates and weights of Theorem 2 (Sec. III.D) for a config:
 * s1 = 2/(6 eps + 1), s21 = 24 eps/(6 eps + 1)^2 (s2 when d = 1),
 * s22 = 4/(6 eps + 3), w0, w1 = 1/6 - (d-1) eps/3 (1/6 for d = 1),
 * w_{1+2d} = eps/6 (0 for d = 1).  out[0..6] = eps, s1, s21, s22, w0, w1, wd. */
lb_status lb_parameters(const lb_config* cfg, double* out7);

/* Number of populations q = 1 + 2 d^2 (3, 9, 19, 33) for dim = 1..4 (0 otherwise). */
int32_t lb_num_populations(int32_t dim);

/* Nodes per chunk of the state layout (4096). */
int64_t lb_state_chunk(void);

/* Elements (doubles) of one state buffer: q * ceil(V / 4096) * 4096.
 * Returns 0 for an invalid config. */
int64_t lb_state_elements(const lb_config* cfg);

/* Bytes of one state buffer: lb_state_elements(cfg) * sizeof(double).
 * Returns 0 for an invalid config. */
size_t lb_state_bytes(const lb_config* cfg);

/* Create a solver over two caller-owned state buffers of lb_state_bytes each
 * (ping-pong; f_a and f_b must not overlap).  hip_stream is a hipStream_t or
 * NULL.  Validates the config (LB_ERR_INVALID_ARG, LB_ERR_UNSTABLE). */
lb_status lb_create(const lb_config* cfg, void* hip_stream, double* f_a, double* f_b,
                    lb_solver** out);

/* Initial state from theta0 (V doubles) and grad theta0 (d x V, or NULL):
 * f_i = w_i theta0 - dt Lambda^{-1} Dbar f^eq with Lambda^{-1} = M^-1 S^-1 M
 * (Sec. IV initialisation, first two terms of the expansion of Theorem 1),
 * in closed form f_i = w_i theta0 - dx w_i (e_i . g)
 *                      - (1/s1 - 1)(dx/6) sum_a (delta_{i,+a} - delta_{i,-a}) g_a.
 * With grad_theta0 == NULL, g is the fourth-order central difference
 * (-theta(x+2) + 8 theta(x+1) - 8 theta(x-1) + theta(x-2)) / (12 dx).
 * Writes f_a and resets the step counter.  If check_theta != 0 the call also
 * verifies theta0 > 0 and finite (Cole-Hopf needs theta > 0, Sec. II) and
 * returns LB_ERR_NONFINITE otherwise; the check synchronises the stream.
 * LB_FLAG_BOUNDED: grad_theta0 is required (LB_ERR_INVALID_ARG if NULL), and
 * theta0 at the two end nodes becomes the boundary theta of time 0. */
lb_status lb_init(lb_solver* s, const double* theta0, const double* grad_theta0,
                  int32_t check_theta);

/* Burgers front end: theta0 (V) and, if grad != NULL, grad theta0 (d x V)
 * from the initial velocity u0 (d x V) of the coupled Burgers equations, by
 * the inverse of the Cole-Hopf transformation u = -2 nu grad(theta)/theta
 * (Sec. II): theta0 = exp(-phi/(2 nu)) with grad(phi) = u0 and phi = 0 at the
 * origin, so theta0(origin) = 1 (theta is defined up to a constant factor,
 * which does not change u).  phi is integrated along x_0 at x_1 = .. = 0, then
 * along x_1 at x_2 = .. = 0, and so on, each cell with the four-node cubic
 * rule dx (-u_{j-1} + 13 u_j + 13 u_{j+1} - u_{j+2})/24 (fourth order);
 * grad theta0 = -u0 theta0/(2 nu) exactly.  u0 must be a periodic gradient
 * field (the potential symmetry of Sec. II) whose line integrals over a
 * period vanish; otherwise theta0 is not periodic.  Allocates and frees a
 * workspace of about V doubles and synchronises the stream. */
lb_status lb_theta_from_velocity(lb_solver* s, const double* u0, double* theta0, double* grad);

/* Advance nsteps >= 0 time steps (evolution equation of Sec. III.A: collide in
 * moment space, then stream), alternating the two buffers.  How the steps are
 * grouped into launches (passes of several steps, see LB_OPT_STEPS_PER_PASS;
 * on 1-D grids of up to 2048 nodes the whole run in one launch) never changes
 * the result: it is bitwise that of single steps.
 * The relaxation rates of Theorem 2 send the third-order moments to their
 * equilibrium (zero) at rate 1, so after every collision the two opposite
 * edge populations of each pair of axes are equal (f for (-1,-1) equals f for
 * (+1,+1), f for (+1,-1) equals f for (-1,+1)).  Launches inside one call
 * (D2Q9, D3Q19, D4Q33) therefore store only the other populations and read
 * each such twin from its partner's plane; the last launch of the call, and a
 * launch that ends with a check (LB_OPT_CHECK_INTERVAL), store all of them, so
 * the current state between calls is always complete.  The first launch of a
 * call reads twins from their partners too unless the state came from lb_init
 * or lb_set_state: a caller that changes the current buffer in place must go
 * through lb_set_state.  After an LB_ERR_HIP return (a launch that failed)
 * the current state is unspecified and must be set again. */
lb_status lb_step(lb_solver* s, int64_t nsteps);

/* LB_FLAG_BOUNDED solvers: advance nsteps >= 0 time steps on the interval.
 * walls is a device array of 2 * nsteps doubles, the boundary theta
 * (left end, right end) at t + dt, t + 2 dt, ..., t + nsteps dt, where t is
 * the current time; the last pair is kept as the boundary theta of the new
 * current time (used by lb_macro and lb_get_state).  Grids of up to 2048
 * nodes run all steps in one launch with the state in LDS.  LB_ERR_STATE on a
 * periodic solver or before lb_init / lb_set_state. */
lb_status lb_step_bounded(lb_solver* s, int64_t nsteps, const double* walls);

/* Options of a solver (lb_set_option).
 * LB_OPT_STEPS_PER_PASS (default 8): the most time steps lb_step advances with
 * one pass over the state in HBM (temporal blocking: the intermediate steps
 * stay on chip).  D2Q9: a run of nsteps is split greedily into passes of 8,
 * 4 and 2 steps (within the limit) and single steps; one wave marches down a
 * strip of columns, neighbouring columns exchange populations by lane shifts
 * and rows are delayed in registers.  D3Q19: passes of 2 steps (x-y tiles
 * marching along z, populations exchanged through LDS) and a single step for
 * an odd remainder, whenever the limit is 2 or more.  Values below 2 make
 * every step a separate launch; others are rounded down to 2, 4 or 8.  D1Q3
 * and D4Q33 take single steps.  Every grouping gives bitwise the result of
 * single steps.  Unknown options are LB_ERR_INVALID_ARG.
 *
 * LB_OPT_CHECK_INTERVAL (default 0 = off): failure detection while stepping.
 * With value k > 0, lb_step counts the steps it runs (across calls; lb_init
 * and lb_set_state restart the count) and, at the end of the first launch
 * that brings the count to k or more, checks theta = sum_i f_i at every node
 * of the current state and restarts the count.  If some theta is not finite
 * or not positive (a diverged run, or a corrupted state: the Cole-Hopf
 * velocity divides by theta, Sec. II), lb_step returns LB_ERR_NONFINITE at
 * once; the state and step counter are those after that launch.  A check
 * reads the state once and synchronises the stream.  Bounded solvers
 * (lb_step_bounded) are not checked. */
enum { LB_OPT_STEPS_PER_PASS = 1, LB_OPT_CHECK_INTERVAL = 2 };
lb_status lb_set_option(lb_solver* s, int32_t option, int32_t value);

/* One time step from an explicit source buffer to an explicit destination
 * buffer (both in the storage layout, lb_state_bytes each, not overlapping).
 * Does not touch the solver's own buffers or step counter. */
lb_status lb_step_buffers(lb_solver* s, const double* src, double* dst);

/* Buffer that holds the current state (f_a or f_b) and the steps taken. */
double* lb_current_state(const lb_solver* s);
int64_t lb_steps_taken(const lb_solver* s);

/* Macroscopic output at the current time t = steps * dt from the
 * pre-collision distribution (Sec. III.C):
 *   theta        = sum_i f_i,
 *   grad_theta_a = -(s1/(dt c_s^2)) sum_i c_{ia} f^ne_i,  f^ne = f - w theta,
 *                  the fourth-order gradient read from the non-equilibrium
 *                  first moment (Theorem 1 and the formula after it);
 *                  c_s^2 = c^2/3 on every lattice here,
 *   u_a          = -2 nu grad_theta_a / theta = (2 - s1) sum_i c_{ia} f^ne_i / theta
 *                  (Cole-Hopf, Sec. II; the two forms agree since 2 - s1 = 6 eps s1).
 * theta (V), u (d x V) and grad_theta (d x V, component a along x_a) may each
 * be NULL; with all three NULL the call does nothing.  LB_FLAG_BOUNDED: the
 * end nodes' distribution is completed with the current boundary theta, so
 * theta there equals it. */
lb_status lb_macro(lb_solver* s, double* theta, double* u, double* grad_theta);

/* Same as lb_macro for an explicit state buffer in the storage layout. */
lb_status lb_macro_buffer(lb_solver* s, const double* state, double* theta, double* u,
                          double* grad_theta);

/* Copy the current pre-collision distribution to f_out in the dense
 * canonical layout (q planes of V doubles, f_out[i*V + k] = f_i(node k)).
 * LB_FLAG_BOUNDED: the population entering each end node is the one the
 * boundary theta determines. */
lb_status lb_get_state(lb_solver* s, double* f_out);

/* Load a dense canonical distribution (q x V) as the current state and set
 * the step counter to step.  LB_FLAG_BOUNDED: the boundary theta of the
 * current time becomes sum_i f_i at each end node, and the population
 * entering an end node is kept only through that sum (lb_get_state returns
 * it to rounding). */
lb_status lb_set_state(lb_solver* s, const double* f_in, int64_t step);

/* Copy a dense q x V array (dense[i*V + k] for population i of node k) into
 * a buffer of lb_state_elements in the chunked order, without any stream
 * shift, and back.  Used for distribution-shaped adjoint buffers. */
lb_status lb_layout_from_dense(lb_solver* s, const double* dense, double* buf);
lb_status lb_layout_to_dense(lb_solver* s, const double* buf, double* dense);

/* ---------------------------------------------------------------------- */
/* Discrete adjoint (reverse mode).  The forward map is f^{n+1} = P C f^n
 * with the per-node collision C = I - M^-1 S M (I - w 1^T) (Sec. III.A) and
 * the streaming permutation P.  g_eps is one device double that every
 * adjoint call increments (+=) by a deterministic reduction; with
 * eps = nu dt / dx^2, dL/dnu = (dt/dx^2) dL/deps.                          */
/* ---------------------------------------------------------------------- */

/* Adjoint of lb_macro_buffer at the state buffer `state`: given g_theta
 * (V, may be NULL) and g_u (d x V, may be NULL) writes lambda = dL/df
 * (canonical node positions, chunked order) and adds the explicit eps
 * dependence of u (through s1) to *g_eps. */
lb_status lb_macro_adjoint(lb_solver* s, const double* state, const double* g_theta,
                           const double* g_u, double* lambda, double* g_eps);

/* One reverse step: state_n is f^n in the storage layout (as written by
 * lb_init/lb_step_buffers), lambda_in = dL/df^{n+1}, lambda_out = dL/df^n
 * (= C^T P^T lambda_in), both canonical and not overlapping; adds
 * <P^T lambda_in, (dC/deps) f^n> to *g_eps. */
lb_status lb_adjoint_step(lb_solver* s, const double* state_n, const double* lambda_in,
                          double* lambda_out, double* g_eps);

/* One checkpoint segment of the reverse sweep, driven from the library (the
 * sqrt(T) checkpointing of the discrete adjoint).  ckpt holds f^{n0} in the
 * storage layout; the call recomputes f^{n0+1} .. f^{n0+m-1} into `work`
 * (m - 1 consecutive state buffers of lb_state_bytes each; may be NULL when
 * m = 1), bitwise as single steps would (on D2Q9 by multi-step passes that
 * store every step, up to LB_OPT_STEPS_PER_PASS steps each) except that the
 * twin populations (lb_step) are not stored: they equal their partners and
 * are read from there, so work is scratch whose twin planes keep whatever
 * they held before.  It then applies
 * the adjoint steps for n = n0+m-1 down to n0.  lambda holds dL/df^{n0+m}
 * on entry and dL/df^{n0} on return; lambda_tmp is a second state buffer
 * used as the ping-pong partner.  lambda on return is bitwise that of m
 * lb_adjoint_step calls.  On D2Q9 the reverse sweep runs in passes of up to
 * min(4, LB_OPT_STEPS_PER_PASS) adjoint steps (the forward passes' one-wave
 * march with every velocity reversed); each wave sums the eps parts of its
 * nodes in a fixed order, so *g_eps is deterministic but rounded differently
 * from the single calls.  Other lattices take one adjoint step per launch
 * and *g_eps is bitwise that of the single calls.  None of the buffers may
 * overlap.  Errors: NULL pointers, m < 0, a bounded solver,
 * LB_ERR_HIP if the partials table cannot grow to m tables. */
lb_status lb_adjoint_segment(lb_solver* s, const double* ckpt, int64_t m, double* work,
                             double* lambda, double* lambda_tmp, double* g_eps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * segment as lb_adjoint_segment, with the same arguments and bitwise the
 * same lambda and *g_eps, but the per-launch partials tables live in a fixed
 * device array of LB_SEGMENT_SCRATCH_DOUBLES doubles (16 MiB) that the
 * library declares at file scope, so the call allocates and frees nothing.
 * Each GPU holds its own copy of that array from the moment the library is
 * loaded until the process ends; its address on a device is looked up when
 * a solver is created there.  A segment of m steps needs nt * (T+1)
 * doubles: on D2Q9 T is the larger of the reverse passes' block count (64-wide
 * strips times row segments) and the per-node kernels' block count B, and nt
 * is the number of reverse launches, at most ceil((m-1)/4) + 2 with the
 * default LB_OPT_STEPS_PER_PASS (m when it is 1); on the other lattices
 * T = B and nt = m.  A segment needing more returns
 * LB_ERR_INVALID_ARG before anything is launched (use lb_adjoint_segment or
 * shorter segments).  Every entry of the tables is written before it is
 * read, so nothing needs clearing between calls.  All solvers on one GPU
 * share its array: calls of this function that overlap in time on one GPU
 * (different host threads, or different streams whose work overlaps) race
 * and give wrong gradients; serialise them. */
#define LB_SEGMENT_SCRATCH_DOUBLES (2 * 1024 * 1024)
lb_status lb_adjoint_segment_static(lb_solver* s, const double* ckpt, int64_t m, double* work,
                                    double* lambda, double* lambda_tmp, double* g_eps);

/* Adjoint of lb_init: given lambda0 = dL/df^0 (canonical) writes g_theta0 (V).
 * If grad_theta0 != NULL the gradient input was independent and its adjoint
 * is written to g_grad (d x V, may be NULL); if grad_theta0 == NULL the
 * fourth-order difference stencil is transposed into g_theta0.  theta0 and
 * grad_theta0 are the inputs given to lb_init; the eps dependence of the
 * initial state is added to *g_eps.  This is the last call of a reverse
 * sweep, so g_nu (one device double, may be NULL) then receives
 * dL/dnu = (dt/dx^2) * (*g_eps), the whole gradient with respect to the
 * viscosity (eps = nu dt/dx^2 is the only place nu enters the scheme).
 * g_nu must not be g_eps. */
lb_status lb_init_adjoint(lb_solver* s, const double* theta0, const double* grad_theta0,
                          const double* lambda0, double* g_theta0, double* g_grad,
                          double* g_eps, double* g_nu);

/* Destroy a solver (does not free the caller's buffers).  NULL is allowed. */
lb_status lb_destroy(lb_solver* s);

/* ---------------------------------------------------------------------- */
/* Batched form: many independent 2-D periodic instances of different sizes
 * and viscosities advanced together.  Instance b occupies elems_b elements
 * (its own chunked state) starting at element offset_b of the pool.         */
/* ---------------------------------------------------------------------- */

/* Total pool elements (doubles) for count 2-D configs; offsets (count) and
 * elems (count) receive each instance's first element and element count.
 * Either output may be NULL.  Returns -1 on an invalid config. */
int64_t lb_batch_layout(const lb_config* cfgs, int32_t count, int64_t* offsets,
                        int64_t* elems);

/* Create a batch over two caller-owned pools of lb_batch_layout elements
 * each.  Only dim = 2 configs are accepted. */
lb_status lb_batch_create(const lb_config* cfgs, int32_t count, void* hip_stream,
                          double* pool_a, double* pool_b, lb_batch** out);

/* Initialise every instance: theta0 and grad are packed pools, instance b's
 * theta0 at element node_offset_b (prefix sum of V_b) and its gradient at
 * 2*node_offset_b (two planes of V_b).  grad may be NULL (fourth-order
 * differences per instance). */
lb_status lb_batch_init(lb_batch* b, const double* theta0, const double* grad);

/* Tile shape of the batched step (Sec. III.A scheme, the same arithmetic in
 * every mode, so all modes give bitwise identical states):
 *   (-S, rows)  S = 2, 4 or 8 steps per pass over each instance: tiles of
 *               128 - 2S columns x rows rows (1 <= rows <= 65535) that keep
 *               the intermediate steps on chip (two waves per tile, sharing
 *               through LDS); a run of n steps takes n / S such passes and
 *               n mod S linear-tile single steps.  (-8, 64) is the default of
 *               a new batch;
 *   (-16-S, rows)  the same with tiles of 64 - 2S columns, one wave per tile
 *               (the march of lb_step's D2Q9 passes);
 *   (0, 0)      one step per pass, linear tiles of 256 consecutive node
 *               indices of one instance (crossing row ends);
 *   (tx, ty)    one step per pass, tx x ty rectangles with tx*ty = 256 and tx
 *               a power of two in [16, 256].
 * Applies to subsequent steps; cached graphs are dropped.  Anything else is
 * LB_ERR_INVALID_ARG. */
lb_status lb_batch_set_tile(lb_batch* b, int32_t tx, int32_t ty);

/* Time candidate tile shapes, one-step and multi-step, per step on the real
 * pools (the current state is left as it was; the other pool is used as
 * scratch and holds no meaningful values afterwards) and keep the fastest;
 * best_tx/best_ty receive the choice (may be NULL).  The trials time the
 * launches that a step call runs between its first and its last. */
lb_status lb_batch_autotune(lb_batch* b, int32_t steps_per_trial, int32_t* best_tx,
                            int32_t* best_ty);

/* Advance every instance nsteps.  With use_graph != 0 the nsteps launches
 * are captured once into a hipGraph (cached per nsteps, starting pool and
 * whether that pool came from lb_batch_init, up to 16 graphs; capturing a 17th
 * first waits for the batch's stream and clears the cache) and replayed with a
 * single hipGraphLaunch.  Launches store twin populations as in lb_step: only
 * the last launch of a call stores all of them, and the first reads them from
 * their partners unless the pool came from lb_batch_init. */
lb_status lb_batch_step(lb_batch* b, int64_t nsteps, int32_t use_graph);

/* theta (packed V_b per instance) and u (packed 2 x V_b per instance, at
 * 2*node_offset_b); either may be NULL. */
lb_status lb_batch_macro(lb_batch* b, double* theta, double* u);

/* Current pool (pool_a or pool_b) and steps taken.  The pool is complete
 * between calls; it is for reading (a changed pool is taken up by
 * lb_batch_init only). */
double* lb_batch_current(const lb_batch* b);
/* Waits for the batch's stream, then frees the cached graphs and tile tables
 * (the pools stay the caller's).  NULL is accepted. */
lb_status lb_batch_destroy(lb_batch* b);

/* Message for the last error on the calling thread ("" if none). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
