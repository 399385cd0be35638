/*
 * lbrs.h -- C ABI of the MI355X (gfx950) implementation of the Lattice
 * Boltzmann Relaxation Scheme (LBRS) for the inviscid gamma-law Euler
 * equations and for scalar laws with quadratic fluxes (Burgers, advection):
 * S. V. Raghurama Rao, R. Deshmukh, S. Kotnala, "A Lattice
 * Boltzmann Relaxation Scheme for Inviscid Compressible Flows",
 * arXiv 1504.07034.
 *
 * The problem the calls solve is the paper's (Sec. II): evolve conserved
 * initial data U0 with the discrete-velocity BGK model whose equilibria are
 * algebraic in U and the flux G(U),
 *     f_i(x + lambda_i dt, t + dt) = (1 - omega) f_i(x, t) + omega f_i^eq(x, t),
 * with exact hopping (lambda dt = dx), then read back U = sum_i f_i.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * All arithmetic is IEEE FP64.  All large buffers are DEVICE pointers that
 *    the caller allocates and owns; the library borrows them until
 *    lbrs_destroy().  The library allocates only its small host-side context
 *    (with, for a context whose fused calls read state back, a pinned host
 *    buffer of under 1 KiB; see lbrs_init).
 *  * Layouts (C order, x fastest):
 *      U  (conserved)  : K planes [K][ny][nx]; K = 3 in 1D (rho, rho u, rho E),
 *                        K = 4 in 2D (rho, rho u, rho v, rho E), K = 1 for a
 *                        scalar law (u)
 *      W  (primitive)  : [K][ny][nx] = (rho, u, p) or (rho, u, v, p), or u
 *      f  (populations): Q*K planes p = i*K + k, velocity order as in the
 *                        paper: D1Q2 (-,+), D1Q3 (-,0,+),
 *                        D2Q4 (-,-), (+,-), (+,+), (-,+); element (p, y, x) at
 *                          LBRS_LAYOUT_PLANAR: (p*ny + y)*nx + x   [Q][K][ny][nx]
 *                          LBRS_LAYOUT_ROWS  : (y*Q*K + p)*nx + x  [ny][Q][K][nx]
 *                        and, in 1D, LBRS_LAYOUT_ROWS is blocked by 64 cells:
 *                          (x/64*Q*K + p)*64 + x%64   [nx/64][Q][K][64]
 *                        (last block padded).  Population-shaped buffers
 *                        of a context (f0, f1, lbrs_get_f/lbrs_set_f, the
 *                        adjoint's fbar) all use the context's layout.
 *    Pointers must be 8-byte aligned (hipMalloc / torch allocations are
 *    256-byte aligned).
 *  * Grid: cell-centred, dx = (x1-x0)/nx, dy = (y1-y0)/ny; 2D requires
 *    dx == dy (the D2Q4 populations hop along cell diagonals).
 *  * Every call that enqueues work does so on the context's HIP stream and
 *    returns without synchronising, except those whose description says
 *    that they wait for the stream (lbrs_get_state(), the counters and
 *    reports, fused PER_STEP lbrs_step() calls, a body's lbrs_init(), ...).
 *  * Return codes: LBRS_OK (0) or a negative lbrs_status; lbrs_strerror()
 *    names them.  An invalid argument is rejected before anything is
 *    enqueued.  A non-physical state (rho <= 0, p <= 0 or a non-finite value;
 *    for a scalar law a non-finite value) met on the device stops the time
 *    loop at that step and is reported by the next lbrs_get_state() as
 *    LBRS_E_NONPHYSICAL with the step index.
 */
#ifndef LBRS_H
#define LBRS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbrs_ctx lbrs_ctx; /* opaque host-side handle */

typedef enum {
    LBRS_OK = 0,
    LBRS_E_INVAL = -1,       /* bad parameter, size or pointer */
    LBRS_E_NOMEM = -2,       /* host allocation failed */
    LBRS_E_HIP = -3,         /* a HIP runtime call failed */
    LBRS_E_NONPHYSICAL = -4, /* rho <= 0, p <= 0 or non-finite state met */
    LBRS_E_STATE = -5        /* call not valid for this context's mode */
} lbrs_status;

/* Discrete-velocity models (Sec. II.A D1Q2, Sec. II.C D1Q3, Sec. II.D D2Q4). */
enum { LBRS_D1Q2 = 0, LBRS_D1Q3 = 1, LBRS_D2Q4 = 2 };

/* Side conditions, given per side in the order x-low, x-high, y-low, y-high.
 * WALL is the paper's free-slip wall by specular reflection (Sec. II.E), with
 * the wall on the first/last node row or column; walls on two perpendicular
 * sides (a corner) are rejected unless a body mask is given (lbrs_params.solid,
 * whose corner rules then apply).  TRANSMISSIVE (zero gradient of the
 * post-collision populations) and PERIODIC are not in the paper.  PERIODIC
 * must be set on both sides of an axis.  DIRICHLET prescribes the state
 * beyond a side (the inflow and post-shock top boundaries of the paper's
 * oblique-shock reflection case, Sec. III, whose treatment the paper does not
 * spell out): the ghost cells across it hold the given conserved states in
 * equilibrium at the step's lattice speed, so every population pulled from
 * across the side is f^eq_i(U_b); at a corner ghost cell the y-side's state
 * applies; the prescribed states enter the global lambda* like interior
 * cells.  DIRICHLET is available for D2Q4 single domains (lbrs_init) and
 * needs lbrs_params.dirichlet for that side.  1D models accept TRANSMISSIVE
 * and PERIODIC on x only. */
enum { LBRS_BC_TRANSMISSIVE = 0, LBRS_BC_PERIODIC = 1, LBRS_BC_WALL = 2, LBRS_BC_DIRICHLET = 3 };

/* Conservation law.  EULER: the gamma-law Euler equations (K = 3 conserved
 * components in 1D, 4 in 2D).  SCALAR: one conserved scalar u (K = 1) with the
 * quadratic fluxes g1(u) = c0 u + c1 u^2/2 and g2(u) = c2 u + c3 u^2/2,
 * c = lbrs_params.scalar_flux: the scalar LBRS the paper starts from
 * (Sec. II.A, Burgers: c = (0, 1, ., .)), its D2Q4 form (Sec. II.D; the 2D
 * Burgers law of the Sec. III test cases: c = (0, 1, 1, 0)), linear advection
 * (c1 = c3 = 0).  Equilibria match u = sum f_i and g = sum lambda_i f_i; the
 * local bound is |g'(u)| in 1D and |g1'(u)| + |g2'(u)| in 2D.  SCALAR takes
 * TRANSMISSIVE, PERIODIC and DIRICHLET sides (no WALL; in 1D DIRICHLET on the
 * x-sides), and the calls lbrs_init, lbrs_step, lbrs_get_state, lbrs_moments,
 * lbrs_get_f, lbrs_set_f, lbrs_prim_to_cons (a copy: u is its own conserved
 * variable) and lbrs_set_tile; the gradient calls are Euler-only
 * (LBRS_E_STATE / LBRS_E_INVAL), and so are the batches. */
enum { LBRS_LAW_EULER = 0, LBRS_LAW_SCALAR = 1 };

/* Lattice speed.  PER_STEP: every step takes the global bound
 * lambda* = max over cells of the local bound (Sec. II.C Jin-Xin choice in 1D,
 * Sec. II.D Bouchut condition in 2D), dt = min(cfl*dx/lambda*, t_end - t) and
 * the lattice speed dx/dt.  FROZEN_INIT: the lattice speed lambda*(U0)/cfl is
 * fixed at lbrs_init (dt = dx/lambda, no clipping at t_end) -- the mode the
 * adjoint calls need.  USER: the fixed lattice speed lambda_user. */
enum { LBRS_LAMBDA_PER_STEP = 0, LBRS_LAMBDA_FROZEN_INIT = 1, LBRS_LAMBDA_USER = 2 };

/* Population layouts.  PLANAR: plane p (= i*K + k) of cell (x, y) at
 * p*nx*ny + y*nx + x.  ROWS in 2D keeps the 16 D2Q4 population rows of a grid
 * row in one contiguous block, [y][p][x], so the 2D step touches two memory
 * pages per row instead of 32; ROWS in 1D keeps the Q*K planes of each block
 * of 64 cells contiguous, [x/64][p][x%64], the last block padded (f_bytes
 * covers the padding): the long-tube Euler step reads and writes nine planes
 * per cell and runs ~15% faster blocked; scalar laws (two or three planes)
 * run faster planar. */
enum { LBRS_LAYOUT_PLANAR = 0, LBRS_LAYOUT_ROWS = 1 };

typedef struct {
    int model;            /* LBRS_D1Q2, LBRS_D1Q3 or LBRS_D2Q4 */
    int nx, ny;           /* cells; ny = 1 for 1D; nx >= 3 (and ny >= 3 in 2D) */
    double x0, x1, y0, y1;/* domain; y0, y1 ignored in 1D */
    double gamma;         /* ratio of specific heats, > 1 (Euler) */
    double omega;         /* relaxation parameter omega = dt/epsilon, in (0, 2) (Sec. II.B) */
    double cfl;           /* in (0, lbrs_cfl_max(model)]: lattice speed = (lambda star) / cfl */
    int bc[4];            /* side conditions, x-low, x-high, y-low, y-high */
    int lambda_mode;      /* LBRS_LAMBDA_* */
    double lambda_user;   /* lattice speed for LBRS_LAMBDA_USER, > 0 */
    int layout;           /* LBRS_LAYOUT_PLANAR (0) or LBRS_LAYOUT_ROWS (1) */
    /* Per side, the prescribed conserved states of a DIRICHLET side: device
     * pointer to [K][n] doubles along the side, n = ny for the x-sides (index
     * = row y) and n = nx for the y-sides (index = column x); NULL for other
     * sides.  Borrowed: the caller keeps the data alive and unchanged while
     * the context exists.  A non-admissible prescribed state is reported
     * like a non-admissible U0 (LBRS_E_NONPHYSICAL at step 0). */
    const double* dirichlet[4];
    int law;              /* LBRS_LAW_EULER (0) or LBRS_LAW_SCALAR (1) */
    double scalar_flux[4];/* SCALAR: c0..c3 of g1(u) = c0 u + c1 u^2/2, g2(u) = c2 u + c3 u^2/2 */
    /* Solid body (D2Q4 Euler single domains): HOST pointer to nx*ny bytes,
     * row-major [y][x], nonzero = solid cell; NULL = no body.  Read by
     * lbrs_init and lbrs_body_codes only.  The Sec. III cases with a body
     * (forward-facing step, backward-facing step of the shock diffraction,
     * ramp) do not give the geometry: it is the caller's mask.  The wall runs
     * through the fluid nodes next to the body, as on a WALL side: a
     * population whose pull source is solid takes the same-node specular
     * image that cancels the normal flux (the Sec. II.E rule) -- across a face
     * (the source's x- or y-neighbour solid) the mirror population with that
     * momentum component negated, in a concave corner (both neighbours solid)
     * the opposite population with both negated, at a convex corner tip (only
     * the diagonal source solid) the opposite population reflected about the
     * corner's bisector (momentum components swapped, times -s_x s_y).
     * Beyond a WALL side every position is solid; elsewhere positions outside
     * the grid are wrapped or clamped onto it and the mask decides.  With a
     * body, WALL sides may meet at corners.  Solid cells hold zero
     * populations, read U = 0 and take no part in lambda* or the
     * admissibility check (their U0 is ignored).  A mask whose image
     * populations would themselves come from solid positions (a fluid gap one
     * cell wide) or with no fluid cell is rejected (LBRS_E_INVAL at
     * lbrs_init).  Body contexts march one way (lbrs_set_tile's alternate must
     * be 0) and have no gradient calls (LBRS_E_STATE). */
    const unsigned char* solid;
} lbrs_params;

/* Sizes in bytes of one population buffer (f0 or f1), of one conserved-state
 * buffer (U, K planes) and of the device scratch area lbrs_init needs (with a
 * body it also holds the 2-byte node codes, nx*ny of them).
 * Any output pointer may be NULL.  Returns LBRS_E_INVAL for invalid params. */
int lbrs_query_sizes(const lbrs_params* p, size_t* f_bytes, size_t* u_bytes,
                     size_t* scratch_bytes);

/* Largest admissible cfl of a model: 1 for D1Q2 and D2Q4, 2/3 for D1Q3.  With
 * the lattice speed (lambda star)/cfl the equilibria are monotone in U (Bouchut's
 * condition, Sec. II.D) when every eigenvalue of df_i^eq/dU is >= 0: for the
 * Sec. II.C D1Q3 equilibria U/3 -+ G/(2 lambda) that needs lambda >= 1.5
 * max |u -+ a|, for D1Q2 lambda >= max |u -+ a|, for D2Q4 lambda >= the
 * Sec. II.D bound.  lbrs_init, lbrs_query_sizes and the batch calls reject a
 * larger cfl (LBRS_E_INVAL) in the PER_STEP and FROZEN_INIT modes.  Returns
 * -1 for an unknown model.  Host only, no GPU needed. */
double lbrs_cfl_max(int model);

/* Node codes of p->solid, computed on the host (no GPU needed), as lbrs_init
 * stores them for the step kernel: h_codes receives nx*ny uint16 values,
 * [y][x]; bits 3i..3i+2 give the rule of population i (D2Q4 order
 * (-,-), (+,-), (+,+), (-,+)) -- 0 pulled, 1 face image across x (population
 * with s_x reversed, x-momentum negated), 2 face image across y, 3 concave
 * corner (opposite population, both momenta negated), 4 convex corner tip
 * (opposite population, momenta swapped times -s_x s_y) -- and bit 15 marks a
 * solid cell.  Returns LBRS_E_INVAL for invalid params, a NULL p->solid or an
 * inadmissible body. */
int lbrs_body_codes(const lbrs_params* p, unsigned short* h_codes);

/* Primitive -> conserved variables on the device: U = (rho, rho u, [rho v,]
 * rho E) with E = p/(rho(gamma-1)) + |u|^2/2 (Sec. II.C); for a scalar law a
 * copy (u is conserved).  d_W and d_U are [K][ny][nx]; they may not alias.
 * Enqueued on hip_stream (NULL = default). */
int lbrs_prim_to_cons(const lbrs_params* p, const double* d_W, double* d_U, void* hip_stream);

/* Create a context and set the populations to equilibrium, f^0 = f^eq(U0)
 * (Sec. II.A: the initial data are given to the populations through their
 * equilibria), with the lattice speed lambda*(U0)/cfl (or lambda_user);
 * lambda*(U0) includes the prescribed states of DIRICHLET sides.
 *   d_U0      [K][ny][nx] conserved initial state (read during this call's
 *             kernels only)
 *   d_f0,d_f1 two population buffers of f_bytes each (ping-pong; borrowed)
 *   d_scratch scratch_bytes of device memory (borrowed; holds t, the step
 *             count, the lambda* reduction slots and the status word)
 *   hip_stream the stream every later call enqueues on (NULL = default)
 * On success *out receives the context.  A non-physical U0 is reported by the
 * next lbrs_get_state() with step index 0.  With a body (p->solid) the node
 * codes are built on the host, copied into d_scratch and the stream is
 * synchronised before the call returns (an inadmissible mask: LBRS_E_INVAL,
 * nothing enqueued).  A 2D Euler context with PER_STEP speeds and no body or
 * DIRICHLET side also gets a pinned host buffer of under 1 KiB (hipHostMalloc)
 * through which fused calls read the state back between their rounds of
 * launches (see lbrs_set_fusion); lbrs_destroy frees it. */
int lbrs_init(lbrs_ctx** out, const lbrs_params* p, const double* d_U0, double* d_f0,
              double* d_f1, void* d_scratch, void* hip_stream);

/* Enqueue max_steps fused collide-and-stream steps (Sec. II.A discrete LBRS
 * update; Sec. II.D in 2D; walls Sec. II.E).  Each step reads the lattice
 * speed from the device, forms U, the flux, the equilibria, relaxes, streams
 * one node along every link, applies the side conditions and reduces the next
 * step's lambda* (with the prescribed states of DIRICHLET sides).  A step whose start time is >= t_end, or that follows a
 * non-physical step, does nothing, so the run stops exactly at t_end
 * (PER_STEP mode clips the last dt).  With lbrs_set_fusion(c, k), k = 2 to 4
 * (2D Euler), the steps run up to k per launch with the same results (see
 * there).
 * Asynchronous, except with fused launches and PER_STEP speeds on a stream
 * that is not being captured: the call then waits for the stream (see
 * lbrs_set_fusion).  A graph captured around single-step calls replays
 * consistently when max_steps is a multiple of six (one launch per step; see
 * lbrs_set_fusion for fused calls). */
int lbrs_step(lbrs_ctx* c, int max_steps, double t_end);

/* Wait for the stream and report the current time, completed step count,
 * the lattice speed of the last step taken (or of f^0 before any step) and
 * the status.  *status is 0 or a bit mask (1 = non-physical); *fail_step is
 * the index (1-based; 0 = the initial state) of the first non-physical state
 * or -1.  Any output pointer may be NULL.  Returns LBRS_E_NONPHYSICAL when the
 * status is set, LBRS_OK otherwise. */
int lbrs_get_state(lbrs_ctx* c, double* t, long long* nsteps, double* lambda,
                   unsigned* status, long long* fail_step);

/* Counters of the fused launches since lbrs_init (lbrs_set_fusion(c, k > 1)),
 * into counts[0 .. n-1] (n <= 14; missing ones 0): [0] launches of two or
 * more steps whose result stood, [1] such launches rolled back (a guessed
 * bound that was wrong), [2] launches that only reduced the bound of f^{n+1},
 * [3] one-step launches, [4] predictions of the next launch's bounds made,
 * [5] predicted bounds that stood, [6] predicted bounds rolled back,
 * [7] cells whose bound the predictions evaluated, [8] launches that listed
 * candidates but left no prediction (too many, none, or a non-physical
 * state), [9] candidates listed, [10] launches whose candidates overflowed
 * the list, [11] of [0], the three-step ones, [12] of [0], the four-step
 * ones (so the steps taken are 2 [0] + [11] + 2 [12] + [3]), [13] fused
 * step launches enqueued (counted on the host; those that found the work
 * done and exited at once included).  With per-step
 * lattice speeds a fused launch guesses the bounds of the states after its
 * first steps (the predictions when the launch before left them, else the
 * current bound while it keeps repeating) and the next launch checks every
 * guess bit for bit, so the counters describe cost only: results are those
 * of single steps.  Waits for the stream. */
int lbrs_pair_stats(lbrs_ctx* c, long long* counts, int n);

/* Moments of the current populations, U = sum_i f_i (eq. "moments_system"),
 * into d_U [K][ny][nx].  Asynchronous. */
int lbrs_moments(lbrs_ctx* c, double* d_U);

/* Copy the current populations to / from d_f [Q][K][ny][nx] (checkpoints).
 * lbrs_set_f also sets the time t and step count n, clears the status, and
 * (PER_STEP mode) re-reduces lambda* from the new populations. */
int lbrs_get_f(lbrs_ctx* c, double* d_f);
int lbrs_set_f(lbrs_ctx* c, const double* d_f, double t, long long n);

/* Objective for the gradient calls (2D only): J = sum of rho^2 over the cells
 * with i in [ix0, ix1) and j in [iy0, iy1), rho from the current populations.
 * Writes J to *d_J (one device double) and the seed of the adjoint,
 * dJ/df_{i,rho}(x) = 2 rho(x) inside the window and 0 elsewhere, to
 * d_fbar [Q][K][ny][nx].  Asynchronous. */
int lbrs_window_objective(lbrs_ctx* c, int ix0, int ix1, int iy0, int iy1, double* d_J,
                          double* d_fbar);

/* Forward step that also stores the step's input moments U^n into
 * d_Utape_n [K][ny][nx] (the tape the adjoint step reads).  2D Euler with
 * no body and no DIRICHLET side, FROZEN_INIT or USER mode only (else
 * LBRS_E_STATE); otherwise identical to lbrs_step(c, 1, +inf). */
int lbrs_step_tape(lbrs_ctx* c, double* d_Utape_n);

/* Two taped forward steps in fused launches (two steps per launch, as
 * lbrs_set_fusion(c, 2)): U^n goes to d_Utape_n and U^{n+1} to d_Utape_n1;
 * equal to two lbrs_step_tape calls to rounding.  Same modes and errors as
 * lbrs_step_tape; the tapes may not alias.  Asynchronous. */
int lbrs_step_tape2(lbrs_ctx* c, double* d_Utape_n, double* d_Utape_n1);

/* k taped forward steps (k = 1 .. 4) in one fused launch (as
 * lbrs_set_fusion(c, k); k = 1 is lbrs_step_tape): slot s of d_Utape
 * [k][K][ny][nx] receives U^{n+s}, the input moments of step s+1; equal to k
 * lbrs_step_tape calls to rounding.  Same modes and errors as
 * lbrs_step_tape, LBRS_E_INVAL for k outside 1 .. 4.  Asynchronous. */
int lbrs_step_tapes(lbrs_ctx* c, int k, double* d_Utape);

/* Adjoint (vector-Jacobian product) of one fixed-speed step, D2Q4 with
 * periodic sides: given fbar^{n+1} = dJ/df^{n+1} and the step's input moments
 * U^n, write fbar^n = dJ/df^n:
 *   fbar*_i(x) = fbar^{n+1}_i(x + s_i)                      (reverse stream)
 *   Ubar(x)    = omega [ (1/4) sum_i fbar*_i
 *                        + (A1(U^n)^T h_x + A2(U^n)^T h_y) / (4 lambda) ],
 *                h_d = sum_i s_{i,d} fbar*_i,  A_d = dG_d/dU   (D2Q4 equilibria)
 *   fbar^n_i   = (1 - omega) fbar*_i + Ubar                 (relaxation)
 * All arrays are [Q][K][ny][nx] / [K][ny][nx]; d_fbar may not alias
 * d_fbar_next.  FROZEN_INIT or USER mode only.  Asynchronous. */
int lbrs_adjoint_step(lbrs_ctx* c, const double* d_Utape_n, const double* d_fbar_next,
                      double* d_fbar);

/* Two adjoint steps in one launch: fbar^n from fbar^{n+2}, equal to
 * lbrs_adjoint_step with d_Utape_n1 (U^{n+1}) followed by lbrs_adjoint_step
 * with d_Utape_n (U^n), to rounding.  Each wavefront forms the rows of
 * fbar^{n+1} and feeds them straight into the second step, so fbar^{n+2} is
 * read and fbar^n written once (half the HBM traffic per step).  Layouts,
 * modes and errors as lbrs_adjoint_step; d_fbar may not alias d_fbar_next2.
 * lbrs_backward_checkpointed uses it when lbrs_set_fusion(c, 2) is on. */
int lbrs_adjoint_step2(lbrs_ctx* c, const double* d_Utape_n1, const double* d_Utape_n,
                       const double* d_fbar_next2, double* d_fbar);

/* k adjoint steps (k = 1 .. 4) in one launch: fbar^n from fbar^{n+k}
 * (d_fbar_next), with slot s of d_Utape [k][K][ny][nx] holding U^{n+s} (the
 * layout lbrs_step_tapes writes); equal to lbrs_adjoint_step with slots k-1,
 * k-2, .., 0 in turn, to rounding.  Each wavefront feeds every row it forms
 * straight into the next step, so fbar^{n+k} is read and fbar^n written once
 * per k steps.  Layouts, modes and errors as lbrs_adjoint_step, LBRS_E_INVAL
 * for k outside 1 .. 4; d_fbar may not alias d_fbar_next.
 * lbrs_backward_checkpointed and lbrs_backward_taped use it with k the
 * context's fusion.  Asynchronous. */
int lbrs_adjoint_steps(lbrs_ctx* c, int k, const double* d_Utape, const double* d_fbar_next,
                       double* d_fbar);

/* Adjoint of the initialisation f^0 = f^eq(U0): Ubar0 = sum_i (df_i^eq/dU)^T
 * fbar0_i at U0.  d_fbar0 [Q][K][ny][nx], d_U0 and d_Ubar0 [K][ny][nx].
 * FROZEN_INIT or USER mode only.  Asynchronous. */
int lbrs_adjoint_init(lbrs_ctx* c, const double* d_fbar0, const double* d_U0, double* d_Ubar0);

/* Adjoint of lbrs_prim_to_cons: given W and Ubar = dJ/dU, write Wbar = dJ/dW
 * = (dU/dW)^T Ubar.  [K][ny][nx] each; d_Wbar may alias neither input.
 * Enqueued on hip_stream. */
int lbrs_prim_to_cons_adjoint(const lbrs_params* p, const double* d_W, const double* d_Ubar,
                              double* d_Wbar, void* hip_stream);

/* Gas at rest with the isentropic pressure p = rho^gamma/gamma (the initial
 * state of an acoustic pulse): U = (rho, 0, [0,] rho^gamma/(gamma(gamma-1))).
 * d_rho [ny][nx], d_U [K][ny][nx].  Enqueued on hip_stream. */
int lbrs_isentropic_to_cons(const lbrs_params* p, const double* d_rho, double* d_U,
                            void* hip_stream);

/* Its adjoint: rhobar = Ubar_rho + Ubar_E rho^(gamma-1)/(gamma-1) = dJ/drho0. */
int lbrs_isentropic_to_cons_adjoint(const lbrs_params* p, const double* d_rho,
                                    const double* d_Ubar, double* d_rhobar, void* hip_stream);

/* Forward sweep of a checkpointed gradient (FROZEN_INIT or USER mode, 2D):
 * from the current state take nsteps steps, first copying the populations
 * before steps j*segment (j = 0 .. ceil(nsteps/segment)-1) into
 * d_ckpt + j*Q*K*nx*ny.  With segment ~ sqrt(nsteps) the store holds
 * ~sqrt(nsteps) population sets.  Asynchronous. */
int lbrs_forward_checkpointed(lbrs_ctx* c, int nsteps, int segment, double* d_ckpt);

/* Backward sweep (periodic D2Q4, FROZEN_INIT or USER mode): on entry d_fbar
 * holds dJ/df after the nsteps steps of lbrs_forward_checkpointed (called
 * last on this context, with the same nsteps, segment and d_ckpt); on return
 * it holds dJ/df^0.  Segments are processed last to first: each is recomputed
 * from its checkpoint with lbrs_step_tape, storing U^n in d_tape (segment
 * planes sets of K*nx*ny doubles), then lbrs_adjoint_step runs backwards
 * through it.  d_work is one population-sized buffer.  Waits once for the
 * stream at entry; the rest is asynchronous.  Leaves the context at the end
 * of the first segment. */
int lbrs_backward_checkpointed(lbrs_ctx* c, int nsteps, int segment, const double* d_ckpt,
                               double* d_tape, double* d_fbar, double* d_work);

/* The same gradient with every step's moments kept instead of checkpoints
 * (no recompute), for problems whose tape fits in device memory: nsteps
 * taped steps (as lbrs_step_tape; fused launches when lbrs_set_fusion(c, 2)
 * is on) from the current state, U^{n0+i} stored at d_tape + i*K*nx*ny
 * (nsteps*K*nx*ny doubles, caller-allocated).  Periodic D2Q4 Euler without
 * body or DIRICHLET side, FROZEN_INIT or USER mode (else LBRS_E_STATE).
 * Asynchronous. */
int lbrs_forward_taped(lbrs_ctx* c, int nsteps, double* d_tape);

/* Backward sweep over a tape of lbrs_forward_taped (same nsteps and d_tape):
 * on entry d_fbar holds dJ/df^{n0+nsteps}, on return dJ/df^{n0}; d_work is
 * one population-sized buffer (not d_fbar).  The context's state is not
 * used or changed.  Same modes and errors as lbrs_forward_taped.
 * Asynchronous. */
int lbrs_backward_taped(lbrs_ctx* c, int nsteps, const double* d_tape, double* d_fbar,
                        double* d_work);

/* Change the stream later calls enqueue on. */
int lbrs_set_stream(lbrs_ctx* c, void* hip_stream);

/* Launch shape of the 2D step.  Each wavefront marches the rows of a tile:
 * a strip of at most 62 columns by a segment of rows; waves loop over the tiles of a
 * persistent grid of the resident workgroups.  rows_per_tile = 0 (the
 * default) picks as many segments as make the tiles one balanced round of the
 * resident waves; otherwise segments of about rows_per_tile rows (1..65536).
 * waves_per_block is 1, 2, 4, 6, 8, 12 or 16 (default 4): the waves of a
 * workgroup march adjacent strips in lockstep.  alternate = 1 (the default)
 * marches odd row segments upwards, through a y-mirrored view of the
 * populations under which the update is exactly invariant, so that
 * neighbouring segments read their shared rows at the same time; 0 marches
 * every segment downwards.  The results are the same bits either way.  Takes
 * effect for later calls; LBRS_E_INVAL for values outside these sets. */
int lbrs_set_tile(lbrs_ctx* c, int rows_per_tile, int waves_per_block, int alternate);

/* Time steps per launch of the 2D Euler step: 1 (the default), 2, 3 or 4.  With
 * k > 1 each wavefront keeps the rows of f^{n+1} it has just streamed in
 * registers and streams them once more, k times (the same Sec. II.D update,
 * k times), so f^n is read and f^{n+k} written once per k steps: 1/k of the
 * HBM traffic per step.  The later steps' lattice speeds are known with
 * FROZEN_INIT or USER speeds.  With PER_STEP speeds each is the global bound
 * of the state before it: a launch guesses them -- a prediction the launch
 * before left (the exact next bounds evaluated around the cells where the
 * bound peaks), else the current bound -- and the next launch checks every
 * guessed bound bit for bit; on a mismatch (or a non-physical intermediate
 * state) that launch goes back to f^n, which the first launch left intact,
 * and redoes the steps with the bounds now known.  Either way t, the step
 * count, every lattice speed, the status, fail_step, the reported state after
 * each lbrs_step call and the populations are those of single steps, bit for
 * bit.  lbrs_step(c, max_steps, t_end) then enqueues a one-thread set-up
 * kernel and, with a fixed speed, (max_steps + k - 2)/k + 1 launches
 * (integer division); with
 * PER_STEP speeds each launch is followed by the prediction kernels (one per
 * guessed step), and a launch whose guess was wrong does no step, so the
 * call enqueues rounds of about max_steps/k + 2 launches, at most 512 (each
 * round with its own set-up for the steps left), waits for the stream after
 * each and reads how far the run got, until max_steps steps are done, t_end
 * is reached or a state is non-physical -- usually one round.  On a stream
 * being captured it instead enqueues max_steps launches (enough whatever
 * the guesses do; with a fixed speed those above), rounded up to a multiple
 * of six, and does not wait: the time state rotates its slots with the
 * launch count modulo six, so the captured graph can be replayed any number
 * of times, each replay continuing the run by up to max_steps steps from
 * where the last one left it, and the context's calls between replays see
 * the state the last replay left.  Launches beyond the work done exit at
 * once.
 * The shape set by lbrs_set_tile applies (strips of at most 64 - 2k columns;
 * automatic segments of at least 4 rows; 16 waves per workgroup run as 12,
 * as 8 with k >= 3 or PER_STEP speeds; alternate is ignored).
 * lbrs_step_tape stays a single step; lbrs_backward_checkpointed recomputes
 * its segments k steps per launch when k > 1 (every step's input moments
 * taped) and runs its adjoint steps k per launch (lbrs_adjoint_steps).
 * LBRS_E_INVAL for other values; LBRS_E_STATE with k > 1 for a 1D,
 * scalar-law, body or DIRICHLET context.  Takes effect for later calls. */
int lbrs_set_fusion(lbrs_ctx* c, int steps_per_launch);

/* ------------------------------------------------------------------------
 * Ragged batch of independent 1D units (shock tubes) in one persistent launch.
 * Every unit is a full problem of the paper's 1D scheme (Sec. II.A update,
 * Sec. II.C equilibria and bound) with its own lbrs_params (model D1Q2 or
 * D1Q3, the same for all units; nx, domain, gamma, omega, cfl, x sides and
 * lambda mode) and its own t_end; the units' cells lie back to back in pools:
 *   U pool  [3][total]     f pool  [Q*3][total]    (unit b at offsets[b])
 * A unit of more than `chunk` cells is split over a team of workgroups that
 * keep their chunk in LDS for the whole run and synchronise once per step.
 * ------------------------------------------------------------------------ */
typedef struct lbrs_batch lbrs_batch;

/* Offsets of the units in the pools (offsets[nunits] = total cells; may be
 * NULL) and the device scratch size for a chunk size (cells per workgroup,
 * >= 3; at most what the LDS holds: 6*(chunk+2) doubles, the post-collision
 * values of the two moving populations).  A unit may span
 * at most 64 workgroups (nx <= 64*chunk).  Needs the GPU (occupancy). */
int lbrs_batch_query(int nunits, const lbrs_params* units, int chunk, long long* offsets,
                     size_t* scratch_bytes);

/* Plan the batch (member jobs on the persistent grid), upload it to
 * d_scratch (256-byte aligned, lbrs_batch_query's size; borrowed), and set
 * every unit to equilibrium f^0 = f^eq(U0) from d_U0.  t_end: host array of
 * nunits end times (NULL: unbounded).  Waits for the stream once. */
int lbrs_batch_init(lbrs_batch** out, int nunits, const lbrs_params* units, const double* t_end,
                    int chunk, const double* d_U0, double* d_f, void* d_scratch, void* hip_stream);

/* Advance every unit by up to max_steps steps (each stops at its t_end or at
 * a non-physical state) in one persistent launch; the launch is captured in a
 * hipGraph the first time and replayed after.  Asynchronous. */
int lbrs_batch_run(lbrs_batch* b, int max_steps);

/* Per-unit time, steps, last lattice speed, status (bit 0 non-physical,
 * bit 1 team barrier gave up) and first non-physical step (or -1), into host
 * arrays of nunits (each may be NULL).  Waits for the stream. */
int lbrs_batch_get_state(lbrs_batch* b, double* t, long long* nsteps, double* lambda,
                         unsigned* status, long long* fail_step);

/* Moments U = sum_i f_i of the whole f pool into d_U [3][total]. */
int lbrs_batch_moments(lbrs_batch* b, double* d_U);

void lbrs_batch_destroy(lbrs_batch* b);

/* ------------------------------------------------------------------------
 * Batch of independent 2D domains (D2Q4, fixed lattice speeds: FROZEN_INIT or
 * USER mode per domain; PER_STEP is rejected).  Domain d occupies cells
 * [off_d, off_d + nx_d*ny_d) of the moment pools ([4][total]) and the
 * population block [16*off_d, 16*(off_d + nx_d*ny_d)) of the population pools,
 * row-interleaved ([ny_d][16][nx_d]).  One launch advances every domain by
 * one step (the same fused step as lbrs_step); the adjoint calls (periodic
 * domains) mirror the single-domain ones.  All calls are asynchronous on the
 * batch's stream except where noted.
 * ------------------------------------------------------------------------ */
typedef struct lbrs_batch2d lbrs_batch2d;

/* Cell offsets (ndom + 1 values, may be NULL) and scratch bytes. */
int lbrs_batch2d_query(int ndom, const lbrs_params* doms, long long* cell_offsets,
                       size_t* scratch_bytes);

/* Plan the tiles, upload the domain table to d_scratch (256-byte aligned,
 * borrowed; waits for the stream once), and reset from d_U0 (see below).
 * d_f0, d_f1: population pools of 16*total doubles each (borrowed). */
int lbrs_batch2d_init(lbrs_batch2d** out, int ndom, const lbrs_params* doms, const double* d_U0,
                      double* d_f0, double* d_f1, void* d_scratch, void* hip_stream);

/* Every domain's lattice speed from U0 (FROZEN_INIT: lambda*(U0_d)/cfl_d),
 * f^0 = f^eq(U0) per domain (Sec. II.A), step count 0. */
int lbrs_batch2d_reset(lbrs_batch2d* b, const double* d_U0);

/* nsteps collide-and-stream steps of every domain: one launch per step, or
 * with lbrs_batch2d_set_fusion(b, k) one launch per k steps (and one more
 * for the remainder: a fused launch for two or more steps, a single step
 * for one). */
int lbrs_batch2d_step(lbrs_batch2d* b, int nsteps);

/* Time steps per forward launch of lbrs_batch2d_step and of the forward
 * sweep of lbrs_batch2d_gradient: 1 (the default), 2, 3 or 4.  With k > 1
 * each wavefront streams the rows of f^{n+1} it has just produced straight
 * into the next step, k times (as lbrs_set_fusion; the speeds are fixed, so
 * nothing is guessed): 1/k of the HBM traffic per step, the same results to
 * rounding.  A domain with a non-physical state after any of the k steps
 * gets its status set.  The gradient's taped recompute and its adjoint steps
 * are fused too (two per launch); lbrs_batch2d_step_tape and
 * lbrs_batch2d_adjoint_step stay single steps.  A change of k re-plans the
 * fused launches' strips (at most 64 - 2k columns) and uploads the domain
 * table (waits for the stream).
 * LBRS_E_INVAL for other values; LBRS_E_HIP if the upload fails. */
int lbrs_batch2d_set_fusion(lbrs_batch2d* b, int steps_per_launch);

/* One step that also stores every domain's input moments U^n in d_Utape [4][total]. */
int lbrs_batch2d_step_tape(lbrs_batch2d* b, double* d_Utape);

/* Adjoint of one step for every domain (periodic domains only, else
 * LBRS_E_STATE); same definition as lbrs_adjoint_step, pools as above. */
int lbrs_batch2d_adjoint_step(lbrs_batch2d* b, const double* d_Utape, const double* d_fbar_next,
                              double* d_fbar);

/* Adjoint of f^0 = f^eq(U0) for every domain: d_Ubar0 [4][total]. */
int lbrs_batch2d_adjoint_init(lbrs_batch2d* b, const double* d_fbar0, const double* d_U0,
                              double* d_Ubar0);

/* Window of the objective: cells whose centres (origin at the domain's lower
 * left corner) lie in the closed square [lo, hi]^2.  Waits for the stream. */
int lbrs_batch2d_set_window(lbrs_batch2d* b, double lo, double hi);

/* J_d = sum over domain d's window of rho^2 into d_J [ndom] (each by one
 * workgroup in a fixed order) and the seed dJ_d/df into d_fbar (pool). */
int lbrs_batch2d_window_objective(lbrs_batch2d* b, double* d_J, double* d_fbar);

/* Moments of the current populations into d_U [4][total]; population
 * checkpoints to/from a pool-sized buffer (set_f also sets the step count). */
int lbrs_batch2d_moments(lbrs_batch2d* b, double* d_U);
int lbrs_batch2d_get_f(lbrs_batch2d* b, double* d_f);
int lbrs_batch2d_set_f(lbrs_batch2d* b, const double* d_f, long long n);

/* Gradients dJ_d/dU0 of every domain's window objective after nsteps steps:
 * reset from d_U0, forward sweep with population checkpoints every `segment`
 * steps (d_ckpt: ceil(nsteps/segment) pools), objective (d_J [ndom]),
 * backward sweep (per segment: recompute with the moment tape d_tape,
 * `segment` sets of [4][total], then reverse adjoint steps; d_fbar, d_work:
 * pools), adjoint of the initialisation into d_Ubar0 [4][total].  With
 * use_graph != 0 the whole sequence is captured in a hipGraph on the first
 * call and replayed by later calls with the same arguments (a call with other
 * pointers, nsteps or segment captures a new graph).  With segment >= nsteps
 * the forward sweep itself writes every step's moments to d_tape (nsteps sets)
 * and the adjoint runs straight back through them: no checkpoint (d_ckpt is
 * not used) and no recompute.  No host synchronisation. */
int lbrs_batch2d_gradient(lbrs_batch2d* b, const double* d_U0, int nsteps, int segment,
                          double* d_ckpt, double* d_tape, double* d_fbar, double* d_work,
                          double* d_J, double* d_Ubar0, int use_graph);

/* Step count, per-domain lattice speed and status (bit 0: a non-physical
 * state met), host arrays of ndom (may be NULL).  Waits for the stream. */
int lbrs_batch2d_get_state(lbrs_batch2d* b, long long* nsteps, double* lambda, unsigned* status);

void lbrs_batch2d_destroy(lbrs_batch2d* b);

/* ------------------------------------------------------------------------
 * No-allocation entry point, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * One whole run -- lbrs_init, lbrs_step(max_steps, t_end) (steps_per_launch
 * steps per launch, 1 to 4, as lbrs_set_fusion) and lbrs_moments --
 * with the same kernels and results, but the time state (t, step count, the
 * lambda* reduction slots, the status and the fused launches' record) lives
 * in a static device array of the library (512 KiB per GPU, kept until the
 * process ends) instead of a caller scratch area, and the context on the
 * stack: the call allocates nothing, host or device.  The caller passes
 * d_U0, the two population buffers (lbrs_query_sizes' f_bytes each), the
 * output d_U [K][ny][nx] and optionally d_state (5 device doubles: t,
 * completed steps, lattice speed of the last step, status, first
 * non-physical step or -1).  Asynchronous on hip_stream (with PER_STEP
 * speeds and steps_per_launch > 1 it enqueues the max_steps launches that
 * suffice whatever the guesses, never the rounds of lbrs_step).  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams, threads) race; calls in one stream are ordered.
 * Parameters as
 * lbrs_init, except that solid bodies (whose node codes would need a staging
 * buffer and more scratch than the array holds) are rejected: LBRS_E_INVAL.
 * LBRS_E_HIP if the array's device address cannot be found. */
int lbrs_run_noalloc(const lbrs_params* p, const double* d_U0, double* d_f0, double* d_f1,
                     int max_steps, double t_end, int steps_per_launch, double* d_U,
                     double* d_state, void* hip_stream);

const char* lbrs_strerror(int code);

/* Free the context (and its pinned host buffer, if lbrs_init made one); the
 * caller's device buffers stay the caller's.  Work enqueued on its stream
 * should have finished. */
void lbrs_destroy(lbrs_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* LBRS_H */
