/*
 * fvlbm.h — C ABI of the MI355X finite-volume lattice Boltzmann library.
 *
 * One call of fvlbm_step advances the cell-centred D2Q9 FVLBM on an unstructured 2D mesh by the
 * three-stage, second-order IMEX Runge-Kutta scheme of arXiv 1812.00394 (Part II), Section 3.1
 * (Eqs. (semibgk), (advection), (collision), (imexone), (imextwo), (sumimeximplicitnew),
 * (fnewstage)), optionally coupled with the k-omega SST model of its Section 2 through the
 * eddy-viscosity relaxation time of Eq. (turbtau), in the order of the algorithm (Steps 0-8) at
 * the end of its Section 3.2.
 *
 * Conventions shared by every entry point
 *   - Every call returns fvlbm_status; nothing throws across the ABI.  On a non-OK status
 *     fvlbm_last_error() returns a message (thread-local, valid until the next call on the
 *     same thread).
 *   - Host arrays are plain C arrays in the caller's cell order ("user order"); the library
 *     renumbers cells internally (Morton, graph-grown tiles or RCM) and never exposes that order.
 *   - Device memory is owned by the caller: fvlbm_state_bytes() says how much, fvlbm_init()
 *     receives it.  The library itself allocates no device memory.
 *   - All device work is enqueued on the HIP stream given to fvlbm_init() (the adjoint's
 *     overlapped recompute on small meshes uses a stream of its own, joined to that stream before
 *     the call returns).  Calls that return host values synchronise that stream; the others are
 *     asynchronous.
 *   - Environment (diagnostics and tests): FVLBM_SWEEP = ring | pair | tiled | tiled-grads | split | face
 *     forces a sweep variant (ring, pair: only where it fits, one or two threads per cell in the
 *     stage sweeps; face: the edge loop with atomics, kept for
 *     the measured comparison with the cell loops; its sums' order, and so the last bits of its
 *     results, vary from run to run); FVLBM_ADJ_OVERLAP = 0 gives the adjoint one set
 *     of segment buffers (no kept second tape, no overlap).  Both are read when a state is created
 *     or a run recorded.
 *   - Distribution functions are indexed by the D2Q9 direction a = 0..8 with lattice
 *     velocities e_a = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1) and
 *     weights 4/9, 1/9 (a=1..4), 1/36 (a=5..8); c_s^2 = 1/3.  Arrays of f are [9][n_cells].
 */
#ifndef FVLBM_H
#define FVLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FVLBM_OK = 0,
    FVLBM_EINVAL = -1,     /* bad argument: sizes, NULL pointers, tau <= 0, too small workspace */
    FVLBM_EMESH = -2,      /* malformed mesh: non-positive area, edge shared by >2 cells,
                              boundary edge unmatched / unassigned, periodic edge without partner */
    FVLBM_ENOMEM = -3,     /* host allocation failed */
    FVLBM_EDEVICE = -4,    /* a HIP call failed (message names it) */
    FVLBM_EDIVERGED = -5,  /* a reduction met a non-finite value */
    FVLBM_ESTATE = -6      /* call not valid for this state (e.g. SST data asked of a laminar state) */
} fvlbm_status;

/* boundary group kinds */
enum {
    FVLBM_WALL = 1,        /* resting no-slip wall */
    FVLBM_MOVING_WALL = 2, /* no-slip wall moving tangentially with the group velocity */
    FVLBM_INLET = 3,       /* prescribed velocity (rotated by theta), k, omega */
    FVLBM_OUTLET = 4,      /* prescribed density; zero-gradient k, omega */
    FVLBM_FARFIELD = 5,    /* free stream (rho, u rotated by theta, k, omega) */
    FVLBM_PERIODIC = 6     /* paired with the edges found at midpoint + periodic_shift */
};

/* storage / arithmetic of f: FP64; FP32 deviations from w_a rho0 (the ring sweeps stream FP32 copies
 * of the geometry, with the LSQ coefficients rounded once from FP64); FP32 deviations whose ring
 * sweeps stream FP64 geometry and form normals, midpoint offsets and LSQ coefficients in FP64 before
 * the FP32 flux arithmetic (ring-tiled sweeps only; its recorded steps run the same kernels, and
 * the adjoint's transposed sweeps take the FP32 copies of the geometry, so its gradient is that of
 * the forward to within the FP32 rounding of the geometry) */
enum { FVLBM_FP64 = 0, FVLBM_FP32_DEV = 1, FVLBM_FP32_DEV_GEO64 = 2 };
enum { FVLBM_ORDER_NONE = 0, FVLBM_ORDER_MORTON = 1, FVLBM_ORDER_RCM = 2, FVLBM_ORDER_TILES = 3 };

#define FVLBM_MAX_GROUPS 16

typedef struct fvlbm_mesh fvlbm_mesh;
typedef struct fvlbm_state fvlbm_state;

/*
 * Physical and numerical parameters (lattice units).
 *   nu         molecular kinematic viscosity; the laminar relaxation time is tau = 3 nu
 *              (Eq. (turbtau) with nu_t = 0)
 *   dt         time step
 *   rho0       reference density (outlet default; the FP32 mode stores f - w_a rho0)
 *   sst        0: laminar; 1: k-omega SST once per step before the three stages (Section 3.2,
 *              Step 1); 2: the SST solved again before the third stage, from k^n, omega^n with the
 *              second stage's macro variables, for that stage's relaxation time, the step keeping
 *              this solve's k, omega, nu_t (Step 5 read literally; the second stage's SST inputs
 *              equal the first's, whose stage solve keeps rho and u).  Its adjoint reverses both
 *              solves: the second from the third stage's tau and the step's k, omega onto the
 *              second stage's field, the first from the tau of stages 1 and 2.
 *   a1 ... beta2  the SST constants listed in Section 2 (C_omega1/2 are derived from them)
 *   theta      inflow angle [rad]: rotates every INLET and FARFIELD velocity
 *   group_*    per boundary group: velocity (u, v), density, k, omega
 *   bface_vals NULL, or [n_bfaces][5] = (u, v, rho, k, omega) per boundary edge in the order
 *              given to fvlbm_mesh_create, replacing the group values (inflow profiles)
 *   jr_group, jr_xmin, eps_tau   the reattachment proxy J_R of fvlbm_forces
 *   limiter    0: the upwind face value of f is the linear reconstruction (Eq. (advection) with
 *              the cell gradient); 1: it is also kept between the values of the two cells that
 *              share the edge (first order at local extrema; for flows around sharp edges);
 *              2: each cell's gradient is scaled (Barth and Jespersen) by the largest factor in
 *              [0, 1] that keeps its reconstructed values at all its edge midpoints within the
 *              least and greatest of its own value and its stencil values (neighbours, boundary
 *              ghosts): bounded on meshes with sliver cells, where the plain reconstruction has
 *              a growing mode.  The adjoint differentiates limiter 1 (through the clip states its
 *              recorded steps keep) and limiter 2 (its reverse runs on the two-kernel transposes,
 *              whichever sweep ran forward).
 *   sst_sweeps 0: the SST equations advance point-implicitly (sinks implicit, face fluxes
 *              explicit).  m in [1, 1000]: they advance implicitly as Section 3.2 says of the
 *              Code_Saturne integration: backward Euler for the increments of k and omega with
 *              first-order upwind convection and two-point diffusion at the new level (level-n
 *              mass fluxes and coefficients), the rest of the second-order flux at level n, and
 *              the point-implicit sinks; the linear system is solved with m Jacobi sweeps from a
 *              zero increment (one SST launch that writes the system, then m - 1 sweep launches,
 *              one launch when m = 1).  Ignored when sst = 0.  The adjoint differentiates it for
 *              m <= 16 (it keeps every sweep's increments; fvlbm_record rejects m > 16 with
 *              FVLBM_ESTATE).  A periodic cell that is its own neighbour across an edge keeps
 *              that coupling on the diagonal (Jacobi with the diagonal of the whole matrix).
 *              Errors: FVLBM_EINVAL outside [0, 1000].
 */
typedef struct {
    double nu, dt, rho0;
    int32_t sst, n_groups;
    double a1, beta_star, kappa, sigma_k1, sigma_w1, beta1, sigma_k2, sigma_w2, beta2;
    double theta;
    double group_u[FVLBM_MAX_GROUPS][2];
    double group_rho[FVLBM_MAX_GROUPS];
    double group_k[FVLBM_MAX_GROUPS];
    double group_w[FVLBM_MAX_GROUPS];
    const double *bface_vals;
    int32_t jr_group, limiter;
    double jr_xmin, eps_tau;
    int32_t sst_sweeps;
} fvlbm_params;

/*
 * Build a mesh from host arrays (copied; the caller keeps ownership of its arrays): the cells of
 * the cell-centred finite-volume discretisation of Section 3.1, with what the method needs of
 * them: the edge normals and lengths of the flux sum of Eq. (advection), the least-squares
 * gradient of its linear upwind reconstruction, and the wall distance d of the SST blending
 * functions F1 and F2 (Section 2).
 *   node_xy       [n_nodes][2]
 *   cell_ptr      [n_cells+1] CSR offsets into cell_nodes; every cell has 3 or 4 nodes listed
 *                 counter-clockwise (positive shoelace area)
 *   bface_nodes   [n_bfaces][2] node pairs of the boundary edges (any orientation)
 *   bface_group   [n_bfaces] group id in [0, n_groups)
 *   group_kind    [n_groups] FVLBM_WALL ... FVLBM_PERIODIC
 *   periodic_shift [n_groups][2] or NULL: translation taking a periodic group's edges onto their
 *                 partner edges
 *   order         internal renumbering (FVLBM_ORDER_*): MORTON sorts the centroids along a Morton
 *                 curve; TILES grows tiles of 256 cells breadth-first on the cell graph from
 *                 Morton-ordered seeds (compact tiles, small halos, on stretched meshes too);
 *                 RCM is reverse Cuthill-McKee; NONE keeps the user's order
 * Computes, in FP64 on the host: cell areas and centroids, edge normals and midpoints, the
 * weighted least-squares gradient coefficients, the wall distance (exact nearest point on the
 * WALL / MOVING_WALL edges) and the renumbering.  Errors: FVLBM_EINVAL, FVLBM_EMESH.
 */
fvlbm_status fvlbm_mesh_create(int64_t n_nodes, const double *node_xy,
                               int64_t n_cells, const int64_t *cell_ptr, const int64_t *cell_nodes,
                               int64_t n_bfaces, const int64_t *bface_nodes, const int32_t *bface_group,
                               int32_t n_groups, const int32_t *group_kind, const double *periodic_shift,
                               int32_t order, fvlbm_mesh **out);
void fvlbm_mesh_destroy(fvlbm_mesh *mesh);

/* counts[0..3] = cells, interior edges, boundary edges (periodic ones counted as interior),
 * maximum edges per cell. */
fvlbm_status fvlbm_mesh_counts(const fvlbm_mesh *mesh, int64_t counts[4]);

/* Host copies of the mesh's FP64 geometry in user order; any pointer may be NULL.
 * area [n], centroid [n][2], wall_dist [n] (1e30 where the mesh has no wall). */
fvlbm_status fvlbm_mesh_geometry(const fvlbm_mesh *mesh, double *area, double *centroid, double *wall_dist);

/* Internal renumbering: perm[i] = user index of internal cell i. */
fvlbm_status fvlbm_mesh_permutation(const fvlbm_mesh *mesh, int64_t *perm);

/* Largest time step at advective Courant number 1 (the explicit convection limit of the IMEX
 * stages): 1 / max over cells c and directions a of sum_edges max(e_a.n, 0) dl / A_c. */
fvlbm_status fvlbm_mesh_max_dt(const fvlbm_mesh *mesh, double *dt);

/* Device bytes fvlbm_init needs for this mesh, precision and SST switch (a forward state; the
 * memory of a recorded run for the adjoint is sized by fvlbm_adjoint_bytes and passed to
 * fvlbm_record). */
fvlbm_status fvlbm_state_bytes(const fvlbm_mesh *mesh, int32_t precision, int32_t sst, size_t *bytes);

/*
 * Step 0 of the algorithm: set f = f_eq(rho, u) per cell (and k, omega when params->sst).
 *   rho [n], u [n][2], k [n], omega [n]: host arrays in user order (k, omega ignored if !sst)
 *   workspace: device memory of at least fvlbm_state_bytes() bytes, 256-byte aligned, owned by
 *              the caller and alive until fvlbm_state_destroy.
 *   hip_stream: the hipStream_t all work of this state is enqueued on (NULL = default stream).
 * The mesh must outlive the state.  Errors: FVLBM_EINVAL, FVLBM_EDEVICE.
 */
fvlbm_status fvlbm_init(const fvlbm_mesh *mesh, const fvlbm_params *params, int32_t precision,
                        const double *rho, const double *u, const double *k, const double *omega,
                        void *workspace, size_t ws_bytes, void *hip_stream, fvlbm_state **out);

/* Replace the state: f [9][n] (FP64, user order, host), and k, omega [n] when SST is on
 * (may be NULL to keep the current ones).  Synchronises the stream. */
fvlbm_status fvlbm_set_state(fvlbm_state *st, const double *f, const double *k, const double *omega);

/*
 * Advance n_steps IMEX steps (Steps 1-7 each).  If residual != NULL, the velocity residual
 * ||u^{n+1} - u^n||_2 / ||u^{n+1}||_2 of the last step is computed in FP64 and returned (this
 * synchronises; for a flow at rest, ||u^{n+1}|| = 0, the absolute norm ||u^{n+1} - u^n||_2); a
 * non-finite residual returns FVLBM_EDIVERGED.  Without a residual nothing is checked: a NaN or an
 * overflow surfaces at the next call that reduces (a residual, fvlbm_moments' totals,
 * fvlbm_forces), which returns FVLBM_EDIVERGED.
 */
fvlbm_status fvlbm_step(fvlbm_state *st, int32_t n_steps, double *residual);

/*
 * Run toward a steady state, the residual-driven long runs of Section 4: fvlbm_step in blocks of
 * check_every steps, the velocity residual of fvlbm_step evaluated after each block (one host
 * synchronisation per block), until it falls below tol or max_steps steps were taken (the last
 * block is shortened to end there).  steps_out (may be NULL): steps taken; residual_out (may be
 * NULL): the last residual.  Errors: FVLBM_EINVAL (NULL state, max_steps < 1, check_every < 1,
 * tol < 0), FVLBM_EDIVERGED (non-finite residual; the state is left as it is).
 */
fvlbm_status fvlbm_run_to_residual(fvlbm_state *st, int64_t max_steps, int32_t check_every, double tol,
                                   int64_t *steps_out, double *residual_out);

/*
 * Advance n_steps steps of the explicit scheme the paper compares the IMEX scheme with (Section
 * 3.1): forward Euler of the semi-discrete equation, Eq. (semibgk), f^{n+1} = f^n + dt (Ga(f^n) +
 * (f_eq(f^n) - f^n) / tau), with the SST update first as in fvlbm_step.  Stable for dt < 2 tau
 * only (the caller's choice).  Needs the ring-tiled sweep (FVLBM_ESTATE otherwise); residual as
 * fvlbm_step.
 */
fvlbm_status fvlbm_step_explicit(fvlbm_state *st, int32_t n_steps, double *residual);

/*
 * Macro fields (Step 7) in FP64, user order.  on_device = 0: host pointers (synchronises);
 * 1: device pointers (asynchronous).  Any field pointer may be NULL.  rho [n], u [n][2],
 * k, omega, nu_t [n] (FVLBM_ESTATE if asked of a laminar state).  totals (host, may be NULL):
 * sum A rho, sum A rho u_x, sum A rho u_y in FP64 (synchronises; FVLBM_EDIVERGED if non-finite).
 */
fvlbm_status fvlbm_moments(fvlbm_state *st, int32_t on_device, double *rho, double *u, double *k,
                           double *omega, double *nu_t, double totals[3]);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the totals of fvlbm_moments (sum A rho, sum A rho u_x, sum A rho u_y, FP64,
 * same kernels and summation order) written to totals_dev, a device pointer to 3 doubles, enqueued
 * on the state's stream without synchronising and without allocating.  The partial sums live in a
 * reduction buffer the library holds itself, 16 KiB per GPU until the process ends (the fixed grid
 * of 512 blocks x 3 sums needs 12 KiB; every size of state fits).  Calls that overlap on one GPU
 * (states on different streams, several host threads) share that buffer and race: order them on one
 * stream.  No non-finite check (read the result).  Errors: FVLBM_EINVAL (NULL, empty state),
 * FVLBM_EDEVICE (launch).
 */
fvlbm_status fvlbm_totals_noalloc(fvlbm_state *st, double *totals_dev);

/* f [9][n] in FP64, user order (for FP32 storage: w_a rho0 added back). */
fvlbm_status fvlbm_get_f(fvlbm_state *st, int32_t on_device, double *f);

/*
 * Surface functionals in FP64 (host results; synchronises): the wall force behind the airfoil's
 * lift and drag and the wall shear behind the backward-facing step's reattachment length, the
 * quantities Section 4 reports for its two turbulent tests.  force[2]: the force of the fluid
 * on the WALL / MOVING_WALL edges of the groups whose bit is set in wall_group_mask, gauge
 * pressure (p - rho0/3) n l plus the wall shear mu (u_c - u_w)_t / d_perp l with mu = rho_c nu.
 * j_r (may be NULL): sum over the walls of group params->jr_group with x_f > jr_xmin of
 * l (1 - tanh(tau_x / eps_tau)) / 2 (smooth reversed-flow length).
 */
fvlbm_status fvlbm_forces(fvlbm_state *st, uint64_t wall_group_mask, double force[2], double *j_r);

/*
 * Lift and drag coefficients of the walls in wall_group_mask (the force of fvlbm_forces, on the
 * airfoil of the paper's Section 4 test): drag along the free-stream direction (cos theta,
 * sin theta), lift along (-sin theta, cos theta), both divided by rho0 u_ref^2 chord / 2.
 * coeffs[2] = (C_l, C_d).  Errors: FVLBM_EINVAL (NULL, u_ref or chord <= 0), FVLBM_EDIVERGED.
 */
fvlbm_status fvlbm_lift_drag(fvlbm_state *st, uint64_t wall_group_mask, double u_ref, double chord, double coeffs[2]);

/*
 * Diagnostic: the convection term Gamma^a of Eq. (advection) of an arbitrary field g, with the
 * boundary treatment of fvlbm_step.  g_in, out: host [9][n] FP64 user order.  Synchronises.
 */
fvlbm_status fvlbm_apply_advection(fvlbm_state *st, const double *g_in, double *out);

/*
 * Per-kernel timing with HIP events recorded on the state's stream around every launch of
 * fvlbm_step.  enable = 1 clears the counters and starts recording, 0 stops.  fvlbm_timing_read
 * synchronises and returns, per kernel id (FVLBM_K_*), the summed duration in ms and the number of
 * launches since recording started.
 */
enum {
    FVLBM_K_SST_A = 0,     /* SST gradients, blending, eddy viscosity, sources */
    FVLBM_K_SST_B = 1,     /* SST fluxes and update, nu_t -> tau */
    FVLBM_K_COLLIDE1 = 2,  /* stage-1 collision */
    FVLBM_K_GRAD = 3,      /* least-squares gradient of a stage field */
    FVLBM_K_SWEEP1 = 4,    /* stage-1 convection + stage-2 collision */
    FVLBM_K_SWEEP2 = 5,    /* stage-2 convection + stage-3 collision */
    FVLBM_K_SWEEP3 = 6,    /* stage-3 convection + combination + macro update */
    FVLBM_K_SST = 7,       /* SST in one ring-tiled launch (replaces SST_A + SST_B) */
    FVLBM_K_EXPLICIT = 8,  /* convection + collision of the explicit scheme */
    FVLBM_K_SST_JACOBI = 9, /* Jacobi sweeps of the implicit SST variant (all of a solve) */
    FVLBM_K_FACE = 10,     /* edge loop with atomics (FVLBM_SWEEP=face): the interior edges' fluxes */
    FVLBM_K_COUNT = 11
};
fvlbm_status fvlbm_timing(fvlbm_state *st, int32_t enable);
fvlbm_status fvlbm_timing_read(fvlbm_state *st, double ms[FVLBM_K_COUNT], int64_t launches[FVLBM_K_COUNT]);

/*
 * Diagnostic: the transpose of the convection operator at g, g_bar = (d Gamma^a(g) / d g)^T lam,
 * and d_theta = d(lam . Gamma^a(g)) / d theta (theta enters through the inlet / far-field ghost
 * states).  g_in, lam, g_bar: host [9][n] FP64 user order; d_theta: one double.  Synchronises.
 */
fvlbm_status fvlbm_apply_advection_adjoint(fvlbm_state *st, const double *g_in, const double *lam, double *g_bar,
                                           double *d_theta);

/*
 * Discrete adjoint (reverse mode) of a recorded run, with checkpointing and recomputation.
 *
 * fvlbm_adjoint_bytes: device bytes of the adjoint workspace for n_steps recorded steps with a
 *   checkpoint every ckpt_every steps: checkpoints (11 n values each), one segment of states
 *   (ckpt_every + 1 of 11 n values) and of stage data (59 n values per step), a second such
 *   segment when the run has more than one, adjoint fields (including those of the implicit SST
 *   variant's reverse, 70 n values, and of the two-kernel transposes with the limiters' reverses,
 *   33 n values and 16 n bytes).
 * fvlbm_record: advances the state n_steps steps exactly as fvlbm_step does, storing the state
 *   (f, k, omega) at the start of every segment and at the end in `workspace` (device memory owned
 *   by the caller, 256-byte aligned, kept alive until the adjoint has run).  Segments have at most
 *   ckpt_every steps and are counted from the end of the run (only the first may be shorter); the
 *   last two (the last one when the run has one segment) are kept whole, with their stage data, in
 *   the two sets of segment buffers, so that the reverse recomputes neither.  With the face-value
 *   limiter (limiter 1) the ring-tiled sweeps keep its clip states in the stage data; after the
 *   other sweeps the reverse forms them again from the recorded stage fields.  Errors:
 *   FVLBM_EINVAL (NULL, n_steps or ckpt_every < 1, workspace misaligned or too small),
 *   FVLBM_ESTATE.
 * fvlbm_adjoint_step: for J = seed[0] F_x + seed[1] F_y + seed[2] J_R of the final state (forces of
 *   the walls in wall_group_mask and the reversed-flow length, as fvlbm_forces), returns
 *   dparams = dJ/d(theta, sigma_k1, sigma_omega1, beta*, a1) in FP64, differentiating the discrete
 *   step exactly (branches of max / min / upwind choices as taken).  Each segment of ckpt_every
 *   steps is recomputed once from its checkpoint, keeping every step's input state and stage data
 *   (the record pass leaves the last two segments in that form); its steps are then reversed from
 *   the last.  With the ring-tiled sweep on meshes of at most 262,144 cells, where one launch leaves
 *   most of the GPU idle, the recompute of the next segment (into the second set of segment
 *   buffers) runs on a stream of the library's own, created on first use, while the current
 *   segment is reversed on the caller's stream; the two are ordered by events and the call returns
 *   with all work on the caller's stream.  The reverse: the combination and stage collisions in closed
 *   form, the convection term by its transpose, the SST update (or the implicit variant's system,
 *   by its transposed Jacobi sweeps and rows), fluxes, closure and LSQ gradients (with the
 *   gradient limiter, through its selections found again) by their transposes.  The state is
 *   restored to the final recorded state afterwards.  A call that changes the state after fvlbm_record
 *   (fvlbm_step, fvlbm_step_explicit, fvlbm_run_to_residual, fvlbm_set_state) drops the recording:
 *   the tape would no longer end at the current state.  Errors: FVLBM_ESTATE without a recording
 *   (never recorded, or dropped), FVLBM_EDIVERGED.
 * fvlbm_adjoint_state: the same reverse run seeded with the adjoint of the final state (host [9][n],
 *   [n], [n] FP64 user order; lam_k / lam_w may be NULL), returning the adjoint of the recorded
 *   initial state and dparams (for dot-product checks).
 */
fvlbm_status fvlbm_adjoint_bytes(const fvlbm_mesh *mesh, int32_t precision, int32_t n_steps, int32_t ckpt_every,
                                 size_t *bytes);
fvlbm_status fvlbm_record(fvlbm_state *st, int32_t n_steps, int32_t ckpt_every, void *workspace, size_t ws_bytes);
fvlbm_status fvlbm_adjoint_step(fvlbm_state *st, uint64_t wall_group_mask, const double seed[3], double dparams[5]);
fvlbm_status fvlbm_adjoint_state(fvlbm_state *st, const double *lam_f, const double *lam_k, const double *lam_w,
                                 double *lam_f0, double *lam_k0, double *lam_w0, double dparams[5]);

/*
 * The adjoint of the lift and drag coefficients of the airfoil test (Section 4, the NACA0012
 * lift/drag table): for J = seed[0] C_l + seed[1] C_d of the final recorded state, with C_l, C_d as
 * fvlbm_lift_drag defines them (the wall force of the groups in wall_group_mask along the lift and
 * drag directions of the inflow angle theta, over rho0 u_ref^2 chord / 2), returns
 * dparams = dJ/d(theta, sigma_k1, sigma_omega1, beta*, a1) in FP64: the reverse run of
 * fvlbm_adjoint_step seeded with dJ/dF, plus the explicit dependence on theta of the two directions
 * (dC_l/dtheta = -C_d, dC_d/dtheta = C_l at fixed force).  coeffs (may be NULL) receives (C_l, C_d)
 * of the final state.  Errors: FVLBM_EINVAL (NULL, u_ref or chord <= 0), FVLBM_ESTATE (no
 * recording), FVLBM_EDIVERGED.
 */
fvlbm_status fvlbm_adjoint_lift_drag(fvlbm_state *st, uint64_t wall_group_mask, double u_ref, double chord,
                                     const double seed[2], double coeffs[2], double dparams[5]);

void fvlbm_state_destroy(fvlbm_state *st);

const char *fvlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FVLBM_H */
