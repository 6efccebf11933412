/*
 * eulbfs.h -- C ABI of the MI355X (gfx950) EULBFS time-step library.
 *
 * EULBFS: enthalpy-based unified lattice Boltzmann flux solver for liquid
 * solidification with volume change (Zhou, Yang, Wang, Wu, Niu; arXiv
 * 2507.03366).  One time step advances the conserved vector
 *     W = (H, p, rho c_s^2 u, rho c_s^2 v, C)                        (Eq. 49)
 * of the cell-centred finite-volume form dW/dt = -div F + F_E (Eqs. 48-52)
 * with the SSP-RK3 scheme of Eq. (58).  The face fluxes F (Eq. 53) come from
 * a local lattice Boltzmann reconstruction at each face (Sec. 2.4, Eqs.
 * 54-56): D2Q9 for the flow field, D2Q9 or D2Q5 for the total enthalpy and
 * the phase field.  After each stage the enthalpy closure H -> (T, F_l)
 * (Eqs. 5-6) and the mixture rule (Eq. 7) give the primitive fields; the
 * expansion source rho c_s^2 (1 - rho_s/rho_l) dF_s/dt (Eq. 26) and its
 * companions (Eqs. 27, 40, 51) couple solidification to the flow.
 *
 * Conventions
 *   - Lattice units: cell size dx (default 1), c_s^2 = 1/3, streaming step
 *     delta_t with 0 < delta_t <= dx/2 (half the smallest cell on a stretched
 *     mesh), fixed update step dt.
 *   - Fields are planes of nx*ny values, row-major, x fastest (index
 *     j*nx + i, cell centre ((i+1/2) dx, (j+1/2) dx) on a uniform mesh).
 *   - Stretched meshes: optional column widths and row heights (see
 *     eulbfs_params.x_width) make the mesh a tensor product of unequal cells.
 *   - Every function returns EULBFS_OK (0) or a negative status; the text of
 *     the last failure is returned by eulbfs_last_error().
 *   - A handle is used by one host thread at a time.  All device work is
 *     enqueued on the stream given at creation (NULL: the default stream).
 *   - Device memory: the caller may pass a workspace of at least
 *     eulbfs_workspace_bytes() bytes (for example a torch uint8 tensor); the
 *     library then allocates no device memory for the state.  With a NULL
 *     workspace the library allocates and frees its own.
 *   - The readings of the paper that this library implements where the text
 *     is silent or garbled are listed with the parameter struct below.
 */
#ifndef EULBFS_H
#define EULBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EULBFS_ABI_VERSION 6u

/* status codes */
#define EULBFS_OK 0
#define EULBFS_EINVAL (-1)    /* bad argument or parameter                        */
#define EULBFS_ENOMEM (-2)    /* workspace too small or allocation failed         */
#define EULBFS_EDEVICE (-3)   /* a HIP call failed                                */
#define EULBFS_EUNSTABLE (-4) /* NaN/Inf, speed above c_s or C out of range; poisoned */
#define EULBFS_EBUSY (-5)     /* no free slot / HBM budget (batch API)            */
#define EULBFS_ENOTSUP (-6)   /* valid request this build does not provide        */

/* boundary rules for a wall side (Secs. 3.1-3.5 state them at the continuous
 * level; the discrete rules are the three-layer ghost ring described below) */
#define EULBFS_FLOW_NOSLIP 0   /* both momentum components odd               */
#define EULBFS_FLOW_FREESLIP 1 /* normal odd, tangential even (symmetry)     */
#define EULBFS_FLOW_OUTLET 2   /* both even (zero gradient); mass may leave  */
#define EULBFS_HEAT_ADIABATIC 0
#define EULBFS_HEAT_DIRICHLET 1 /* cold surface at T_w                       */

#define EULBFS_FP64 0 /* FP64 fields and arithmetic                                     */
#define EULBFS_FP32 1 /* FP32 flux arithmetic, p, M and dF_s/dt; H and C stored and combined in FP64 */

#define EULBFS_KERNEL_FUSED 0 /* one fused flux + update kernel per RK stage      */
#define EULBFS_KERNEL_SPLIT 1 /* ghost fill, primitives, face fluxes, update apart */
#define EULBFS_KERNEL_AUTO 2  /* FUSED with the tile shape that create timed
                                 fastest on the initial state (cached per
                                 process for the grid, precision and lattice);
                                 FUSED 32x16 (FP64) or 32x32 (FP32) on a
                                 stretched mesh */

/* One side of the domain.  Sides are indexed 0: x-, 1: x+, 2: y-, 3: y+.
 * periodic must agree on opposite sides.  For a wall:
 *   ghost layer k = 1..3 mirrors interior layer k-1; pressure even; momentum
 *   by `flow`; H even (adiabatic) or, for a Dirichlet wall, T_g = 2 T_w -
 *   T_mirror and H_g from the inverse of Eqs. (5)-(6); wetting C_g = C_mirror
 *   + (2k-1) dx (4/xi) cos(theta) C_w (1 - C_w), with C_w the first interior
 *   cell (theta = 90 deg is a plain no-flux mirror).  On the wall face the
 *   mass flux is 0 (unless outlet), the phase-field flux is 0 and the heat
 *   flux is 0 when adiabatic. */
typedef struct {
    int32_t periodic;
    int32_t flow;
    int32_t heat;
    int32_t reserved;
    double T_w;       /* EULBFS_HEAT_DIRICHLET wall temperature           */
    double theta_deg; /* equilibrium contact angle through the liquid, deg */
    double theta_adv; /* contact-angle hysteresis window [theta_rec,      */
    double theta_rec; /* theta_adv], deg; 0, 0: none (see below)          */
} eulbfs_bc;
/* Wetting wall (Secs. 3.4-3.5): the ghost C of layer k (k = 1, 2, 3 outward)
 * is C of the mirrored cell + (2k - 1) dx (4/xi) cos(theta) C_w (1 - C_w), C_w
 * the first interior cell, i.e. dC/dn = -(4/xi) cos(theta) C (1 - C) at the
 * wall; theta = 90 deg is a plain no-flux wall.  Sec. 3.5 names advancing and
 * receding angles without a rule for them; with a window, theta is the
 * apparent angle of the first three interior cells along the normal (dC/dn at
 * the wall from the quadratic through their centres) clamped to [theta_rec,
 * theta_adv]: a contact line inside the window keeps its angle, one outside
 * is driven to the nearer bound.  Where C_w (1 - C_w) <= 1e-3 theta_deg is
 * used.  A window needs 0 < theta_rec <= theta_deg <= theta_adv < 180. */

/* Problem parameters (all in lattice units).
 * Readings of the paper implemented by this library:
 *   - D2Q9 weights 4/9, 1/9, 1/36; D2Q5 weights 1/3, 1/6; c_s^2 = 1/3.
 *   - f* = f^eq(x_f) + (1 - 1/(2 tau_f)) f^neq-m (Eq. 37 prints '-').
 *   - mu_c = 2 beta C(C-1)(2C-1) - kappa lap C, beta = 12 sigma/xi,
 *     kappa = 3 xi sigma/2 (Sec. 2.3.1 prints '+ kappa').
 *   - f^eq-m (Eqs. 33-34): f^eq with the old-level face density, without the
 *     leading 1 of Gamma.
 *   - C source of Eq. (40) kept in row 5 of F_E (Eq. 51 prints 0 there).  The
 *     paper's F_s in Eq. (40) is 1 - F_l, the solid share of the condensed
 *     phase, and C d(1 - F_l)/dt is the rate at which the cell's volume turns
 *     solid; the source is (1 - rho_s/rho_l) dF_s/dt with the cell's solid
 *     fraction F_s = C (1 - F_l), the lagged rate of the volume source of
 *     Eq. (26), so the condensed volume grows by exactly the dilatation of the
 *     freezing material (c_source = 0).  c_source = 1 multiplies that rate by
 *     C once more (the printed factor applied to the cell's F_s), which loses
 *     (1 - r) xi/4 of condensed volume per unit length of frozen interface.
 *   - C_p,ref = (C_p,s + C_p,l)/2; H = C_p T + L F_l in all phases; the solid
 *     fraction entering Eq. (7) is F_s = C (1 - F_l); C and F_s clamped to
 *     [0, 1] where they enter Eq. (7) or the closure.
 *   - central gradients, 5-point Laplacian, points on the face average both
 *     sides' extrapolations (Eq. 54), old-level face values are the average
 *     of both sides' extrapolations to the face centre.
 *   - dF_s/dt lagged by one step; momentum projected M <- (1 - F_s) M after
 *     each RK stage (rigid solid, Eq. 25).
 */
typedef struct {
    uint32_t struct_size; /* sizeof(eulbfs_params)                       */
    uint32_t abi_version; /* EULBFS_ABI_VERSION                          */
    int32_t nx, ny;       /* cells; >= 4 each                            */
    int32_t lattice_hg;   /* 9 (paper) or 5: lattice of h and g          */
    int32_t precision;    /* EULBFS_FP64 or EULBFS_FP32                  */
    int32_t kernel;       /* EULBFS_KERNEL_*: FUSED (any tile) and AUTO
                             give the same bits, SPLIT agrees to rounding */
    int32_t surf_model;   /* 0: F_surf = -C grad mu_c (Sec. 2.4)
                             1: F_surf = -F_l C grad mu_c (Sec. 3.5)     */
    double dx;            /* cell size (along a direction with no width
                             array, see x_width below)                   */
    double delta_t;       /* streaming step (Sec. 2.5 step 1)            */
    double dt;            /* update step of Eq. (58)                     */
    double rho[3], mu[3], lambda[3], cp[3]; /* [solid, liquid, gas], Eq. (7) */
    double latent;        /* L                                           */
    double T_s, T_l;      /* solidus, liquidus (Eqs. 5-6); T_s <= T_l    */
    double sigma, xi;     /* surface tension, interface width            */
    double mobility, Qg;  /* M_c and Q_g of Eq. (41): tau_g = 1/2 + M_c/(Q_g delta_t) */
    double gx, gy;        /* gravity; G = rho g in Eq. (51)              */
    eulbfs_bc bc[4];
    int32_t tile_x, tile_y; /* fused-kernel tile (32x8, 64x4, 16x16, 64x8,
                               32x16, 32x32); 0 picks 32x8; AUTO ignores it */
    const double* x_width;  /* host array of nx column widths, or NULL: dx     */
    const double* y_width;  /* host array of ny row heights, or NULL: dx       */
    int32_t c_source;       /* C source of Eq. (40), 0 or 1 (readings above)   */
    int32_t reserved;
} eulbfs_params;
/* Stretched meshes (Eq. 52 holds for any cell; the paper runs uniform ones).
 * With x_width or y_width set the mesh is the tensor product of those cells:
 * column i spans [sum_{m<i} w_m, sum_{m<=i} w_m], V = w_i h_j, S = h_j on x
 * faces and w_i on y faces.  Gradients and lap(C) are the derivatives of the
 * parabola through a cell centre and its two neighbours (the central
 * differences of a uniform mesh); Eq. (54) extrapolates from each cell by its
 * own half width to the face; one delta_t for the whole mesh, at most half
 * the smallest width.  Ghost cells take the width of the cell they copy, so a
 * wall lies midway between a ghost and its mirror: the wetting offset uses
 * the distance between them in place of (2k - 1) dx, and the hysteresis
 * angle reads dC/dn from the parabola through the first three cell centres.
 * Widths must be finite and > 0; both arrays are copied by eulbfs_create and
 * may be freed afterwards.  FUSED and AUTO run such a mesh on the fused kernel
 * with 32x16 tiles in FP64 and 32x32 in FP32 (tile_x and tile_y are ignored,
 * nothing is autotuned), SPLIT on the split kernels; a batch steps it with its
 * 32x16 tiles (every tile shape gives the same bits).
 * Diagnostic integrals weight each cell by w_i h_j and the tip height by h_j. */

/* Initial state. */
#define EULBFS_INIT_PRIMITIVE 0 /* 6 planes: T, F_l, C, u, v, p                */
#define EULBFS_INIT_CONSERVED 1 /* 6 planes: H, p, Mx, My, C, dF_s/dt (restart) */
#define EULBFS_INIT_ANALYTIC 2  /* the closed-form fields of *shape, built on the
                                   device; planes and on_device are not read   */

/* Closed-form initial fields (EULBFS_INIT_ANALYTIC).  With cell centres x_i,
 * y_j ((i + 1/2) dx on a uniform mesh, the running sums of the widths on a
 * stretched one):
 *   C    UNIFORM: c0.  LAYER: the flat interface of Eq. (61) at s = h0,
 *        (1 + tanh(2 (h0 - s) / xi)) / 2 with s = x_i (axis 0) or y_j (axis 1).
 *        DROPLET: the circle of Eq. (62) (with the distance to the centre),
 *        (1 + tanh(2 (r0 - r) / xi)) / 2, r = sqrt((x_i - x0)^2 + (y_j - y0)^2).
 *   T    t_in where C > 1/2, else t_out; plus t_amp times a number uniform in
 *        [-1, 1) drawn for cell n = j nx + i by the splitmix64 generator (state
 *        seed + (n + 1) 0x9E3779B97F4A7C15, its output mix, top 53 bits) when
 *        t_amp is not 0.
 *   F_l  fl0.   u, v  u_in C, v_in C (0 where u_in, v_in are 0).   p  0.
 * These primitive fields then take the EULBFS_INIT_PRIMITIVE path. */
#define EULBFS_PROFILE_UNIFORM 0
#define EULBFS_PROFILE_LAYER 1
#define EULBFS_PROFILE_DROPLET 2
typedef struct {
    int32_t profile;      /* EULBFS_PROFILE_*                            */
    int32_t axis;         /* LAYER: 0 across x, 1 across y               */
    double c0;            /* UNIFORM: C                                  */
    double h0;            /* LAYER: position of C = 1/2                  */
    double x0, y0, r0;    /* DROPLET: centre and radius                  */
    double t_out, t_in;   /* T where C <= 1/2 and where C > 1/2          */
    double t_amp;         /* amplitude of the seeded temperature noise   */
    uint64_t seed;
    double fl0;           /* F_l                                         */
    double u_in, v_in;    /* velocity per unit C                         */
} eulbfs_shape;

typedef struct {
    int32_t kind;
    int32_t on_device;    /* 1: planes point to device memory             */
    const double* planes; /* 6 * nx * ny doubles, plane after plane       */
    const eulbfs_shape* shape; /* EULBFS_INIT_ANALYTIC: host memory, read
                                  before the call returns              */
} eulbfs_init;
/* EULBFS_INIT_PRIMITIVE: H = (1 - F_l)(H_s + C_p^S (T - T_s)) + F_l (H_l +
 * C_p^L (T - T_l)) with H_s = C_p^S T_s, H_l = C_p^L T_l + L (so a liquid
 * given below T_m recalesces to the heat-balance state of Sec. 3.4), and
 * M = rho c_s^2 (u, v) with rho from Eq. (7) after the closure of that H.
 * The planes are copied before eulbfs_create returns. */

/* Field and scalar selectors for eulbfs_query / eulbfs_set_field.
 * Fields: nx*ny doubles (converted from FP32 storage when precision is FP32). */
#define EULBFS_FIELD_H 0
#define EULBFS_FIELD_P 1
#define EULBFS_FIELD_MX 2
#define EULBFS_FIELD_MY 3
#define EULBFS_FIELD_C 4
#define EULBFS_FIELD_FSDOT 5 /* lagged dF_s/dt                                 */
#define EULBFS_FIELD_T 6
#define EULBFS_FIELD_FL 7
#define EULBFS_FIELD_FS 8
#define EULBFS_FIELD_RHO 9
#define EULBFS_FIELD_U 10
#define EULBFS_FIELD_V 11
#define EULBFS_FIELD_MUC 12
#define EULBFS_FIELD_W_ALL 13    /* 6 planes: H, p, Mx, My, C, dF_s/dt (checkpoint) */
#define EULBFS_FIELD_W_GHOSTED 14 /* 5 planes of (nx+6)*(ny+6): state with its ghost ring */
/* Scalars: EULBFS_SCALAR_DIAG fills EULBFS_NDIAG doubles:
 *   [0] sum rho dV, [1] sum C dV, [2] sum H dV, [3] sum F_s dV, [4] max |u|,
 *   [5] non-finite cell count, [6] sum_j F_s(nx/2, j) dy (tip height on the
 *   middle column), [7] time, [8] steps taken, [9] dt, [10] min C,
 *   [11] max C, [12] sum_i clamp(C(i, 0)) dx (wetted length on the y- wall:
 *   the spreading diameter D of Sec. 3.5 for a drop on that wall, D/D_0 its
 *   spreading factor), [13] sum_j clamp(C(nx/2, j)) dy (height of the
 *   condensed phase on the middle column: the apex or bounce height H_b of
 *   Sec. 3.5, Table 7, for a drop centred there)
 * Widths replace dx and dy on a stretched mesh.  The sums are FP64 and
 * deterministic (fixed two-pass order, no atomics). */
#define EULBFS_SCALAR_DIAG 100
#define EULBFS_NDIAG 14
/* Watchdog (eulbfs_run, eulbfs_query, eulbfs_batch_query of the integrals): the
 * state is unstable when a cell is non-finite, a speed exceeds the lattice
 * sound speed c_s = 1/sqrt(3), or the order parameter leaves [-EULBFS_C_MARGIN,
 * 1 + EULBFS_C_MARGIN] (F_s = clamp(C)(1 - F_l) itself is in [0, 1] by
 * construction). */
#define EULBFS_C_MARGIN 0.5

/* Host-only: validate parameters.  msg (may be NULL) receives the reason.
 * Besides the ranges stated above: xi must span two cells (2 dx, the smallest
 * width on a stretched mesh), and dt must lie within the stability bounds of
 * the explicit SSP-RK3 step (-2.51 on the real axis, sqrt(3) on the imaginary
 * one) for the diffusive processes on the actual mesh: heat (largest lambda /
 * (rho C_p) of the phases), momentum (2 mu / rho + c_s^2 delta_t, the
 * compressive viscous mode of the flux), the Cahn-Hilliard operator
 * M_c (kappa l^2 + 2 beta l) and the acoustic mode c_s dt (1/dx + 1/dy), with
 * l the largest eigenvalue of the compact finite-volume Laplacian on the mesh
 * (wall cells stiffer where the value is held: Dirichlet temperature, no-slip
 * momentum). */
int eulbfs_check_params(const eulbfs_params* prm, char* msg, size_t msg_len);

/* Host-only: bytes of device workspace a solver with these parameters needs
 * (0 if the parameters are invalid). */
size_t eulbfs_workspace_bytes(const eulbfs_params* prm);

/* Create a solver: validates prm, carves the workspace (d_ws, ws_bytes) or
 * allocates one (d_ws == NULL), writes the initial state.  hip_stream is a
 * hipStream_t (NULL: default stream).  On failure *out is NULL. */
int eulbfs_create(const eulbfs_params* prm, const eulbfs_init* init, void* d_ws, size_t ws_bytes,
                  void* hip_stream, struct eulbfs_solver** out);
typedef struct eulbfs_solver* eulbfs_t;

/* Enqueue nsteps SSP-RK3 steps (Eq. 58); asynchronous. */
int eulbfs_step(eulbfs_t h, int64_t nsteps);

/* eulbfs_step of min(nsteps, the steps that bring the time to t_end) (the
 * fixed dt reaches t_end after ceil((t_end - t)/dt) steps; t_end = INFINITY
 * for nsteps alone; NaN is EULBFS_EINVAL), then synchronise the stream and
 * run the watchdog: EULBFS_EUNSTABLE (and a poisoned handle) if a cell is
 * non-finite, a speed |u| exceeds the lattice sound speed c_s = 1/sqrt(3)
 * (the flux reconstruction assumes low Mach number) or C leaves its range
 * (EULBFS_C_MARGIN). */
int eulbfs_run(eulbfs_t h, int64_t nsteps, double t_end);

/* Read a field (EULBFS_FIELD_*) or the diagnostics (EULBFS_SCALAR_DIAG) into
 * out (bytes large enough; host memory unless out_on_device).  Synchronises.
 * The diagnostics go through the watchdog of eulbfs_run; on an unstable state,
 * or a handle poisoned before, the output is still written and the call
 * returns EULBFS_EUNSTABLE. */
int eulbfs_query(eulbfs_t h, int32_t what, void* out, size_t bytes, int32_t out_on_device);

/* Overwrite one conserved plane (FIELD_H..FIELD_FSDOT) or all six
 * (FIELD_W_ALL) from nx*ny doubles per plane.  Synchronises. */
int eulbfs_set_field(eulbfs_t h, int32_t what, const void* in, size_t bytes, int32_t in_on_device);

/* Evaluate the residual R(W) of Eq. (57) for the current state with the
 * split kernels: R (5 planes nx*ny), Fx (5 planes (nx+1)*ny, face i at
 * x = i dx), Fy (5 planes nx*(ny+1), face j at y = j dx); any may be NULL.
 * Doubles, host memory unless on_device.  A diagnostic call: it allocates
 * temporary device scratch (freed before it returns) unless the solver was
 * created with EULBFS_KERNEL_SPLIT, whose workspace holds it.  Synchronises. */
int eulbfs_residual(eulbfs_t h, double* R, double* Fx, double* Fy, int32_t on_device);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): eulbfs_residual with
 * its device scratch (split-kernel planes, residual planes, staging) in a
 * static array of EULBFS_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends, instead of a temporary
 * allocation.  Same arguments, outputs and synchronisation as eulbfs_residual;
 * calls no hipMalloc or hipFree.  The solver's device must be current.
 * EULBFS_EINVAL when the grid needs more scratch than the array holds (square
 * grids up to 495 x 495 cells in FP64, 634 x 634 in FP32).  Every call on one device shares that device's
 * array (nothing in it has to start at zero; it keeps the last call's
 * contents): calls that overlap on one device race. */
#define EULBFS_NOALLOC_SCRATCH_BYTES (64u << 20)
int eulbfs_residual_noalloc(eulbfs_t h, double* R, double* Fx, double* Fy, int32_t on_device);

/* Release a solver; NULL is accepted. */
int eulbfs_destroy(eulbfs_t h);

/* The schedule a solver steps with: kernel is EULBFS_KERNEL_FUSED or _SPLIT
 * (AUTO resolves to FUSED), tile_x x tile_y the fused kernel's tile (the one
 * EULBFS_KERNEL_AUTO picked; on a stretched mesh 32 x 16 in FP64, 32 x 32 in
 * FP32; 0 x 0 for the split kernels).  Any output
 * pointer may be NULL.  Host call, no device work.  Returns EULBFS_EINVAL for
 * a NULL handle. */
int eulbfs_schedule(eulbfs_t h, int32_t* kernel, int32_t* tile_x, int32_t* tile_y);

/* Text of the last failure on this handle (or, for h == NULL, of the last
 * failure of a create or host-only call on this thread). */
const char* eulbfs_last_error(eulbfs_t h);

/* ---------------------------------------------------------------------------
 * Batched solves (many independent grids of uneven size advanced by one
 * launch per RK stage over the tiles of all of them).  A batch owns one device arena; requests
 * are admitted into slots while their footprint fits the HBM budget.
 * ------------------------------------------------------------------------- */
typedef struct eulbfs_batch* eulbfs_batch_t;

/* Create a batch with an arena of hbm_budget bytes (allocated by the library
 * when d_ws is NULL, else carved from d_ws of ws_bytes >= hbm_budget, 256-byte
 * aligned) and at most max_slots resident requests, all of one precision
 * (EULBFS_FP64 or EULBFS_FP32).  Work is enqueued on hip_stream. */
int eulbfs_batch_create(size_t hbm_budget, int32_t max_slots, int32_t precision, void* d_ws,
                        size_t ws_bytes, void* hip_stream, eulbfs_batch_t* out);

/* Footprint in the arena of one request with these parameters. */
size_t eulbfs_batch_request_bytes(const eulbfs_params* prm);

/* Admit a request that will run nsteps steps.  Its initial state is copied
 * into the arena before the call returns (host planes through pinned memory
 * on the batch's own upload stream, which the batch stream waits for) without
 * waiting for the ticks in flight.  EULBFS_EBUSY when no slot or not
 * enough contiguous arena is free; EULBFS_EINVAL for bad parameters or a
 * precision that differs from the batch's.  *slot receives the slot index.
 * The request steps with the batched kernel (the batch's tile shape, below)
 * whatever its kernel and tile fields say. */
int eulbfs_batch_admit(eulbfs_batch_t b, const eulbfs_params* prm, const eulbfs_init* init,
                       int64_t nsteps, int32_t* slot);

/* Advance every resident unfinished request by the same number of steps:
 * min(steps, the smallest number of steps any of them still has to run),
 * with one launch per RK stage (per h/g lattice and fast-path group present)
 * over the tiles of all of them.  Enqueues and returns; waits only while two
 * earlier ticks are still running on the device.  A tick that finishes a
 * request also enqueues its FP64 integrals, copied to pinned host memory. */
int eulbfs_batch_tick(eulbfs_batch_t b, int32_t steps);

/* Slots whose requests have finished on the device (up to cap), in slot
 * order.  Does not block. */
int eulbfs_batch_poll(eulbfs_batch_t b, int32_t* done, int32_t cap, int32_t* n);

/* eulbfs_query on the request in a slot.  EULBFS_SCALAR_DIAG of a finished
 * request (as reported by eulbfs_batch_poll) into host memory is read from the
 * pinned copy without waiting; every other query synchronises. */
int eulbfs_batch_query(eulbfs_batch_t b, int32_t slot, int32_t what, void* out, size_t bytes,
                       int32_t out_on_device);

/* Free a slot and its arena range.  Waits for the stream only when the request
 * has not finished on the device (its planes may still be in use). */
int eulbfs_batch_release(eulbfs_batch_t b, int32_t slot);

/* Tile shape of the batched kernel for requests on uniform meshes (requests
 * on stretched meshes always take 32 x 16).  EULBFS_BATCH_TILE_AUTO, the
 * default, picks it on the live mix: every tick's launches are timed with
 * events, and two back-to-back ticks that advance the same requests by the
 * same steps with different shapes give a paired sample of their time ratio.
 * Until the first pair the ticks alternate between the shapes; then a tick
 * runs the shape that the running geometric mean of the paired ratios
 * favours, and every EULBFS_BATCH_EXPLORE-th tick the other one (a mix that
 * yields no pair within 4 * EULBFS_BATCH_EXPLORE timed ticks of each shape is
 * judged by the summed time per cell-step of each shape instead).  The fixed
 * values pin one shape.  Every shape gives the same bits.  EULBFS_EINVAL for
 * another value. */
#define EULBFS_BATCH_TILE_AUTO 0
#define EULBFS_BATCH_TILE_32x16 1
#define EULBFS_BATCH_TILE_64x8 2
#define EULBFS_BATCH_EXPLORE 8
int eulbfs_batch_set_tile(eulbfs_batch_t b, int32_t tile);

/* What the tile choice has measured (completed ticks only; no blocking). */
typedef struct eulbfs_batch_sched {
    int32_t next_tile;            /* EULBFS_BATCH_TILE_32x16 or _64x8: the shape of the next tick */
    int32_t reserved;
    double ns_per_cell_step[2];   /* device time per cell-step over every timed tick of each shape
                                     (32 x 16, 64 x 8); 0 before the first */
    int64_t ticks_timed[2];
    double time_ratio;            /* time of 64 x 8 over 32 x 16 on paired ticks (running geometric
                                     mean); 0 before the first pair */
    int64_t pairs;
} eulbfs_batch_sched;
int eulbfs_batch_schedule(eulbfs_batch_t b, eulbfs_batch_sched* out);

int eulbfs_batch_destroy(eulbfs_batch_t b);

const char* eulbfs_batch_last_error(eulbfs_batch_t b);

#ifdef __cplusplus
}
#endif
#endif /* EULBFS_H */
