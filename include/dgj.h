/*
 * dgj: implicit discontinuous-Galerkin compressible Navier-Stokes hot path
 * on AMD MI355X (gfx950).  C ABI.
 *
 * Method: arxiv 2002.04222, "Implicit high-order discontinuous Galerkin
 * compressible flow solver" (Nektar++).  The library evaluates
 *   R(u) = M^-1 L(u)                               (Sec. 3.1, Eq. 13)
 *   N(u) = u - S - dt a M^-1 L(u)                  (Sec. 3.2, Eq. 20)
 *   J v ~ (N(u + eps v) - N(u)) / eps              (Sec. 4.2.2, Eq. 25-26)
 *   P^-1 q by block-relaxed Jacobi BRJ(J)          (Sec. 4.2.2, Eq. 27-31)
 * and advances u by implicit Runge-Kutta (SDIRK2/3/4, backward Euler), BDF2
 * or explicit ERK2 steps (Sec. 3.2, Sec. 4.3, Appendix A), the implicit ones
 * with Newton (Eq. 21-23) and restarted right-preconditioned GMRES (Eq. 24).
 * Viscous face terms by interior penalty (Eq. 12) or LDG; Roe, LLF, HLL,
 * HLLC or AUSM+ Riemann fluxes; the boundary kinds of Sec. 4.3; affine boxes
 * or curved isoparametric elements (Sec. 3.1).
 *
 * Conventions for every entry point below:
 *  - Array arguments are DEVICE pointers (on the device current when the
 *    context was created) to caller-owned, contiguous FP64 buffers, unless
 *    the parameter description says "host".  The library never frees them.
 *  - State layout is [element][variable][mode]: variables
 *    (rho, rho u_1..rho u_d, E); modes of the orthonormal tensor Legendre
 *    basis phi_i(xi) = sqrt((2i+1)/2) P_i(xi) on [-1,1]^d, mode index
 *    i + n (j + n k), x fastest, n = P + 1.  n_unknowns = n_elem (d+2) n^d.
 *  - Elements are affine boxes or isoparametric maps of the reference
 *    cube (dgj_mesh.geo_nodes); faces are f = 2*axis + side (side 0 at
 *    xi_axis = -1).  face_nbr[e][f] is the element across face f, which
 *    meets it with its face 2*axis + (1 - side), face points aligned, or
 *    marks a boundary face (dgj_mesh).
 *  - Work is enqueued on the context's stream.  Entry points that need a
 *    scalar on the host (norms for eps, chi and the GMRES Hessenberg
 *    entries) synchronise that stream; the rest are asynchronous.
 *  - Every int-returning function returns DGJ_OK or a negative status; the
 *    message of the last failure is available from dgj_last_error().
 *    Inputs are not modified on failure except where stated.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef DGJ_H
#define DGJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DGJ_OK = 0,
  DGJ_EINVAL = -1,       /* bad argument */
  DGJ_EHIP = -2,         /* HIP runtime error */
  DGJ_ENOMEM = -3,       /* device allocation failed */
  DGJ_ENOTCONV = -4,     /* Newton budget exhausted */
  DGJ_ENAN = -5,         /* non-finite norm met */
  DGJ_ESINGULAR = -6,    /* zero pivot in a preconditioner block */
  DGJ_EUNSUPPORTED = -7  /* combination of sizes or options not built */
};

/* Time integrators (Sec. 4.3, Appendix A).  SDIRK4 is the six-stage table with
 * an explicit first stage, its first column equal to the second and its
 * abscissae the row sums; BDF2 is the constant-step form with a
 * backward-Euler start; ERK2 is explicit (no preconditioner, no Newton). */
enum { DGJ_BEULER = 1, DGJ_SDIRK2 = 2, DGJ_SDIRK3 = 3, DGJ_SDIRK4 = 4, DGJ_BDF2 = 12, DGJ_ERK2 = 20 };
#define DGJ_MAX_STAGES 6
enum { DGJ_PC_F64 = 0, DGJ_PC_F32 = 1, DGJ_PC_BF16 = 2 };

typedef struct dgj_ctx dgj_ctx;

/* Boundary condition kinds.  No formulas are given in the paper, which
 * only names the kinds its solver offers (Sec. 4.3): all of them are built,
 * with the readings below (periodic faces are ordinary interior faces;
 * symmetry and slip wall are one kind; time-dependent Dirichlet data are
 * given by setting the field again between steps).  A boundary face takes the interior trace and
 * a ghost state with the interior gradient, and the interior face fluxes
 * (Riemann flux, interior-penalty viscous terms) apply:
 *  DGJ_BC_FARFIELD: 1D characteristic far field.  With u_n the outward
 *    normal velocity and c the sound speed, R+ = u_n + 2c/(gamma-1) comes
 *    from the interior and R- = u_n - 2c/(gamma-1) from the freestream;
 *    tangential velocity and entropy p/rho^gamma come from the interior
 *    where u_nb = (R+ + R-)/2 > 0, else from the freestream, blended by
 *    w = (1 + tanh(u_nb / (0.02 c_b)))/2, c_b = (gamma-1)(R+ - R-)/4, so that
 *    the ghost state is differentiable where u_nb changes sign (a sharp
 *    switch there stalls Newton).  Supersonic inflow: the freestream state;
 *    supersonic outflow: the interior state.
 *  DGJ_BC_WALL: adiabatic no-slip wall.  Ghost = interior with the
 *    momentum negated (zero wall velocity); the energy components of the
 *    viscous flux and of the symmetric interior-penalty term are zero (no
 *    heat flux through the wall).
 *  DGJ_BC_DIRICHLET: the ghost state is a given state at every face point
 *    (dgj_set_bc_field), e.g. an exact solution applied weakly.
 *  DGJ_BC_SLIP: slip wall / symmetry plane.  Ghost = interior with the
 *    normal momentum mirrored; no heat flux and no tangential viscous
 *    traction (only the normal viscous traction) through the face.
 *  DGJ_BC_ISOTHERMAL: no-slip wall at the temperature of the id's state.
 *    Ghost: velocity negated, interior pressure, temperature mirrored
 *    about the wall temperature (a fluid at rest sees a stationary contact).
 *  DGJ_BC_EXTRAPOLATE: zero-order extrapolation, ghost = interior.
 *  DGJ_BC_PRESSURE_OUT: ghost = interior with the id's pressure where the
 *    outflow is subsonic, the interior state where supersonic.
 *  DGJ_BC_PRESSURE_IN: ghost = the id's density and velocity with the
 *    interior pressure where the inflow is subsonic, the id's state where
 *    supersonic. */
enum { DGJ_BC_FARFIELD = 0, DGJ_BC_WALL = 1, DGJ_BC_DIRICHLET = 2, DGJ_BC_SLIP = 3, DGJ_BC_ISOTHERMAL = 4,
       DGJ_BC_EXTRAPOLATE = 5, DGJ_BC_PRESSURE_OUT = 6, DGJ_BC_PRESSURE_IN = 7 };

/* Mesh of affine boxes (host arrays, copied by dgj_create). */
typedef struct {
  int32_t dim;                /* 2 or 3 */
  int32_t P;                  /* polynomial order per direction */
  int32_t nq;                 /* Gauss points per direction (P+2 built) */
  int64_t n_elem;
  const double *elem_origin;  /* host [n_elem][dim] lower corner */
  const double *elem_h;       /* host [n_elem][dim] edge lengths */
  const int32_t *face_nbr;    /* host [n_elem][2*dim]: element across the face, or -(id+1)
                                 for a face on boundary id (0 <= id < n_bc) */
  int32_t n_bc;               /* number of boundary ids; 0 for periodic meshes */
  const int32_t *bc_kind;     /* host [n_bc]: one of the DGJ_BC_* kinds (NULL if n_bc = 0) */
  const double *bc_state;     /* host [n_bc][dim+2]: the given conserved state of each far-field,
                                 isothermal-wall and pressure id (rho > 0, p > 0); entries of
                                 the other ids are not read */
  int32_t geo_order;          /* curved elements: order g of the element maps (1..7) */
  const double *geo_nodes;    /* host [n_elem][(g+1)^dim][dim] or NULL (affine boxes).  When
                                 set, elements are isoparametric: x(xi) = sum_c X_c l_c(xi),
                                 tensor Lagrange polynomials through the equispaced nodes
                                 -1 + 2i/g, node c = i0 + (g+1)(i1 + (g+1) i2); every map must
                                 have a positive Jacobian at the Gauss points.  Neighbours
                                 must share their face nodes (face points aligned as above).
                                 elem_origin and elem_h are then not read.  Curved meshes
                                 carry per-point metrics and a dense mass matrix per element
                                 (Sec. 3.1), and dgj_project_tgv is not available on them. */
} dgj_mesh;

/* Non-dimensional gas and flux options (Sec. 2). */
typedef struct {
  double gamma, Pr, Re, Ma;
  double T_ref_K;             /* Sutherland reference temperature, kelvin */
  int32_t visc_law;           /* 0 constant mu = 1/Re, 1 Sutherland */
  int32_t flux_mode;          /* 0 Navier-Stokes, 1 Euler, 2 scalar diffusion test */
  int32_t riemann;            /* 0 Roe, 1 local Lax-Friedrichs, 2 HLL, 3 HLLC, 4 AUSM+ (Sec. 4.3 lists
                                 these among its solver's fluxes) */
  int32_t viscous;            /* viscous face terms (Sec. 4.3 names both): 0 interior penalty
                                 (Eq. 12), 1 LDG -- auxiliary gradient q = grad u + the lifted
                                 face jumps (u_hat from the face's left element, the element that
                                 meets it with side 1, or the mean of interior and ghost states on
                                 a boundary), viscous flux with q_hat from the right element and
                                 a penalty on the jump, no symmetric term.  LDG runs on affine
                                 boxes and single instances; its preconditioner blocks are the
                                 interior-penalty ones. */
} dgj_phys;

/* Implicit solver options (Sec. 3.2, Sec. 4.2.2). */
typedef struct {
  int32_t scheme;             /* DGJ_SDIRK2, DGJ_SDIRK3, DGJ_SDIRK4, DGJ_BEULER, DGJ_BDF2 or
                                 DGJ_ERK2 (batches: SDIRK2 and SDIRK3 only) */
  double newton_rtol;         /* alpha of Eq. 23 */
  int32_t newton_max;
  int32_t gmres_restart;      /* 30 in the paper; 1..60 */
  double gmres_rtol;          /* 5e-2 in the paper */
  int32_t gmres_max;          /* total GMRES iterations per Newton step */
  int32_t brj_sweeps;         /* J of Eq. 28 (7) */
  double brj_omega;           /* omega of Eq. 28 (1) */
  int32_t pc_precision;       /* DGJ_PC_F64 / F32 / BF16 storage of D^-1 */
  int32_t pc_freeze;          /* steps a built preconditioner is kept (10) */
  int32_t pc_refresh_its;     /* single instances: rebuild the preconditioner at S_m before a
                                 stage when the last Newton step's GMRES took more iterations
                                 than this, and retry a failed stage once from S_m with blocks
                                 rebuilt at S_m (0: the paper's fixed freeze only); not in the
                                 paper, which keeps the blocks for pc_freeze steps */
  int32_t ortho;              /* GMRES orthogonalisation: 0 modified Gram-Schmidt (one projection
                                 at a time), 1 classical Gram-Schmidt applied twice (all
                                 projections of a pass at once: two batched reductions per
                                 iteration instead of k + 1; single instances only) */
} dgj_solver;

/* Per-step statistics filled by dgj_sdirk_step. */
typedef struct {
  int32_t stages;
  int32_t newton_its[DGJ_MAX_STAGES];      /* 0 for an explicit stage */
  int32_t gmres_its[DGJ_MAX_STAGES][64];   /* per stage, per Newton iteration */
  double nres[DGJ_MAX_STAGES][65];         /* ||N|| per stage before each Newton iteration and at exit */
  int32_t pc_built;           /* 1 if this step (re)built the preconditioner */
  int32_t residual_evals;     /* residual evaluations in the step */
  int32_t status;
  double t_total_ms;          /* host wall time of the step */
  double t_pc_build_ms;       /* of which preconditioner build */
  int32_t guess_used[DGJ_MAX_STAGES];      /* per stage: 0 S_m, 1 extrapolated, 2 learned */
  double guess_norm[DGJ_MAX_STAGES][3];    /* ||N|| of the S_m, extrapolated and learned guesses
                                              (0 if not evaluated) */
  double guess_blend[DGJ_MAX_STAGES][2];   /* the learned blend weights (c0, c1) (0 if not evaluated) */
} dgj_step_stats;

/* Create a context on the current device for the discretisation of Sec. 3.1
 * (Eq. 9-13: mesh, basis, quadrature, gas of Sec. 2) and the implicit solver
 * of Sec. 3.2 and 4.2.2 (options above); hip_stream may be NULL (default
 * stream).  Copies the mesh and options; allocates the library's device
 * workspaces (freed by dgj_destroy); the preconditioner's blocks and build
 * scratch are allocated by the first dgj_precond_build or step and kept. */
int dgj_create(const dgj_mesh *mesh, const dgj_phys *phys, const dgj_solver *solver, void *hip_stream,
               dgj_ctx **out);
void dgj_destroy(dgj_ctx *ctx);
/* Number of FP64 unknowns of one state vector. */
int dgj_sizes(const dgj_ctx *ctx, int64_t *n_unknowns);
const char *dgj_last_error(const dgj_ctx *ctx);

/* Initial condition: L2 projection (Sec. 3.1) of the Taylor-Green vortex
 * at T = 1 (2D: u = sin x cos y, v = -cos x sin y, p = p_inf +
 * (cos 2x + cos 2y)/4; 3D: u = sin x cos y cos z, v = -cos x sin y cos z,
 * w = 0, p = p_inf + (cos 2x + cos 2y)(cos 2z + 2)/16; rho = p / p_inf,
 * p_inf = 1/(gamma Ma^2)), plus noise_amp * sigma_v * noise on every
 * coefficient, sigma = (1,..,1, p_inf/(gamma-1) + 1/2).  noise may be
 * NULL.  u: output state. */
int dgj_project_tgv(dgj_ctx *ctx, const double *noise, double noise_amp, double *u);

/* R = M^-1 L(u)  (Eq. 13).  The interior-penalty residual is evaluated by
 * one fused kernel (one workgroup per element: volume terms, the modal face
 * traces of the element and of its neighbours, the face fluxes in each
 * face's canonical orientation -- every interior face by both of its
 * elements, with bitwise the same result, so element sums still cancel
 * exactly -- lifting and M^-1), the LDG residual by a volume, a face-flux and
 * a lift kernel with the traces and face fluxes staged in the context's
 * scratch. */
int dgj_residual(dgj_ctx *ctx, const double *u, double *R);
/* Evaluate the interior-penalty residual with the fused kernel (1, the
 * default) or with the three kernels (0), for comparisons: the two agree to
 * rounding (different summation orders of the traces). */
int dgj_set_residual_kernels(dgj_ctx *ctx, int32_t fused);
/* Autotuner of the residual's workgroup shapes (not in the paper).  Fused
 * kernel: times it at state u, reps launches each, with every tile of
 * elements per workgroup (2D: 1, 2, 4, 8; 3D: 1) and workgroup size (64,
 * 128, 256; 3D also 192), taken in that order, that gives each element at
 * least a thread per face point in whole half-wavefronts (3D: wavefronts),
 * and keeps the fastest; chosen = {size, elements per workgroup, 0},
 * times_ms[i] = the i-th tile's time.  Three kernels (LDG): times each kernel alone with
 * workgroups of 64, 128 and 256 threads (its other inputs left in place by
 * one evaluation) and keeps the fastest per kernel; chosen: (volume, face,
 * lift), times_ms [kernel][64, 128, 256].  chosen: host [3] or NULL;
 * times_ms: host [3][3] or NULL.  Results are unchanged (the kernels sum in
 * the same order for every workgroup size) except on curved meshes, where
 * the M^-1 product's partial sums follow the workgroup size.  Synchronises
 * the stream.  Not for batch groups (dgj_batch_autotune). */
int dgj_autotune(dgj_ctx *ctx, const double *u, int32_t reps, int32_t *chosen, double *times_ms);

/* N = u - S - dt_a M^-1 L(u)  (Eq. 20), dt_a = dt a^mm. */
int dgj_stage_residual(dgj_ctx *ctx, const double *u, const double *S, double dt_a, double *N);

/* Jv = (N(u + eps v) - N_u) / eps  (Eq. 25) with N_u = N(u) stored by the
 * caller.  eps <= 0 selects eps = ||u||_2 sqrt(2^-52) (Eq. 26; synchronises
 * to read the norm).  u + eps v is formed once per call into a buffer the
 * context owns (the rounding of the product, then the sum) and read by the
 * residual kernels as the state. */
int dgj_jfnk_matvec(dgj_ctx *ctx, const double *u, const double *N_u, const double *S, double dt_a,
                    const double *v, double eps, double *Jv);

/* Build the BRJ preconditioner at state u_p for dt_a (Eq. 29-31; the last
 * two terms of Eq. 30 dropped as in the paper).  Synchronises.  Returns
 * DGJ_ESINGULAR if a block has a zero pivot (the context then has no
 * preconditioner). */
int dgj_precond_build(dgj_ctx *ctx, const double *u_p, double dt_a);

/* out = P^-1 q by brj_sweeps sweeps of Eq. 28 from q^0 = 0.  Requires a
 * built preconditioner.  out must not alias q. */
int dgj_precond_apply(dgj_ctx *ctx, const double *q, double *out);

/* dgj_precond_apply that allocates nothing, for callers that cannot call
 * hipMalloc (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Its BRJ iterates (and the mass product of curved
 * meshes) live in a static device array of the library, 3 x 2^21 FP64
 * values (48 MiB) on every GPU it runs on, held until the process ends:
 * contexts of more than 2^21 unknowns get DGJ_EINVAL.  Every call on one GPU
 * shares that array, which keeps the last call's contents (nothing in it
 * needs to start at zero): calls that overlap on one GPU, from any context
 * or stream, race.  Same result as dgj_precond_apply (same kernels, same
 * order).  Requires a built preconditioner; out must not alias q. */
int dgj_precond_apply_static(dgj_ctx *ctx, const double *q, double *out);

/* Change the storage precision of the BRJ blocks (DGJ_PC_F64 / F32 / BF16;
 * Sec. 4.2.2 stores them in single precision) for the following builds; the
 * held preconditioner is released, so the next step or dgj_precond_apply
 * needs a build first. */
int dgj_set_pc_precision(dgj_ctx *ctx, int32_t pc_precision);

/* L2 projection onto the modes of values given at the volume Gauss points:
 * f[e][v][q] (device, q = q0 + nq (q1 + nq q2), x fastest) -> u[e][v][m],
 * u_e = M_e^-1 (integral of phi_m f over the element, by the Gauss rule)
 * (Sec. 3.1, Eq. 13's mass matrix).  Initial states, forcing terms. */
int dgj_project(dgj_ctx *ctx, const double *f, double *u);

/* Source term: s[e][v][m] (device, copied; NULL removes it) is added to
 * M^-1 L(u) in every residual the context evaluates, so R, N (Eq. 20), the
 * Frechet matvec and the steps solve M du/dt = L(u) + M s.  For a forcing f
 * of the equations, s is its projection (dgj_project). */
int dgj_set_source(dgj_ctx *ctx, const double *s);

/* Ghost states of the Dirichlet faces: g[e][f][v][p] (device, copied;
 * n_elem x 2 dim x (dim+2) x nq^(dim-1) values), f = 2 axis + side, p over the
 * face's Gauss points with the tangential reference axes in increasing
 * order, the first fastest.  Only faces whose boundary id has the Dirichlet
 * kind are read.  Needed before any residual or preconditioner build on a
 * mesh with Dirichlet boundaries (DGJ_EINVAL otherwise, or when the mesh has
 * none). */
int dgj_set_bc_field(dgj_ctx *ctx, const double *g);

/* Export of the stored inverse mass matrices of a curved mesh (tests):
 * out[e][m][n] (device, n_elem (P+1)^(2d) values).  DGJ_EINVAL on boxes. */
int dgj_mass_inverse(dgj_ctx *ctx, double *out);

/* Copy the stored block inverses, converted to FP64, into out
 * [n_elem][nb][nb] with nb = (d+2)(P+1)^d, row-major per element. */
int dgj_precond_diag_inverse(dgj_ctx *ctx, double *out);

/* Solve J x = b approximately by restarted right-preconditioned GMRES
 * (Arnoldi by the solver's ortho choice, Givens rotations, x0 = 0) with
 * the Jacobian-free J at (u, N_u, S, dt_a) and eps as in dgj_jfnk_matvec;
 * uses the built
 * preconditioner if any.  *iters receives the iteration count. */
int dgj_gmres(dgj_ctx *ctx, const double *u, const double *N_u, const double *S, double dt_a, double eps,
              const double *b, double *x, int32_t *iters);

/* Solve N(u) = 0 (Eq. 20) by Newton from the guess in u (in/out) with
 * source S; newton_its / gmres_its (host, may be NULL, gmres_its sized
 * newton_max) receive the iteration counts.  Uses the built preconditioner
 * if any. */
int dgj_newton(dgj_ctx *ctx, const double *S, double dt_a, double *u, int32_t *newton_its, int32_t *gmres_its);

/* One time step of size dt on u (in/out) with the context's scheme
 * (Eq. 17-23).  Runge-Kutta: S_m = u^n + sum_{i<m} a^mi E^i; an implicit
 * stage solves N(u^m) = 0 by Newton and sets E^m = (u^m - S_m)/a^mm, an
 * explicit stage (a^mm = 0) sets E^m = dt M^-1 L(S_m); u^{n+1} = u^n +
 * sum b^i E^i.  BDF2: one solve with S = (4 u^n - u^{n-1})/3 and dt a =
 * 2 dt/3, where u^{n-1} is the incoming u of the previous call; the first
 * call after create or dgj_reset_history, and a call whose dt differs
 * (exactly) from the previous call's, is a backward-Euler step.  (Re)builds
 * the preconditioner at the incoming u when none is held, when it is
 * pc_freeze steps old, or when dt a^mm changed, and at a stage's S_m under
 * the pc_refresh_its rules (ERK2 builds none).  stats may be NULL (the
 * stats of a retried stage are the retry's).  On DGJ_ENOTCONV / DGJ_ENAN u
 * is left unchanged and stats tell where. */
int dgj_sdirk_step(dgj_ctx *ctx, double *u, double dt, dgj_step_stats *stats);

/* Forget the step history: BDF2's previous state and the stage increments
 * the Newton guesses extrapolate from.  For callers that change u between
 * steps (a restart, a new initial condition). */
int dgj_reset_history(dgj_ctx *ctx);

/* ---- Newton initial guess (not in the paper, which starts from S_m,
 * Eq. 21).  With inc_n = u^m - S_m the converged increment of stage m at
 * step n and i_k = inc_{n-k}: the extrapolated guess is S_m + i_1 after one
 * step and S_m + 2 i_1 - i_2 after two; the learned guess, after three,
 *   S_m + 2 i_1 - i_2 + c0 (i_1 - i_2) + c1 (i_1 - 2 i_2 + i_3),
 * c = (c0, c1) the mean over the elements of a per-element MLP's two
 * outputs (c = 0: the extrapolated guess; c = (0, 1): third-order
 * extrapolation).  The blend is global because ||N|| punishes corrections
 * that differ between elements or variables far more than it rewards their
 * fit.  Whichever candidate has the smallest ||N|| starts Newton, which then
 * stops at the same absolute tolerance alpha ||N(S_m)|| for all.
 * mode: 0 S_m (the paper), 1 extrapolated, 2 learned with the extrapolated
 * guess as fallback. */
int dgj_set_guess(dgj_ctx *ctx, int32_t mode);

/* Record, for every stage of each following dgj_sdirk_step, S_m and the
 * increment u^m - S_m into caller device buffers [stages][n_unknowns]
 * (training data).  NULL stops recording. */
int dgj_set_record(dgj_ctx *ctx, double *S_rec, double *inc_rec);

/* MLP of `hidden` units per layer, n_in = 2 nb, n_out = 2 (nb = (d+2)(P+1)^d):
 * z1 = x W1 + b1, h1 = tanh z1, z2 = h1 W2 + b2, h2 = tanh z2, y = h2 W3 + b3.
 * Parameters packed W1[n_in][H], b1[H], W2[H][H], b2[H], W3[H][n_out], b3[n_out]
 * (FP32 master copy, BF16 copy for the matrix-core products).  params_host:
 * host FP32 initial values (NULL: zeros).  For callers that train and use a
 * learned guess. */
int dgj_mlp_create(dgj_ctx *ctx, int32_t hidden, const float *params_host);
int dgj_mlp_sizes(const dgj_ctx *ctx, int64_t *n_params, int32_t *n_in, int32_t *n_out);
/* device FP32 parameter vectors of n_params values */
int dgj_mlp_get_params(dgj_ctx *ctx, float *out);
int dgj_mlp_set_params(dgj_ctx *ctx, const float *params);
/* Features X[e][2 nb] (FP32, device) of the learned guess from the three
 * previous increments i1, i2, i3 (FP64 states, device):
 * [(i1 - i2) / s_v, (i2 - i3) / s_v], s_v the RMS of i1 - i2 over the
 * context's elements per variable (1 where that is zero). */
int dgj_mlp_features(dgj_ctx *ctx, const double *i1, const double *i2, const double *i3, float *X);
/* Pooled forward pass: cbar[k] = mean over the rows of MLP(X)[r][k] (host,
 * n_out values; FP64 sums); keeps the activations for dgj_mlp_pool_backward. */
int dgj_mlp_pool(dgj_ctx *ctx, const float *X, int64_t rows, double *cbar);
/* Gradient of a loss L(cbar) of the last pooled forward pass with respect
 * to the parameters, given dL/dcbar (host, n_out values): into grad (device
 * FP32, n_params, may be NULL) and the context's gradient buffer. */
int dgj_mlp_pool_backward(dgj_ctx *ctx, const double *dLdc, float *grad);
/* Train on records written through dgj_set_record over n_steps >= 4
 * consecutive steps (S_rec, inc_rec: [n_steps][stages][n_unknowns]; S_rec
 * is not used by the features).  Each (step k >= 3, stage) pair is one
 * sample with loss ||F c - r||^2 / ||r||^2, r = inc_k - 2 i_1 + i_2 the
 * extrapolated guess's error and F c = c0 (i_1 - i_2) + c1 (i_1 - 2 i_2 + i_3)
 * the learned correction; `epochs` passes of Adam steps, one per sample.
 * *last_loss: mean loss of the last pass. */
int dgj_mlp_fit(dgj_ctx *ctx, const double *S_rec, const double *inc_rec, int32_t n_steps, int32_t epochs, double lr,
                double *last_loss);
/* Copy the stored stage increments of the three previous steps out
 * ([3][stages][n_unknowns]: i_1, i_2, i_3, stages of the context's scheme;
 * may be NULL) and/or in (may be NULL), to restart a run from a saved point. */
int dgj_guess_state(dgj_ctx *ctx, double *inc_out, const double *inc_in);
/* Y[rows][n_out] = MLP(X[rows][n_in]) */
int dgj_mlp_forward(dgj_ctx *ctx, const float *X, int64_t rows, float *Y);
/* gradient of mean((Y - T)^2) into grad (device FP32, may be NULL), loss to *loss (host, may be NULL) */
int dgj_mlp_grad(dgj_ctx *ctx, const float *X, const float *T, int64_t rows, float *grad, double *loss);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error */
int dgj_mlp_train_step(dgj_ctx *ctx, const float *X, const float *T, int64_t rows, double lr, double *loss);

/* ---- Batches of independent instances (periodic meshes of different
 * sizes, polynomial orders and gas parameters, one shared solver setting).
 * Instances of one (dim, P, nq) share every kernel launch; GMRES, Newton and
 * SDIRK run in lockstep with per-instance scalars and masks, each instance
 * going through exactly the operations of its single-instance run.  The
 * batch state is one device vector: instance i occupies
 * [offsets[i], offsets[i] + counts[i]) in the usual [element][variable][mode]
 * layout (instances of equal order are stored next to each other, so the
 * order in the vector can differ from the order of creation).  For callers that advance many
 * small problems at once. */
typedef struct dgj_batch dgj_batch;
int dgj_batch_create(int32_t n, const dgj_mesh *meshes, const dgj_phys *phys, const dgj_solver *solver,
                     void *hip_stream, dgj_batch **out);
/* The same call under the name the interface sketch of the batching form
 * uses. */
int dgj_create_batch(int32_t n, const dgj_mesh *meshes, const dgj_phys *phys, const dgj_solver *solver,
                     void *hip_stream, dgj_batch **out);
void dgj_batch_destroy(dgj_batch *batch);
const char *dgj_batch_last_error(const dgj_batch *batch);
/* on != 0 (default): each Krylov step of each order's instances (BRJ sweeps,
 * matvec, Gram-Schmidt) is captured once into a hipGraph on the batch's own
 * stream and replayed; 0: plain launches. */
int dgj_batch_set_graphs(dgj_batch *batch, int32_t on);
/* dgj_autotune for every order group of the batch at the batch state u
 * (layout of dgj_batch_sizes); drops captured graphs.  chosen: host
 * [n_groups][3] or NULL (at most one entry per distinct (dim, P, nq));
 * n_groups: host, set to the number of groups, or NULL. */
int dgj_batch_autotune(dgj_batch *batch, const double *u, int32_t reps, int32_t *chosen, int32_t *n_groups);
/* total unknowns; per instance offsets[n] and counts[n] (host, may be NULL) */
int dgj_batch_sizes(const dgj_batch *batch, int64_t *n_total, int64_t *offsets, int64_t *counts);
/* dgj_project_tgv for every instance (noise in the batch layout, may be NULL) */
int dgj_batch_project_tgv(dgj_batch *batch, const double *noise, double noise_amp, double *u);
/* R = M^-1 L(u) for every instance */
int dgj_batch_residual(dgj_batch *batch, const double *u, double *R);
/* One SDIRK step of every instance, dt (host [n]) per instance; optional
 * host outputs newton_its[n][4] and gmres_its[n][4] (total per stage).
 * Preconditioners are rebuilt at the incoming state every pc_freeze steps
 * or when an instance's dt changes (pc_refresh_its is not applied). */
int dgj_batch_sdirk_step(dgj_batch *batch, double *u, const double *dt, int32_t *newton_its, int32_t *gmres_its);

#ifdef __cplusplus
}
#endif
#endif
