/*
 * vip.h - C ABI of the MI355X (gfx950) library for the virtual interpolation
 * point (VIP) method of Park, Jo and Choe, "Virtual Interpolation Point Method
 * for Viscous Flows in Complex Geometries" (arXiv 1401.6513).
 *
 * The library builds moving-least-squares (MLS) shape functions on a node set
 * (Section 3 of the paper), assembles the VIP operators (Section 4) and
 * advances the incompressible Navier-Stokes equations by the fractional step of
 * Section 2 (eqs. 12-15), all on one GPU.
 *
 * Conventions for every entry point:
 *  - Return value: VIP_OK (0) or a negative VIP_E_* code.  No C++ exception
 *    crosses the ABI.  After an error, vip_last_error() describes it.
 *  - Host arrays ("host" below) are read during the call and copied; the
 *    caller keeps ownership.
 *  - Device arrays ("device" below) are caller-owned HIP device allocations of
 *    the stated length, FP64, in the caller's node order.  The library never
 *    frees them.  Work is enqueued on the context's stream; a call returns
 *    after its results are complete on that stream unless stated otherwise.
 *  - A context is bound to one device and one stream and is not thread-safe.
 */
#ifndef VIP_H_
#define VIP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
enum {
  VIP_OK = 0,
  VIP_E_INVALID = -1,       /* bad argument (sizes, NaN coordinates, unknown enum) */
  VIP_E_SINGULAR = -2,      /* an MLS moment matrix could not be factorised, or a
                               point kept fewer than min_neighbours neighbours
                               after support growth (index in vip_last_error) */
  VIP_E_NOT_CONVERGED = -3, /* Krylov solve hit its iteration limit; outputs are
                               still written and stats filled */
  VIP_E_HIP = -4,           /* a HIP runtime call failed */
  VIP_E_NOT_BUILT = -5,     /* vip_build_stencils has not succeeded on this context */
  VIP_E_NONFINITE = -6      /* NaN or Inf met in the state or in a solve */
};

/* ---- boundary kinds (one per boundary-table entry) ----------------------- */
enum {
  VIP_BC_DIRICHLET = 0, /* u = value[0], v = value[1]; dphi/dn = 0 */
  VIP_BC_SLIP = 1,      /* the component along the dominant axis of the normal is
                           held at its value, the other has zero normal
                           derivative; dphi/dn = 0 */
  VIP_BC_OUTLET = 2     /* traction free: du/dn = Re p n_x, dv/dn = Re p n_y with
                           p from the previous step; phi = 0 */
};

/* ---- options -------------------------------------------------------------- */
enum { VIP_W_CUBIC_SPLINE = 0, VIP_W_PAPER = 1 };  /* weight function Phi (Section 3) */
enum { VIP_I_MLS = 0, VIP_I_EXACT = 1 };            /* identity in eq. 12: D^[0,0] or I */
enum { VIP_P_FP64 = 0, VIP_P_MIXED = 1 };           /* pressure and predictor solves: FP64
                                                       Krylov, or FP32 inner Krylov in FP64
                                                       iterative refinement */
enum { VIP_K_AUTO = 0, VIP_K_PCG = 1, VIP_K_BICGSTAB = 2 };
/* Poisson start vector in vip_step: zero; the previous increment phi_n; phi_n + alpha e +
 * gamma (e - e_old) with e = phi_n - phi_(n-1) and e_old = phi_(n-1) - phi_(n-2), the linear
 * and quadratic extrapolations in time (EXTRAP; alpha = gamma = 1 is the quadratic one); or the
 * same plus beta c with c the learned network's correction (LEARNED).  The coefficients
 * minimise the FP64 residual ||b - L phi0||_2 over the directions available (e after two steps,
 * e - e_old after three), and the corrected vector replaces phi_n only if that lowers the
 * residual. */
enum { VIP_WS_ZERO = 0, VIP_WS_PREV = 1, VIP_WS_LEARNED = 2, VIP_WS_EXTRAP = 3 };
enum { VIP_PC_JACOBI = 0, VIP_PC_AMG = 1 };         /* Poisson preconditioner */

typedef struct {
  int weight;             /* VIP_W_*; default VIP_W_CUBIC_SPLINE */
  int identity;           /* VIP_I_*; default VIP_I_MLS */
  int precision;          /* VIP_P_*; default VIP_P_FP64 */
  int krylov;             /* VIP_K_*; AUTO: PCG if the pressure matrix is symmetric, else BiCGStab */
  int warmstart;          /* VIP_WS_*; default VIP_WS_ZERO */
  int min_neighbours;     /* support growth threshold; default 12 */
  double vip_offset;      /* VIP distance from the node, fraction of h; default 0.5 */
  double period[2];       /* periodic box lengths, 0 = not periodic (both or neither) */
  double poisson_tol;     /* ||b - L phi||_2 / ||b||_2 in FP64; default 1e-8 */
  double helmholtz_tol;   /* same measure for eq. 12; default 1e-12 */
  double inner_tol;       /* relative tolerance of each FP32 inner solve (MIXED: pressure and
                             predictor solves); default 1e-5 */
  int max_iters;          /* Krylov iteration limit per solve; default 200000 */
  int check_every;        /* iterations between host convergence checks; default 16 */
  int preconditioner;     /* VIP_PC_*; default VIP_PC_AMG: aggregation multigrid V-cycle
                             (2x2-cell aggregates, Galerkin coarse matrices, damped Jacobi
                             smoothing, 2 sweeps before and after on every level; dense
                             coarsest solve), built at the first solve */
  int learned_precond;    /* 1: with VIP_WS_LEARNED and VIP_P_MIXED on a non-singular lattice-based
                             pressure system, the learned network also preconditions every FP64
                             refinement pass: the pass adds alpha d + beta c, d the FP32 inner
                             correction of the pass residual r and c the network's correction of r,
                             (alpha, beta) minimising ||r - alpha L d - beta L c||_2 (a flexible
                             two-direction step, so a nonlinear preconditioner is allowed); when the
                             network's direction does not lower that residual below the best
                             multiple of d alone, the pass adds d as usual.  Default 0. */
} vip_options;

typedef struct {
  int poisson_iters;      /* Krylov iterations of the Poisson solve (inner total if MIXED) */
  int poisson_outer;      /* refinement passes (1 for FP64) */
  int helmholtz_iters;    /* iterations of the two predictor solves (the larger) */
  int krylov_used;        /* VIP_K_PCG or VIP_K_BICGSTAB */
  double poisson_residual;   /* final ||b - L phi||_2 / ||b||_2, FP64 */
  double helmholtz_residual; /* the larger of the two predictor residuals */
  double border_lambda;      /* multiplier of the bordered singular system, else 0 */
  int warm_start;            /* start vector actually used: VIP_WS_* */
  double warm_ratio;         /* VIP_WS_LEARNED, VIP_WS_EXTRAP: ||b - L phi0|| / ||b - L phi_n|| of
                                the corrected start vector (used if < 1), else 0 */
  double warm_alpha;         /* alpha of the used correction, else 0 */
  double warm_beta;          /* beta of the used correction (VIP_WS_LEARNED), else 0 */
  int poisson_fp64_fallback; /* 1: with VIP_P_MIXED an FP32 correction broke down or stopped
                                gaining (less than 2x on the FP64 residual), and the Poisson solve
                                finished with FP64 iterations from its FP64 iterate; else 0 */
  int learned_pc_passes;     /* learned_precond: refinement passes that took the network's
                                direction */
  double learned_pc_ratio;   /* learned_precond: product over the passes of the predicted residual
                                with the network's direction over that of the best multiple of d
                                alone (1 if never taken; < 1 is what the network gained) */
  double warm_gamma;         /* coefficient of the second difference e - e_old in the used start
                                vector (VIP_WS_EXTRAP, VIP_WS_LEARNED), else 0 */
} vip_step_stats;

/* Fill *opt with the defaults listed above. */
void vip_default_options(vip_options* opt);

/* Create a context on HIP device `device` using HIP stream `stream` (NULL =
 * the default stream; a torch stream handle may be passed).  *out receives
 * the context, owned by the caller until vip_destroy.  Read once here from the
 * environment (all results keep their bits either way): VIP_NO_CANON=1 sends every
 * row through the general sliced-ELL path; VIP_CNN_LAYERED=1 runs the learned start
 * vector's network layer by layer instead of in one fused launch; VIP_AMG_GAMMA,
 * VIP_AMG_NU, VIP_AMG_NU_COARSE override the multigrid over-correction and sweep
 * counts (these change results); VIP_MAX_GRID sets the block count of the reducing
 * vector kernels (default 2048, read once per process; it changes the order of the
 * partial sums and so the last bits); VIP_NO_DELTA=1 keeps the general rows on int32 columns
 * instead of int16 row-relative ones (same bits); VIP_NO_GRAPH=1 launches the multigrid
 * V-cycle's coarse levels one by one instead of replaying them as one captured HIP graph
 * (same bits; the graph is captured on a private stream and launched on `stream`, which may
 * be the null stream); VIP_DEBUG=1 prints solver progress to stderr. */
int vip_create(void** out, int device, void* stream);

/* Release every device allocation of the context and the context itself. */
int vip_destroy(void* ctx);

/* Text of the last error on this context (never NULL; empty if none). */
const char* vip_last_error(const void* ctx);

/*
 * Build the stencils and every operator for a node set (Sections 3 and 4).
 *
 *  nodes_xy   host, [n_nodes][2] FP64: node coordinates (the set Lambda).
 *  bnd_idx    host, [n_bnd] int64: node index of each boundary-table entry
 *             (distinct, in [0, n_nodes)).
 *  bnd_normal host, [n_bnd][2] FP64: outward unit normal of the flow domain.
 *  bnd_kind   host, [n_bnd] int32: VIP_BC_*.
 *  bnd_value  host, [n_bnd][2] FP64: prescribed velocity (read where held).
 *  basis_order  2 (the quadratic basis of Section 3; other values are rejected).
 *  support_radius  rho of Section 3 (absolute); grown by 1.25, at most twice,
 *             where fewer than min_neighbours nodes lie strictly inside.
 *  h          lattice spacing: VIPs sit at x_i +- vip_offset*h along the axes;
 *             Neumann rows use points at vip_offset*h and 2*vip_offset*h along
 *             the inward normal.
 *  opt        options (NULL = defaults).
 *
 * Errors: VIP_E_INVALID (n_nodes <= 0, n_bnd < 0, NaN coordinates, bad
 * indices or kinds, rho <= 0, h <= 0, basis_order != 2, a periodic box
 * shorter than twice the largest support); VIP_E_SINGULAR; VIP_E_HIP.
 * Rebuilding on the same context replaces the previous node set.
 */
int vip_build_stencils(void* ctx, const double* nodes_xy, int64_t n_nodes,
                       const int64_t* bnd_idx, const double* bnd_normal,
                       const int32_t* bnd_kind, const double* bnd_value, int64_t n_bnd,
                       int basis_order, double support_radius, double h,
                       const vip_options* opt);

/*
 * vip_build_stencils for node sets whose spacing varies from node to node (stepwise adaptive
 * distributions, Section 5.5), with a support radius that follows the local spacing: rho(xbar)
 * of Section 3.  h_node (host, [n_nodes] FP64, > 0) is each node's local spacing; an
 * evaluation point that belongs to node i (the node itself, its VIPs, or the inner points of
 * the Neumann row of boundary node i) gets the support radius support_radius * h_node[i] / h,
 * grown as in vip_build_stencils; node i's VIPs sit at vip_offset * h_node[i] and its Neumann
 * points at vip_offset * h_node[i] and twice that.  h is the reference spacing (the finest);
 * h_node[i] = h for every node gives vip_build_stencils' result.  Other arguments, errors and
 * ownership as vip_build_stencils; VIP_E_INVALID also for h_node NULL or an entry that is not
 * finite and positive.
 */
int vip_build_stencils_adaptive(void* ctx, const double* nodes_xy, int64_t n_nodes,
                                const int64_t* bnd_idx, const double* bnd_normal,
                                const int32_t* bnd_kind, const double* bnd_value, int64_t n_bnd,
                                int basis_order, double support_radius, double h,
                                const double* h_node, const vip_options* opt);

/* Replace the solver options of a built context (stencil-defining fields such
 * as weight, vip_offset, period and min_neighbours are ignored here). */
int vip_set_options(void* ctx, const vip_options* opt);

/*
 * One fractional step (eqs. 12-15): AB2 convection by VIP fluxes, the
 * Crank-Nicolson predictor with the boundary rows, the pressure Poisson
 * equation, the VIP-gradient projection at interior nodes and the pressure
 * update p = phi - dt/(2 Re) Delta phi.
 *
 *  u, v, p  device, [n_nodes] FP64, updated in place.
 *  dt, Re   time step and Reynolds number (> 0).  A change of dt or Re
 *           re-assembles the Helmholtz operators and restarts AB2 (the first
 *           step uses N^(n-1) = N^n).
 *  The predictor solve starts from 3 u*(n-1) - 3 u*(n-2) + u*(n-3) once three
 *  earlier steps of the same dt and Re have converged (2 u*(n-1) - u*(n-2) after
 *  two, u*(n-1) after one, else the right-hand side); the start does not change
 *  what it converges to.
 *  stats    host, may be NULL.
 * Returns with the step's statistics final and its last kernels (the projection) enqueued on
 * the context's stream: work the caller orders after it on that stream sees the new u, v, p;
 * elsewhere (the host, other streams) synchronize that stream first.
 * Errors: VIP_E_NOT_BUILT, VIP_E_INVALID, VIP_E_NOT_CONVERGED (state is still
 * advanced), VIP_E_NONFINITE, VIP_E_HIP.
 */
int vip_step(void* ctx, double* u, double* v, double* p, double dt, double Re,
             vip_step_stats* stats);

/* Forget the AB2 history, the previous pressure increment and the three previous
 * predictor solutions (the predictor solve then starts from its right-hand side). */
int vip_reset_history(void* ctx);

/*
 * Solve the pressure Poisson system of eq. 13 with the context's boundary
 * rows: interior rows Delta phi = rhs, Neumann rows, outlet rows phi = 0; for a
 * singular system (periodic, or no outlet) the bordered form
 * Delta phi + lambda = rhs, sum(phi) = 0.
 *
 *  rhs  device, [n_nodes] FP64 (boundary-row entries are the row right-hand sides).
 *  phi  device, [n_nodes] FP64: start vector on entry if use_x0 != 0, solution on exit
 *       (the last iterate after VIP_E_NOT_CONVERGED; unspecified after other errors).
 *  tol  relative FP64 residual target.
 *  stats host, may be NULL (poisson_* fields and border_lambda are filled).
 * As vip_step, returns with phi's last writes possibly still enqueued on the context's stream.
 */
int vip_poisson_solve(void* ctx, const double* rhs, double* phi, double tol, int use_x0,
                      vip_step_stats* stats);

/* ---- learned start vector of the pressure solve ------------------------------
 * Not part of the paper's method: a convolutional network on the lattice image
 * of the node set (pixel (i, j) <-> node at (xmin + i h, ymin + j h); nodes off
 * the lattice, such as curved-wall nodes, are left out) predicts the change of
 * the pressure increment phi from one step to the next.  Layers: four 3x3
 * convolutions 3 -> 32 -> 32 -> 32 -> 1 with zero padding, ReLU after the first
 * three; BF16 weights and activations, FP32 sums, FP32 master weights trained
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on a masked mean squared error.
 * The network corrects the extrapolated start vector phi_n + e, e = phi_n - phi_(n-1):
 * input channels r h^2 / s, b h^2 / rms(b h^2), lattice mask, where r = b - L (phi_n + e)
 * is the residual left by extrapolation and s = rms(r h^2) over lattice nodes; output y,
 * the correction c = s y / h^2 (training target (phi_(n+1) - phi_n - e) h^2 / s).  With
 * VIP_WS_LEARNED, vip_step starts the solve from phi_n + alpha e + beta c (alpha, beta
 * and the acceptance rule at VIP_WS_*); the Krylov solve to poisson_tol always decides
 * the result, so the network changes the iteration count, never the accuracy.
 *
 * Parameters are one flat FP64 host vector of vip_learn_n_params() values:
 * W1 [3][3][3][32], b1 [32], W2 [3][3][32][32], b2 [32], W3 [3][3][32][32],
 * b3 [32], W4 [3][3][32][1], b4 [1]; W[ky][kx][ci][co] multiplies input channel
 * ci at pixel (i + ky - 1, j + kx - 1) into output channel co at (i, j).
 * The network, its Adam moments and the captured snapshots belong to the
 * context and survive vip_build_stencils (snapshots are lattice images).
 */

/* Number of network parameters (19,681). */
int vip_learn_n_params(void);

/* He-uniform weights U(+-sqrt(6 / fan_in)) drawn with splitmix64 from `seed`,
 * zero biases; Adam moments cleared. */
int vip_learn_init(void* ctx, uint64_t seed);

/* Set (host, [n]) or read back the FP32 master parameters; n must equal
 * vip_learn_n_params() (VIP_E_INVALID otherwise; non-finite values rejected).
 * Setting clears the Adam moments.  Reading before any set: VIP_E_NOT_BUILT. */
int vip_learn_set_params(void* ctx, const double* theta, int64_t n);
int vip_learn_get_params(void* ctx, double* theta, int64_t n);

/*
 * Run the network on host images (checks and tools).
 *  x       host [batch][height][width][3] input channels (rounded to BF16).
 *  target  host [batch][height][width] (may be NULL if loss, grad are NULL and lr <= 0).
 *  mask    host [batch][height][width] loss weights (same condition).
 *  y       host [batch][height][width] output, may be NULL.
 *  loss    host scalar, may be NULL: sum(mask (y - target)^2) / sum(mask).
 *  grad    host [vip_learn_n_params()] gradient of loss, may be NULL.
 *  lr      > 0: also take one Adam step with that gradient (learning rate lr).
 * Errors: VIP_E_NOT_BUILT (no parameters), VIP_E_INVALID (sizes <= 0 or more
 * than 2^28 pixels, NULL x).
 */
int vip_learn_eval(void* ctx, const double* x, const double* target, const double* mask, int batch,
                   int height, int width, double* y, double* loss, double* grad, double lr);

/*
 * Run the network on host images with the single fused launch that vip_step uses for the
 * learned start vector (all four layers in one pass down strips of 58 output columns, the
 * activations in LDS rings of two rows per layer), rather than the layer-by-layer training
 * pass of vip_learn_eval.  Same arithmetic as vip_learn_eval's forward pass (the same bits),
 * without loss or gradient.  The launch is timed as which = 1 of vip_kernel_timing.
 *  x  host [batch][height][width][3] input channels (rounded to BF16).
 *  y  host [batch][height][width] output.
 * Errors: VIP_E_NOT_BUILT (no parameters), VIP_E_INVALID (sizes <= 0, batch > 65535, more
 * than 2^28 pixels, more than 65535 strips of rows (height above about 10.4 million), NULL x
 * or y).
 */
int vip_learn_infer(void* ctx, const double* x, int batch, int height, int width, double* y);

/* Training data: while fewer than max_snapshots are held, each vip_step that
 * knows the last change of the increment stores one snapshot (input image and
 * target).  0 stops capturing.  The node set must be
 * lattice based (VIP_E_INVALID from vip_step otherwise). */
int vip_learn_capture(void* ctx, int max_snapshots);
int vip_learn_snapshot_count(void* ctx, int* count);
int vip_learn_clear(void* ctx);   /* drop every snapshot */

/* `iters` Adam steps on batches of `batch` random crop x crop windows of the
 * snapshots (splitmix64 from seed and the step count; loss mask = lattice
 * pixels at least 4 pixels inside the crop); *last_loss (may be NULL) gets
 * the last batch loss.  Errors: VIP_E_NOT_BUILT, VIP_E_INVALID (no snapshots,
 * iters <= 0, batch outside [1, 1024], crop outside [12, 1024], lr <= 0),
 * VIP_E_NONFINITE (loss became NaN or Inf). */
int vip_learn_train(void* ctx, int iters, int batch, int crop, double lr, uint64_t seed,
                    double* last_loss);

/* ---- operator access (parity checks and tools) ---------------------------- */
enum {
  VIP_OP_IDENTITY = 0,  /* D^[0,0] at the nodes (N rows) */
  VIP_OP_LAPLACIAN = 1, /* D^[2,0] + D^[0,2] at the nodes (N rows) */
  VIP_OP_VIP_E = 2,     /* Psi^[0,0] at the east VIP of each interior node (N rows) */
  VIP_OP_VIP_W = 3,
  VIP_OP_VIP_N = 4,
  VIP_OP_VIP_S = 5,
  VIP_OP_NORMAL1 = 6,   /* Psi^[0,0] at x_b - d n_b, one row per boundary entry */
  VIP_OP_NORMAL2 = 7,   /* Psi^[0,0] at x_b - 2 d n_b */
  VIP_OP_POISSON = 8,   /* pressure matrix with boundary rows (N rows, no border) */
  VIP_OP_HELM_U = 9,    /* predictor matrix of u (needs one vip_step or vip_assemble) */
  VIP_OP_HELM_V = 10,
  VIP_OP_POISSON32 = 11 /* FP32 copy of VIP_OP_POISSON (values returned widened) */
};

/* Rows, the largest row length and the number of stored entries (without
 * slice padding) of operator `which`; any output pointer may be NULL. */
int vip_operator_shape(void* ctx, int which, int64_t* n_rows, int64_t* max_width, int64_t* nnz);

/* Copy operator `which` to host arrays [n_rows][max_width]: cols (int32, -1 in
 * padding) and vals (FP64, 0 in padding). */
int vip_get_operator(void* ctx, int which, int32_t* cols, double* vals);

/* y = A x for operator `which` with N rows over N columns; device x, y [N]. */
int vip_apply(void* ctx, int which, const double* x, double* y);

/* Assemble the Helmholtz operators for (dt, Re) without stepping. */
int vip_assemble(void* ctx, double dt, double Re);

/* Geometry of the build, host outputs: vip_xy [n_nodes][4][2] (VIP coordinates
 * e, w, n, s; zeros on boundary rows), d_ew and d_ns [n_nodes] (VIP spacings,
 * 1 on boundary rows), rho_node [n_nodes] (support radius used at each node).
 * Any pointer may be NULL. */
int vip_get_geometry(void* ctx, double* vip_xy, double* d_ew, double* d_ns, double* rho_node);

/* VIP convection flux (Section 4.1 item 1) of device u, v into device nx, ny
 * [n_nodes] (zero on boundary rows). */
int vip_convection(void* ctx, const double* u, const double* v, double* nx, double* ny);

/* VIP divergence (Section 4.1 item 2) of device u, v into device div [n_nodes]
 * (zero on boundary rows). */
int vip_divergence(void* ctx, const double* u, const double* v, double* div);

/* VIP gradient (Section 4.1 item 3) of device f into device gx, gy [n_nodes]
 * (zero on boundary rows). */
int vip_gradient(void* ctx, const double* f, double* gx, double* gy);

/* ---- body forces (Section 5.4: drag and lift coefficients, Strouhal number) ---------------
 *
 * Force on a body from the fluid, F = -sum over its surface of t dS with the traction of
 * Section 5.4, t = -p n + (1/Re) du/dn, n the outward normal of the flow domain (the boundary
 * table's normal, pointing into the body); du/dn is the normal derivative of the boundary
 * rows, (3 u_b - 4 u(x_b - d n) + u(x_b - 2 d n)) / (2 d) with
 * d = vip_offset h and the values at the inner points interpolated by Psi^[0,0] (exact for
 * quadratics).  dS is the trapezoid weight of the closed chain of surface nodes, half the
 * chords to the previous and the next node.  For the cylinder cases (D = 1, U = 1) the drag
 * and lift coefficients are C_D = 2 F_x and C_L = 2 F_y.
 *
 *  u, v, p   device [n_nodes] FP64 state (p as vip_step leaves it).
 *  Re        Reynolds number (> 0; the viscosity is 1/Re).
 *  surf_idx  host [n_surf] int64: node indices of the body surface in order around it
 *            (on adaptive node sets d follows each surface node's local spacing)
 *            (entry k adjacent to k-1 and k+1, the last to the first); each must be a
 *            boundary node.  n_surf >= 3.
 *  force     host [2]: F_x, F_y.
 * The work arrays (the surface list and one traction pair per node) belong to the context
 * and grow as needed.  Errors: VIP_E_NOT_BUILT, VIP_E_INVALID (NULL arguments, n_surf < 3,
 * Re <= 0, an index out of range or not a boundary node), VIP_E_HIP.
 */
int vip_forces(void* ctx, const double* u, const double* v, const double* p, double Re,
               const int64_t* surf_idx, int64_t n_surf, double* force);

/* vip_forces for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and
 * result, with the surface list and the per-node traction terms in a fixed device scratch
 * array of 1 MiB per GPU that the library holds until the process ends, instead of the
 * context's work arrays.  It calls no hipMalloc or hipFree.  Every kernel writes the scratch
 * entries it later reads, so nothing has to start at zero; calls that overlap on one GPU
 * (several streams or contexts at once) share that array and race.  n_surf is limited to
 * what fits (43680 surface nodes); larger n_surf returns VIP_E_INVALID with the limit in
 * vip_last_error.  Other errors as vip_forces. */
int vip_forces_noalloc(void* ctx, const double* u, const double* v, const double* p, double Re,
                       const int64_t* surf_idx, int64_t n_surf, double* force);

/* Dominant frequency of a real signal sampled at spacing dt (host [n], n >= 8): the maximum
 * of the periodogram of the mean-removed, Hann-windowed signal, located on the DFT bins
 * k / (n dt), k >= 1, then refined between the neighbouring bins by golden-section search on
 * the continuous spectrum.  *freq gets the frequency; *amp (may be NULL) the amplitude of a
 * sinusoid with that peak.  For the lift history of a cylinder (D = 1, U = 1) the Strouhal
 * number is the frequency.  Host computation, no context.  Errors: VIP_E_INVALID (NULL
 * arguments, n < 8, dt <= 0, non-finite samples). */
int vip_spectral_peak(const double* signal, int64_t n, double dt, double* freq, double* amp);

/* Rows of the system layout that are translation-invariant lattice-interior copies of one
 * reference row (same lattice offsets, bitwise equal values), per value set (host counts[7]):
 * [0] FP64 pressure matrix, [1] predictor matrix of u, [2] of v, [3] nodes whose rows of the
 * four VIP operators, D^[0,0] and the Laplacian are all canonical (the per-step products of
 * eqs. 12-15 and the convection, divergence and gradient entry points), [4] FP32 pressure
 * matrix, [5] FP32 predictor matrix of u, [6] of v (the FP32 sets with their row sums);
 * described[7]: rows of 64-row slices whose rows are all canonical on consecutive pixels of
 * one lattice row (their kernels read one descriptor per slice instead of per-row data);
 * *taps = entries of the reference row.  Products over these rows skip the column and value
 * streams and give the same bits.  All counts are 0 when VIP_NO_CANON=1 was set at
 * vip_create, or for node sets that are not lattice based.  Host outputs, may be NULL. */
int vip_canonical_rows(void* ctx, int64_t* counts, int64_t* described, int* taps);

/* Column stream of the general (non-canonical) rows.  Where every stored column of a 64-row
 * slice lies within +-32767 of its row, the pressure and predictor matrices also hold the
 * slice's columns as int16 row-relative offsets, and the solve-phase kernels read those (2 bytes
 * per entry instead of 4; the results keep their bits); other slices (rows next to far-numbered
 * nodes, such as body-surface nodes listed last) read the int32 columns.  VIP_NO_DELTA=1 at
 * vip_create keeps every row on int32.  *sys_entries = stored entries of the system layout,
 * *sys_entries_int16 = those in int16 slices, *amg_levels = coarse multigrid levels built so far
 * (the hierarchy is built at the first Poisson solve), *amg_levels_delta = those with int16
 * slices.  Host outputs, may be NULL.  Errors: VIP_E_NOT_BUILT. */
int vip_column_bytes(void* ctx, int64_t* sys_entries, int64_t* sys_entries_int16, int* amg_levels,
                     int* amg_levels_delta);

/* Average duration (ms) of a kernel over its launches since the last reset, measured with
 * HIP events on the context stream while timing is enabled; *count receives the number of
 * timed launches.  which = 0: the pressure-solve SpMV (the first SpMV of each Krylov
 * iteration; launches after the solve stopped on the device are not counted); which = 1:
 * the learned start vector's inference (the fused 4-layer launch, also that of
 * vip_learn_infer, or each 32 -> 32 layer when VIP_CNN_LAYERED=1 was set at vip_create); which = 2: the predictor's two-system SpMV
 * (k_bicg_v); 3: the predictor's t = A s launch with s formed inside (one per system: k_bicg_ts,
 * or k_bicg_t); 4: the predictor's two-system update pass (on lattice tiles k_bicg_e, which
 * applies the last iteration's x and r update and forms the new p; otherwise k_bicg_x;
 * VIP_NO_FUSE=1 at vip_create keeps the separate passes); 5: the post-smoothing sweeps of
 * the finest FP32 multigrid level (k_sweep); 6: the predictor right-hand side
 * (k_predictor_rhs, VIP convection and AB2).  Launches after a solve stopped on the device
 * (they return at once) are not counted.  enable = 0
 * stops timing; reset = 1 clears it.  Errors: VIP_E_INVALID (unknown which). */
int vip_kernel_timing(void* ctx, int which, int enable, int reset, double* avg_ms, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* VIP_H_ */
