/*
 * tmop.h -- C ABI of the MI355X (gfx950) implementation of the data-parallel
 * hot path of high-order TMOP mesh optimization:
 *
 *   V. Dobrev, P. Knupp, Tz. Kolev, K. Mittal, V. Tomov, "The Target-Matrix
 *   Optimization Paradigm for High-Order Meshes", arXiv:1807.09807.
 *
 * The library evaluates the variational objective (Section 2.3, eq. 2.4)
 *
 *   F(x) = sum_E sum_q  w_q det(W_q) mu(T_q),   T = A W^{-1},
 *
 * where A is the Jacobian of the element map of the high-order position
 * field x (Section 2.1, eqs. 2.1-2.2), together with its gradient and its
 * Hessian action (Section 3.4), and runs the Newton method of Section 3.4
 * with the positivity and 1.2-growth line search.
 *
 * Conventions shared by every call:
 *  - Positions, gradients and directions are DEVICE arrays of doubles in
 *    component-major layout: x[c * n_node + I], c < dim.  They are owned by
 *    the caller; outputs never alias inputs.
 *  - A `stream` argument is a hipStream_t (NULL = the null stream).  Calls
 *    marked "async" only enqueue work; calls marked "syncs" wait for the
 *    stream before returning.
 *  - Every call returns a status: 0 = success, > 0 = warning (outputs are
 *    valid), < 0 = error (outputs untouched).  No C++ exception crosses
 *    this interface.  A context is not thread-safe: calls on one context
 *    must not overlap in time.
 *  - Reference element [0,1]^dim; the nodal basis on each element is the
 *    tensor product of Lagrange polynomials at the order-p Gauss-Lobatto-
 *    Legendre points, local node index i = i0 + (p+1)*(i1 + (p+1)*i2)
 *    (first reference coordinate fastest).
 */
#ifndef TMOP_H
#define TMOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmop_ctx tmop_ctx;   /* opaque, owned by the library */

/* Status codes. */
enum {
  TMOP_OK = 0,
  TMOP_W_INVERTED = 1,     /* det A <= 0 at some quadrature point: outside the
                              domain of the barrier metrics (Section 3.2) */
  TMOP_W_MAXIT = 2,        /* Newton stopped after max_it iterations */
  TMOP_W_LSFAIL = 3,       /* no admissible step length was found: the
                              termination rule of Section 3.4 */
  TMOP_E_ARG = -1,         /* invalid argument */
  TMOP_E_TARGET = -2,      /* a target matrix has det W <= 0 (Section 3.1) */
  TMOP_E_NOMEM = -3,       /* device or host allocation failed */
  TMOP_E_HIP = -4,         /* a HIP runtime call failed */
  TMOP_E_UNSUPPORTED = -5, /* valid, but no kernel is built for this (dim, p, Q) */
  TMOP_E_SCRATCH = -6      /* tmop_energy_noalloc: the problem needs more
                              energy partials than its fixed scratch holds */
};

/* Quality metrics mu(T), tau = det T, |.| the Frobenius norm (Section 3.2). */
enum {
  TMOP_MU1 = 1,       /* 2D, no barrier: |T|^2                    (Table 3.1) */
  TMOP_MU2 = 2,       /* 2D shape:      |T|^2 / (2 tau) - 1       (Table 3.1) */
  TMOP_MU7 = 7,       /* shape+size, 2D and 3D: |T - T^{-t}|^2    (Section 3.2) */
  TMOP_MU9 = 9,       /* 2D shape+size: tau |T - T^{-t}|^2        (Table 3.1) */
  TMOP_MU14 = 14,     /* 2D shape+size+alignment: |T - I|^2       (Section 3.2) */
  TMOP_MU77 = 77,     /* 2D size:       (tau - 1/tau)^2 / 2       (Table 3.1) */
  TMOP_MU98 = 98,     /* 2D shape+size+alignment: |T - I|^2 / tau (Section 4.3) */
  TMOP_MU302 = 302,   /* 3D shape:      |T|^2 |T^{-1}|^2 / 9 - 1 */
  TMOP_MU303 = 303    /* 3D shape:      |T|^2 / (3 tau^{2/3}) - 1 (Table 3.1) */
};

/* Quadrature rules on [0,1] (Section 3.3), n1d points per direction. */
enum { TMOP_GAUSS_LEGENDRE = 0, TMOP_GAUSS_LOBATTO = 1 };

/* Arithmetic of the element kernels.  TMOP_MIXED_FP32 runs the basis
 * contractions and the metric derivatives in FP32 with FP32 accumulation;
 * det A, the positivity test and the sum of F stay FP64.  Both take and
 * return FP64 arrays. */
enum { TMOP_FP64 = 0, TMOP_MIXED_FP32 = 1 };

/* Inner linear solver of the Newton step (Section 3.4).  The Hessian is
 * indefinite away from the optimum (barrier metrics are not convex).
 *  TMOP_INNER_SHIFTED_CG (default): conjugate gradients on H + tau I, the
 *    added multiple of the identity of Nocedal and Wright (Numerical
 *    Optimization, 2nd ed., Algorithm 3.3) with a CG run as the test of
 *    positive definiteness: tau_0 = 0 if the free diagonal of H is
 *    positive, else beta - min diag; while CG meets curvature
 *    p.(H + tau I)p <= 0, tau <- max(2 tau, beta) and CG restarts;
 *    beta = shift_beta * mean |diag H| over the free DOFs.  The direction
 *    solves a positive definite system, so it always descends.
 *  TMOP_INNER_CG: Steihaug's truncated CG: at non-positive curvature it
 *    returns -M^{-1} g at the first step, else the current iterate.
 *  TMOP_INNER_MINRES: MINRES, the solver of the paper's results (Section
 *    5), which accepts indefinite systems.
 * The scalar recurrences of all three run on the device; the host reads
 * their state back after inner iterations 1, 2, 4, 8, 16, 24, ... only. */
enum { TMOP_INNER_CG = 0, TMOP_INNER_MINRES = 1, TMOP_INNER_SHIFTED_CG = 2 };

/* Preconditioner of the inner solver: none, or Jacobi, M = |diag H| on the
 * free DOFs, from tmop_hessian_diagonal at the current iterate. */
enum { TMOP_PREC_NONE = 0, TMOP_PREC_JACOBI = 1 };

/* Target matrices W (Section 3.1: W may be chosen at every quadrature
 * point; det W > 0). */
enum {
  TMOP_TGT_CONST = 0,      /* one dim x dim matrix for every point */
  TMOP_TGT_ISO_PER_QP = 1, /* W_q = s_q I, one size s_q > 0 per quadrature
                              point: the targets W_2 scaled by a
                              space-dependent factor and W_3 of Section 3.1 */
  TMOP_TGT_PER_ELEM = 2,   /* one general dim x dim matrix per element */
  TMOP_TGT_PER_QP = 3      /* one general dim x dim matrix per quadrature
                              point */
};

typedef struct {
  int32_t dim;                /* 2 (quadrilaterals) or 3 (hexahedra) */
  int32_t order;              /* polynomial order p >= 1 of the position field */
  int64_t n_elem;             /* number of elements, >= 1 */
  int64_t n_node;             /* number of nodes (DOFs per component), >= 1 */
  const int32_t *elem_node;   /* HOST [n_elem][(p+1)^dim] global node ids in
                                 [0, n_node), local order as above */
  const uint8_t *fixed;       /* HOST [dim][n_node], 1 = Dirichlet DOF held at
                                 its input value by the Newton solver; NULL =
                                 no fixed DOF.  Energy, gradient and Hessian
                                 action ignore it. */
} tmop_mesh;

typedef struct {
  int32_t kind;               /* TMOP_GAUSS_LEGENDRE or TMOP_GAUSS_LOBATTO */
  int32_t n1d;                /* points per direction; must be >= p + 1, the
                                 minimum of Section 3.3 */
} tmop_quadrature;

typedef struct {
  int32_t kind;               /* TMOP_TGT_CONST, TMOP_TGT_ISO_PER_QP,
                                 TMOP_TGT_PER_ELEM or TMOP_TGT_PER_QP */
  const double *W;            /* HOST.  TMOP_TGT_CONST: row-major dim x dim,
                                 det W > 0.  TMOP_TGT_ISO_PER_QP: the sizes
                                 [n_elem][n1d^dim], all > 0, point index
                                 q0 + n1d q1 (+ n1d^2 q2) (first reference
                                 coordinate fastest).  TMOP_TGT_PER_ELEM:
                                 [n_elem][dim][dim] row-major matrices.
                                 TMOP_TGT_PER_QP: [n_elem][n1d^dim][dim][dim]
                                 in the point order above.  Every matrix
                                 finite with det W > 0, else TMOP_E_TARGET.
                                 The device keeps W^{-1} and det W of each
                                 (d^2 + 1 doubles per element or per point,
                                 twice: element and colour order) */
} tmop_target;

typedef struct {
  double rtol;                /* stop when |g| <= max(rtol |g0|, atol); the paper
                                 uses 1e-12 (Section 5) */
  double atol;
  int32_t max_it;             /* Newton iterations */
  double cg_rtol;             /* inner truncated-CG tolerance relative to |g| */
  int32_t cg_max_it;
  double ls_shrink;           /* alpha <- ls_shrink * alpha, starting at 1 */
  int32_t ls_max;             /* step lengths tried per iteration */
  double f_growth;            /* accept only if F(x+) < f_growth F(x)  (1.2) */
  double g_growth;            /* and |g(x+)| < g_growth |g(x)|          (1.2) */
  double *hist_F;             /* optional HOST [max_it + 1]: F after each
                                 iteration (entry 0 = initial); NULL = off */
  double *hist_gnorm;         /* optional HOST [max_it + 1]: |g| likewise */
  int32_t *hist_cg;           /* optional HOST [max_it + 1]: CG iterations */
  double ftarget;             /* also stop (TMOP_OK) once F <= ftarget; default
                                 -HUGE_VAL = off */
  int32_t cg_forcing;         /* 0: inner tolerance cg_rtol.  1: inexact Newton,
                                 tolerance max(cg_rtol, min(0.5,
                                 sqrt(|g|/|g0|))) */
  double *hist_time;          /* optional HOST [max_it + 1]: seconds since the
                                 call started, at each accepted iterate */
  int32_t inner;              /* TMOP_INNER_SHIFTED_CG (default), TMOP_INNER_CG
                                 or TMOP_INNER_MINRES; MINRES stops when its
                                 residual estimate (the M^{-1} norm with a
                                 preconditioner) falls to the inner
                                 tolerance times its initial value */
  int32_t precond;            /* TMOP_PREC_NONE (default) or TMOP_PREC_JACOBI */
  double shift_beta;          /* TMOP_INNER_SHIFTED_CG: the floor of tau
                                 relative to the mean |diag H|; default 1e-3,
                                 must be > 0 */
} tmop_newton_opts;

typedef struct {
  int32_t iters;              /* accepted Newton steps */
  int32_t cg_iters;           /* total inner iterations (Hessian actions), CG
                                 or MINRES */
  int32_t ls_shrinks;         /* rejected step lengths */
  int32_t neg_curv;           /* truncated CG: inner solves ended by
                                 non-positive curvature; shifted CG: CG
                                 restarts with a larger shift */
  double F0, F;               /* objective at the start and at the end */
  double gnorm0, gnorm;       /* |g| over the free DOFs, start and end */
  double min_detA;            /* smallest det A at the end */
} tmop_newton_report;

/* Fills `opts` with the defaults: rtol 1e-12, atol 0, max_it 50, cg_rtol
 * 1e-8, cg_max_it 1000, ls_shrink 0.5, ls_max 30, growth factors 1.2, no
 * history, shifted CG (shift_beta 1e-3) without preconditioner. */
void tmop_newton_default_opts(tmop_newton_opts *opts);

/* Builds a context on the current HIP device for the objective of eq. 2.4
 * on the given mesh, quadrature (Section 3.3), target (Section 3.1) and
 * metric (Section 3.2), computing in `precision`.  Host arrays are copied;
 * the caller may free them on return.  Arguments are validated before any
 * device work: TMOP_E_ARG for a bad dimension, order, size, node id,
 * quadrature (n1d < p + 1) or metric/dimension pair; TMOP_E_TARGET when
 * det W <= 0; TMOP_E_UNSUPPORTED when no kernel is built for (dim, p, n1d).
 * On success *out owns all device memory of the context. */
int tmop_setup(const tmop_mesh *mesh, const tmop_quadrature *quad,
               const tmop_target *target, int32_t metric, int32_t precision,
               tmop_ctx **out);

/* F(x) of eq. 2.4 and the smallest det A over all quadrature points (the
 * positivity test of Section 3.4).  x: device [dim][n_node].  F and
 * min_detA: host pointers.  Returns TMOP_W_INVERTED (with both values
 * written) when min_detA <= 0.  Deterministic.  Syncs `stream`. */
int tmop_energy(tmop_ctx *ctx, const double *x, double *F, double *min_detA,
                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): F and
 * min det A exactly as tmop_energy (same kernels, same reduction order, so
 * bitwise the same values), with the energy partials, the final reduction
 * and its result in a fixed file-scope device array of the library instead
 * of the context's buffers.  The call allocates nothing (no hipMalloc,
 * hipFree, event or library allocation); the per-launch timing of
 * tmop_timing_enable does not cover it.  Limit: at most 65,536 workgroups
 * of partials summed over the objective's terms (1 MiB + 4 KiB of scratch
 * per GPU, held until the process ends); the 64^3 Q2 hexahedral mesh with
 * its single term needs exactly 65,536.  Larger problems return
 * TMOP_E_SCRATCH before any device work.  The context's device must be
 * current (else TMOP_E_ARG).  Every call on one GPU shares that GPU's
 * array and leaves the last call's contents there: calls that overlap in
 * time on one GPU (other streams, threads or contexts) race and must be
 * serialized by the caller.  Nothing in the array needs to start at zero.
 * Syncs `stream` (the result is read back to the host). */
int tmop_energy_noalloc(tmop_ctx *ctx, const double *x, double *F, double *min_detA,
                        void *stream);

/* g = dF/dx (Section 3.4) over all DOFs, fixed ones included.  x, g: device
 * [dim][n_node]; g is overwritten.  Deterministic.  Async. */
int tmop_gradient(tmop_ctx *ctx, const double *x, double *g, void *stream);

/* g = s * dF/dx, where s is the DEVICE scalar *scale (NULL: s = 1), folded
 * into the quadrature weights of the gradient kernel: the chain rule of a
 * reverse-mode caller (upstream gradient times dF/dx, Section 3.4) without
 * a host round trip.  Otherwise as tmop_gradient.  Async. */
int tmop_gradient_scaled(tmop_ctx *ctx, const double *x, const double *scale, double *g,
                         void *stream);

/* Hv = (d^2F/dx^2) v, the Hessian of Section 3.4 applied to v, over all
 * DOFs.  x, v, Hv: device [dim][n_node]; Hv is overwritten.
 * Deterministic.  Async. */
int tmop_hessian_apply(tmop_ctx *ctx, const double *x, const double *v,
                       double *Hv, void *stream);

/* The sizes of the target W_3 = (det A(x0))^(1/dim) I of Section 3.1 at
 * every quadrature point of the mesh x0: sizes[e][q] = (det A)^(1/dim)
 * (same layout as the TMOP_TGT_ISO_PER_QP sizes; the real root, so NaN in
 * 2D and negative in 3D where det A < 0).  Works on any context.  x0:
 * device [dim][n_node]; sizes: device [n_elem][n1d^dim], caller-owned.
 * Returns TMOP_W_INVERTED when det A <= 0 at some point.  Syncs. */
int tmop_target_sizes_w3(tmop_ctx *ctx, const double *x0, double *sizes, void *stream);

/* Replaces the per-point target sizes of a TMOP_TGT_ISO_PER_QP context by
 * the device array sizes [n_elem][n1d^dim] (copied).  TMOP_E_ARG for other
 * contexts; TMOP_E_TARGET (context unchanged) unless every size is finite
 * and > 0 (Section 3.1).  Syncs. */
int tmop_set_target_sizes(tmop_ctx *ctx, const double *sizes, void *stream);

/* diag = the diagonal of d^2F/dx^2 (Section 3.4) over all DOFs: entry
 * (c, I) is the Hessian action on the unit vector of DOF (c, I), read at
 * (c, I), i.e. sum over the elements E holding I of
 * sum_q w_q det W  dT : mu''(T)[dT],  dT = e_c (grad w_i)^T W^{-1}.  The
 * Jacobi preconditioner of tmop_newton_solve.  x, diag: device
 * [dim][n_node]; diag is overwritten, not aliasing x.  Deterministic.
 * Async. */
int tmop_hessian_diagonal(tmop_ctx *ctx, const double *x, double *diag, void *stream);

/* How the gradient, the energy + gradient and the Hessian action add the
 * element contributions to shared nodes (Section 3.4 sums them over the
 * elements holding each node):
 *  TMOP_SCATTER_COLOURS (the default of 3D meshes with colours of more
 *    than 49,152 elements on average, 131,072 in the mixed path): one launch
 *    per element colour; the
 *    elements of a colour share no node, each adds to its nodes in place.
 *  TMOP_SCATTER_TILES (2D only, on request): one launch over every
 *    element in tiles of neighbouring elements; each workgroup accumulates
 *    its tile's nodes on chip, adding its elements in rounds of elements
 *    that share no node, and writes the nodes only its tile holds; a second
 *    pass adds the tiles' partial sums at nodes shared by several tiles.
 *    Selecting it the first time builds the tiles on the host from a
 *    device-to-host copy of the connectivity (device memory: about 2 bytes
 *    per element node, 8 per tile node and 24 per node on a tile border);
 *    a mesh beyond the tile limits is refused.  FP64
 *    gradient tiles stage one vector component at a time when the tiles
 *    would not otherwise all fit on the device at once; the environment
 *    variable TMOP_TILE_SPLIT=0 or =1, read when the tiles are built,
 *    forces that choice off or on (same results bit for bit).
 *  TMOP_SCATTER_ELEMENTS (the default of 2D meshes and of 3D meshes with
 *    colours of at most 49,152 elements on average, 131,072 in the mixed
 *    path): one launch over every
 *    element, each element writing its contributions to the entries of its
 *    nodes in an element vector (dim x (p+1)^dim values per element, FP64
 *    or, in the mixed path, FP32; each node's entries contiguous, in
 *    ascending element order), then a pass that sums each node's entries in
 *    that order, in FP64.  Selecting it on a context that did not start
 *    with it builds the entry map on the host (a device-to-host copy of the
 *    connectivity; 4 bytes per element node and per node) and allocates the
 *    vector; it syncs the device.
 * All are deterministic (fixed summation orders, which differ between
 * them, so results agree to rounding).  The other calls are not affected. */
enum { TMOP_SCATTER_COLOURS = 0, TMOP_SCATTER_TILES = 1, TMOP_SCATTER_ELEMENTS = 2 };

/* Selects the scatter mode of ctx.  TMOP_E_ARG for an unknown mode,
 * TMOP_E_UNSUPPORTED (mode unchanged) for tiles on a 3D context or a 2D
 * mesh beyond the tile limits, and for the element vector past 2^31
 * entries; TMOP_E_NOMEM if a buffer cannot be allocated.  Building the
 * tiles or the element vector on first selection syncs the device. */
int tmop_set_scatter(tmop_ctx *ctx, int32_t mode);

/* The scatter mode in effect on ctx (the mesh's default until
 * tmop_set_scatter changes it).  TMOP_E_ARG for a null argument. */
int tmop_get_scatter(const tmop_ctx *ctx, int32_t *mode);

/* ------------------------------------------------------------------------
 * Section 4 objectives.  Each adds a term to the F of every call above
 * (energy, gradient, Hessian action, diagonal, energy + gradient, Newton);
 * they combine.  The terms run after the primary metric term and add to
 * its outputs, so the calls keep their layouts and their determinism.
 *
 * First restricted node movement algorithm (Section 4.3.1, eq. 4.2): adds
 *   sum_E sum_q w_q det W delta |x(q) - x_init(q)|^2
 * (the displacement integrated over the target elements; x(q) is the
 * finite element field of eq. 2.1 at the point, det W the primary
 * target's, per point for TMOP_TGT_ISO_PER_QP).  Its gradient is
 * 2 delta M (x - x_init) and its Hessian 2 delta M per component, with M the
 * target-weighted mass matrix.  x_init: device [dim][n_node], copied
 * (caller keeps ownership).  delta = 0 removes the term (x_init may then be
 * NULL).  TMOP_E_ARG unless delta is finite and >= 0 (context unchanged).
 * Syncs. */
int tmop_set_restriction(tmop_ctx *ctx, double delta, const double *x_init, void *stream);

/* Composite metric of eq. 4.1 with two terms (Section 5.2.4 form):
 *   F = sum_E sum_q w_q [eta1 det W mu(A W^-1) + omega_q mu2(A W2^-1)],
 *   omega_q = eta2 * eta2_q[e][q] * det W2,
 * each term integrated over its own target element.  W2: host, row-major
 * dim x dim, det W2 > 0 (else TMOP_E_TARGET).  eta2_q: host
 * [n_elem][n1d^dim] per-point weights (point index q0 + n1d q1 (+ n1d^2 q2),
 * the space-dependent weight of Section 5.2.4), or NULL for 1.  eta1, eta2
 * and every eta2_q finite and >= 0 (else TMOP_E_ARG).  metric2: a metric of
 * the context's dimension; 0 removes the second term and keeps eta1.
 * Contexts with a constant target only (else TMOP_E_UNSUPPORTED).  Replaces
 * an earlier second term or replication; after TMOP_E_NOMEM or TMOP_E_HIP
 * the earlier second term may be gone.  The device keeps omega_q per point (two
 * copies, element and colour order) and W2^-1 in the kernel arguments.
 * Syncs. */
int tmop_set_combo(tmop_ctx *ctx, int32_t metric2, const double *W2, double eta1, double eta2,
                   const double *eta2_q, void *stream);

/* Second restricted node movement algorithm (Section 4.3.2): the metric
 *   mu'(T0, T) = (1 - gamma) mu_98(T0) + gamma mu(T),  T0 = A W0^-1,
 * with W0 = A(x_init) at every quadrature point, integrated over the
 * primary target element (weight det W for both parts).  gamma in [0, 1]
 * (else TMOP_E_ARG); gamma = 0 keeps x_init, gamma = 1 is the plain
 * objective.  x_init: device [dim][n_node], read once (W0^-1 is stored per
 * point).  TMOP_E_TARGET (context unchanged) if det A(x_init) <= 0 at a
 * point.  mu_98 = |T - I|^2 / tau for the context's dimension.  Contexts
 * with a constant target only (else TMOP_E_UNSUPPORTED).  Replaces an
 * earlier second term; after TMOP_E_NOMEM or TMOP_E_HIP the earlier second
 * term may be gone.  Syncs. */
int tmop_set_replication(tmop_ctx *ctx, double gamma, const double *x_init, void *stream);

/* F and min det A as tmop_energy (eq. 2.4), and g = dF/dx as tmop_gradient
 * (Section 3.4), in one pass over the elements: the line search of Section
 * 3.4 needs both at every trial point.  The energy partials ride along in
 * the gradient's colour launches.  g: device [dim][n_node], caller-owned, not aliasing x.
 * Returns TMOP_OK, TMOP_W_INVERTED (min det A <= 0; F, g still computed) or
 * an error.  Syncs the stream. */
int tmop_energy_gradient(tmop_ctx *ctx, const double *x, double *F, double *min_detA, double *g,
                         void *stream);

/* Minimizes F over the free DOFs with Newton's method (Section 3.4):
 * direction from truncated CG (Steihaug) or MINRES (Section 5), optionally
 * Jacobi preconditioned, on the Hessian restricted to the free DOFs; step
 * lengths 1, s, s^2, ... until det A > 0 at every
 * quadrature point, F(x+) < f_growth F(x) and |g(x+)| < g_growth |g(x)|.
 * x: device [dim][n_node], updated in place (fixed DOFs keep their value).
 * opts: host, NULL = defaults.  report: host, may be NULL.  Returns TMOP_OK
 * on convergence, TMOP_W_MAXIT, TMOP_W_LSFAIL (x = last accepted iterate),
 * or TMOP_W_INVERTED if the input mesh is inverted (x untouched).  Syncs. */
int tmop_newton_solve(tmop_ctx *ctx, double *x, const tmop_newton_opts *opts,
                      tmop_newton_report *report, void *stream);

/* ------------------------------------------------------------------------
 * Derivative-free solver (Section 3.4, eq. 3.3, variational form): every
 * node in turn moves to the position that minimizes its patch quality
 *   Q(x_i) = sum over the elements E holding node i of sum_q w_q det W mu(T),
 * by the Nelder-Mead simplex method over its free components; sweeps stop
 * when no node moved more than t (max norm) in a sweep.  Nodes are visited
 * by colour (greedy in node order: a node takes the smallest colour not
 * used by a node it shares an element with); the nodes of one colour have
 * disjoint patches and move at once, which gives the same result as
 * visiting them one after the other.  Nelder-Mead after Lagarias, Reeds,
 * Wright and Wright (1998): reflection 1, expansion 2, contraction 1/2,
 * shrink 1/2; initial simplex x_i, x_i + s e_k with s = step (det W)^(1/d);
 * a node stops when every vertex lies within xtol of the best one or after
 * max_evals evaluations.  Q = +inf where det A <= 0 at a patch point, so a
 * valid mesh stays valid.  FP64 in every precision mode.  Contexts with a
 * constant target and no Section 4 term only (else TMOP_E_UNSUPPORTED). */
typedef struct {
  double t;                   /* sweep tolerance (Section 3.4: 1e-5 for unit volume) */
  int32_t max_sweeps;         /* default 100 */
  double step;                /* initial simplex edge / target size, default 0.1 */
  double xtol;                /* Nelder-Mead simplex size at which a node stops, default 1e-6 */
  int32_t max_evals;          /* Nelder-Mead evaluations per node and sweep, default 200 */
} tmop_dfo_opts;

typedef struct {
  int32_t sweeps;             /* sweeps done */
  int32_t converged;          /* 1 when the last sweep moved no node by t or more */
  double F0, F;               /* F_V at the start and at the end */
  double max_move;            /* largest node move of the last sweep */
} tmop_dfo_report;

void tmop_dfo_default_opts(tmop_dfo_opts *opts);

/* One sweep over all nodes.  x: device [dim][n_node], updated in place
 * (fixed components keep their value).  opts: host, NULL = defaults.
 * *max_move: the largest max-norm move of a node.  TMOP_E_ARG for invalid
 * options (step <= 0, xtol < 0, max_evals < 1).  The first call builds the
 * node colouring on the host; TMOP_E_UNSUPPORTED (x untouched) when a node
 * belongs to more elements than one workgroup's patch holds (at least 2^dim:
 * 4 for 2D and 8 for 3D meshes with 4 points per direction, e.g. a
 * valence-5 vertex of a 2D mesh).  Syncs. */
int tmop_dfo_sweep(tmop_ctx *ctx, double *x, const tmop_dfo_opts *opts, double *max_move, void *stream);

/* Sweeps until the largest move of a sweep is below t (TMOP_OK) or
 * max_sweeps (TMOP_W_MAXIT); TMOP_W_INVERTED (x untouched) if the input
 * mesh is inverted.  report: host, may be NULL.  Syncs. */
int tmop_dfo_solve(tmop_ctx *ctx, double *x, const tmop_dfo_opts *opts, tmop_dfo_report *report,
                   void *stream);

/* ------------------------------------------------------------------------
 * Learned initial guess for the Newton method of Section 3.4 (a layer on
 * top of the paper's method): a per-element MLP on 2D Q2 meshes that maps
 * an element's 9 nodes, relative to its centroid and divided by the target
 * size h (W = h I), to a displacement of those nodes in units of h.
 *   18 -> 64 -> 64 -> 64 -> 18, GELU on the hidden layers.
 * Feature / output index c * 9 + i (component c, local node i).  The
 * parameters are one flat FP32 array of TMOP_MLP_NPARAMS values:
 *   W1[18][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][18] b4[18]
 * The layers compute with the weights rounded to BF16 (nearest even) and
 * FP32 biases, activations and accumulation; training keeps FP32 master
 * weights and Adam moments (beta1 0.9, beta2 0.999, eps 1e-8).  Features X,
 * outputs Y and labels L are DEVICE float arrays [n][18]. */
#define TMOP_MLP_NPARAMS 10706
typedef struct tmop_mlp tmop_mlp;

/* New network on the current device from HOST params (copied); Adam state
 * zeroed. */
int tmop_mlp_create(const float *params, tmop_mlp **out);
void tmop_mlp_destroy(tmop_mlp *mlp);
/* Current FP32 master parameters to HOST params.  Syncs the device. */
int tmop_mlp_get_params(tmop_mlp *mlp, float *params);
/* Y = MLP(X) for n samples.  Async. */
int tmop_mlp_forward(tmop_mlp *mlp, const float *X, float *Y, int64_t n, void *stream);
/* dparams (DEVICE [TMOP_MLP_NPARAMS]) = d(sum dY * Y)/dparams, taken through
 * the BF16-valued weights; dX (DEVICE [n][18], or NULL) likewise.  Async. */
int tmop_mlp_backward(tmop_mlp *mlp, const float *X, const float *dY, int64_t n, float *dparams,
                      float *dX, void *stream);
/* One Adam step on the mean squared error between MLP(X) and L over n
 * samples; *loss (HOST, may be NULL) receives the loss before the step.
 * Syncs when loss != NULL. */
int tmop_mlp_train_step(tmop_mlp *mlp, const float *X, const float *L, int64_t n, float lr,
                        double *loss, void *stream);
/* Element features of x (ctx: dim 2, order 2, constant isotropic target
 * W = h I; other contexts return TMOP_E_UNSUPPORTED, as do the two calls
 * below) into X [n_elem][18].  Async. */
int tmop_mlp_features(tmop_ctx *ctx, const double *x, float *X, void *stream);
/* Training labels: ((x* - x) on the element minus its element mean) / h
 * into L [n_elem][18].  Async. */
int tmop_mlp_labels(tmop_ctx *ctx, const double *x, const double *xstar, float *L, void *stream);
/* Initial guess: x_out = x + h * (average over the elements containing each
 * node of MLP(features(x))), fixed DOFs of the mesh unchanged.  x, x_out:
 * DEVICE [2][n_node], not aliased.  Deterministic.  Async. */
int tmop_mlp_propose(tmop_ctx *ctx, tmop_mlp *mlp, const double *x, double *x_out, void *stream);

/* ------------------------------------------------------------------------
 * Per-launch timing of the element kernels (a measurement aid, not part of
 * the method): while enabled, every element-kernel launch of ctx (one per
 * energy evaluation; one per colour for gradient, Hessian action and
 * energy + gradient, the zero fill of the output excluded) is bracketed by
 * two HIP events on the caller's stream; tmop_timing_read waits for them and
 * returns the summed device time in milliseconds and the number of launches
 * for one operation: 0 energy, 1 gradient, 2 Hessian action, 3 energy +
 * gradient (tmop_energy_gradient), 4 Hessian diagonal, 5 target sizes,
 * 6 the W0 data of tmop_set_replication, 7 the displacement-penalty
 * kernels of tmop_set_restriction (every operation).  Slots 0..4 count the
 * second metric term's launches with the primary ones.
 * tmop_timing_enable(ctx, on) clears the totals and turns timing on (1) or
 * off (0).  Both return TMOP_OK, TMOP_E_ARG (NULL ctx / out pointers, op
 * outside 0..7) or TMOP_E_HIP. */
int tmop_timing_enable(tmop_ctx *ctx, int enable);
int tmop_timing_read(tmop_ctx *ctx, int op, double *ms_total, int64_t *launches);

/* Releases the context and all its device memory.  NULL is a no-op. */
void tmop_destroy(tmop_ctx *ctx);

/* Static description of a status code. */
const char *tmop_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* TMOP_H */
