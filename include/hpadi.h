/*
 * hpadi — ADI solver for the tensor-product hp-FEM discretisation of the
 * screened Poisson equation on a rectangle, for AMD MI355X (gfx950).
 *
 * Method: Knook, Olver and Papadopoulos, "Quasi-optimal complexity hp-FEM
 * for the Poisson equation on a rectangle" (arXiv 2402.11299).
 *
 *   -Laplace(u) + omega^2 u = f  on [ax,bx] x [ay,by], zero Dirichlet or zero
 *   Neumann conditions (Sec. 1 eq. poisson, Sec. 3.3), discretised in the
 *   hat + integrated-Legendre bubble basis (Sec. 2) as the generalised
 *   Sylvester equation (Sec. 3.2 eq. 2d:poisson)
 *
 *       A_Y^x U M^y + M^x U A_Y^y = G,   A_Y = K + (omega^2/2) M,   G = T_x F T_y^T,
 *
 *   and solved with the generalised ADI of Sec. 5 (Alg. 2), whose shifted
 *   1D systems are factorised by the reverse Cholesky of Sec. 4 (Alg. 1).
 *
 * Conventions for every call:
 *  - Return value: HPADI_OK (0) or a negative status; hpadi_strerror() gives
 *    text.  No C++ exception crosses this interface.
 *  - 1D coefficient order is the paper's degree-major order (Sec. 2.2):
 *    [hats | W_0 of elements 1..n | W_1 of elements 1..n | ... | W_{p-2}];
 *    Dirichlet keeps the interior hats (vertices 1..n-1), Neumann all n+1
 *    hats.  N = n p - 1 (Dirichlet) or n p + 1 (Neumann).  Piecewise
 *    Legendre coefficients (degrees 0..p) are ordered [P_0 block | P_1 block
 *    | ...], Nleg = (p+1) n.
 *  - 2D arrays are row-major: entry (i, j) at ptr[i*ld + j], i the x index
 *    (rows, Sec. 3.2), j the y index; ld >= number of columns.
 *  - Pointers named *_dev are device (HIP) memory owned by the caller;
 *    pointers named host/buf are host memory owned by the caller.  Handles
 *    and all device scratch they need are owned by the library and released
 *    by the matching *_destroy.
 *  - Device work is stream-ordered on the plan's stream (NULL = the default
 *    stream).  Calls that return data to the host (statistics, exports)
 *    synchronise that stream.  A handle is not thread-safe; distinct handles
 *    are independent.
 */
#ifndef HPADI_H
#define HPADI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HPADI_OK = 0,
    HPADI_EINVAL = -1,     /* invalid argument or size */
    HPADI_ENOTSPD = -2,    /* a factorisation met a pivot <= 0 (or NaN) */
    HPADI_ESINGULAR = -3,  /* Neumann with omega^2 <= 0: A_Y is singular */
    HPADI_EINTERVAL = -4,  /* spectral intervals not disjoint (assumption P2 of Sec. 5) */
    HPADI_ENOCONV = -5,    /* tolerance not reached; the best iterate is returned */
    HPADI_EHIP = -6,       /* a HIP runtime call failed */
    HPADI_ENOMEM = -7      /* device or host allocation failed */
};

enum { HPADI_DIRICHLET = 0, HPADI_NEUMANN = 1, HPADI_ROBIN = 2 };
enum { HPADI_FP64 = 0, HPADI_MIXED = 1 };

typedef struct hpadi_op1d_s* hpadi_op1d;
typedef struct hpadi_plan_s* hpadi_plan;

/* Per-solve statistics (host struct filled by hpadi_solve). */
typedef struct {
    int J;               /* ADI iterations per inner solve */
    int rounds;          /* refinement rounds (1 for FP64) */
    int iters;           /* total ADI iterations run */
    int status;          /* HPADI_OK or HPADI_ENOCONV */
    double interval[4];  /* [a, b, c, d] used by the plan */
    double est_rel_err;  /* estimated relative error of U (mixed mode) */
    double res_rel;      /* last FP64 relative residual ||G - A U|| / ||G|| (mixed mode) */
    int fp32_rounds;     /* rounds run with FP32 sweeps (mixed mode) */
    int J_refine;        /* ADI iterations per FP64 refinement round (mixed mode; J for FP64 plans) */
    double t_ms[3];      /* mixed mode: GPU time of the FP32 rounds, of the FP64 rounds (ADI sweeps,
                            right-hand side and final mass solve) and of the FP64 residuals, in ms,
                            from events on the plan's stream; 0 for FP64 plans (no synchronisation:
                            use hpadi_plan_timing) */
} hpadi_stats;

/* Options for hpadi_plan_create_ex (zero-initialise, then set fields). */
typedef struct {
    double inner_tol;   /* mixed mode: tolerance of the shift family of the FP32 rounds (0 = 3e-7) */
    int max_rounds;     /* mixed mode: refinement round limit (0 = 8) */
    int lines_per_block; /* half-sweep workgroup width: 1, 4 or 8 lines (0 = 4); 1 needs n % 64 == 0 on
                            that axis (else 8); 4 also selects 4-column panels in the internal layout */
    int fixed_rounds;   /* mixed mode: run exactly this many rounds, no host decision (0 = adaptive) */
    int fp32_rounds;    /* mixed mode: leading rounds with FP32 sweeps; later rounds are FP64 (0 = 1) */
    int col_lines_per_block; /* column half-sweeps only: 1, 4 or 8 lines (0 = as lines_per_block) */
    double refine_tol;  /* mixed mode: tolerance of the shift family of the FP64 refinement rounds
                           (0 = tol / inner_tol, clamped to [tol, 0.1]); later FP64 rounds
                           take the loosest of 0.1, 0.03, 0.01, ... that the previous round's
                           bound allows (built on first use) */
    int row_lines_per_block; /* row half-sweeps only: 1, 4 or 8 lines (0 = as lines_per_block) */
} hpadi_options;

/* ---- 1D operators (Sec. 2, Sec. 3.1, App. A) -------------------------- */

/* Mesh [a, b] with n elements of degree p (p >= 1, n >= 1).  breaks: host
 * array of n+1 increasing points, or NULL for a uniform mesh on [a, b].
 * bc: HPADI_DIRICHLET or HPADI_NEUMANN.  Host-only; EINVAL on bad sizes. */
int hpadi_op1d_create(int n, int p, double a, double b, const double* breaks, int bc,
                      hpadi_op1d* out);
/* The same with a condition per end (Sec. 3.3, general boundary conditions): bc_left and
 * bc_right are HPADI_DIRICHLET (the end's hat is dropped), HPADI_NEUMANN (kept) or
 * HPADI_ROBIN: alpha u + du/dn = 0 at that end, the hat kept and alpha v(x) u(x) of the
 * variational form added to K (alpha >= 0; alpha = 0 is Neumann).  Mixed conditions choose a
 * different kind per end.  Inhomogeneous Robin data g enters the right-hand side as
 * g v(x) at the end, i.e. g added to the end hat's entry of each column (row) of G.
 * The hats kept are those of vertices first..last, first = 0 unless the left end is
 * Dirichlet (then 1), last = n unless the right end is Dirichlet (then n - 1). */
int hpadi_op1d_create_ex(int n, int p, double a, double b, const double* breaks, int bc_left, int bc_right,
                         double alpha_left, double alpha_right, hpadi_op1d* out);
/* N (basis size) and Nleg = (p+1) n (Legendre coefficients per dimension). */
int hpadi_op1d_dims(hpadi_op1d op, int* N, int* Nleg);
/* Dense row-major host copies: K and M are N x N, T = R^T M_P is N x Nleg
 * (Sec. 3.1).  Any pointer may be NULL to skip it.  For tests. */
int hpadi_op1d_export(hpadi_op1d op, double* K, double* M, double* T);
void hpadi_op1d_destroy(hpadi_op1d op);

/* ---- Precomputation of Alg. 2 (host) ---------------------------------- */

/* [lo, hi] containing the generalised eigenvalues of (K + omega2/2 M, M)
 * (Alg. 2 precomputation; Sec. 5.2 lemma "Spectrum").  Lower end: the smallest
 * eigenvalue of -u'' on the interval with the operator's end conditions (pi^2/l^2 for
 * Dirichlet at both ends, 0 for Neumann at both, (pi/(2l))^2 for one of each, a
 * bisection root for Robin ends), plus omega2/2: a Galerkin eigenvalue is never below
 * it.  Upper end from a Lanczos iteration with a 1% margin.  ESINGULAR for Neumann at
 * both ends with omega2 <= 0. */
int hpadi_interval(hpadi_op1d op, double omega2, double out[2]);

/* Iteration count J = ceil(log(16 gamma) log(4/tol)/pi^2) and Zolotarev shifts
 * p_j > 0 > q_j (Alg. 2) for intervals [a,b] (of A,D) and [c,d] (of B,C) given
 * as iv[4] = {a, b, c, d}.  If J_in > 0 it overrides the computed J.  Writes
 * *J and, when p/q are non-NULL, up to maxJ shifts each.  EINTERVAL if the
 * intervals overlap or are empty; EINVAL if J exceeds maxJ. */
int hpadi_shifts(const double iv[4], double tol, int J_in, int* J, double* p, double* q, int maxJ);

/* ---- Plans: factorised shift families + device workspace --------------- */

/* Precomputation of Alg. 2 for A = A_Y^x, D = M^x, C = M^y, B = -A_Y^y:
 * interval (NULL = hpadi_interval on both axes; else {a, b, c, d}), J and
 * shifts for tol (FP64) or for the inner tolerance (MIXED), and the reverse
 * Cholesky factorisations (Alg. 1) of K_x + (omega2/2 - q_j) M_x,
 * K_y + (omega2/2 + p_j) M_y and of M_y, computed on the GPU in FP64 (plus
 * FP32 copies in MIXED mode).  hip_stream: a hipStream_t or NULL.  The
 * operators are copied; they may be destroyed afterwards.  Synchronises the
 * stream.  ENOTSPD if a factorisation fails, ESINGULAR / EINTERVAL as above.
 * EINVAL for p > 129 or more than 65 hats on an axis (n > 64 elements with
 * Dirichlet conditions, n > 64 with Neumann): the hat block of a line is solved
 * by one 64-lane wavefront. */
int hpadi_plan_create(hpadi_op1d x, hpadi_op1d y, double omega2, double tol, int precision,
                      const double* interval, void* hip_stream, hpadi_plan* out);
int hpadi_plan_create_ex(hpadi_op1d x, hpadi_op1d y, double omega2, double tol, int precision,
                         const double* interval, void* hip_stream, const hpadi_options* opts,
                         hpadi_plan* out);
/* Alg. 2 for A U C - D U B = F with general operators along each axis:
 * A = coef[0] K_x + coef[1] M_x, D = M_x, C = M_y, B = -(coef[2] K_y + coef[3] M_y), i.e.
 * A_x U M_y + M_x U A_y = G with A_x, A_y any positive definite combinations of the
 * stiffness and mass matrices (anisotropic diffusion coef[0] u_xx + coef[2] u_yy, unequal
 * screening).  hpadi_plan_create_ex is the case {1, omega2/2, 1, omega2/2}; hpadi_load,
 * hpadi_solve and hpadi_apply work on the general operator.  EINVAL unless coef[0] > 0 and
 * coef[2] > 0; ESINGULAR for a negative coef[1] or coef[3], or a zero one on an axis with
 * Neumann conditions at both ends.  Other arguments as hpadi_plan_create_ex. */
int hpadi_plan_create_general(hpadi_op1d x, hpadi_op1d y, const double coef[4], double tol, int precision,
                              const double* interval, void* hip_stream, const hpadi_options* opts,
                              hpadi_plan* out);
/* J and (when non-NULL) the J shifts p, q and the interval of the plan's ADI
 * family (the inner family in MIXED mode). */
int hpadi_plan_info(hpadi_plan plan, int* J, double* p, double* q, double interval[4]);
/* Host copy of one FP64 factor in structured form, for tests.  axis 0 = x
 * (j-th factor of K_x + (omega2/2 - q_j) M_x), axis 1 = y (K_y + (omega2/2 +
 * p_j) M_y); j = -1 is the factor of the mass matrix of that axis.  Layout of buf
 * (len >= 2(p-1)n + 4n + 2 n_h doubles):
 *   invd[(p-1)n]  1 / diagonal of L at bubble (m, e), index m n + e
 *   link[(p-1)n]  L[(m, e), (m-2, e)] at index m n + e (0 for m < 2)
 *   cpl[4n]       L[(pi, e), hat] at index 4e + 2 pi + side, side 0 = left
 *                 vertex of e, 1 = right vertex (0 when that hat is absent)
 *   invd0[n_h]    1 / diagonal of the hat factor L0
 *   link0[n_h]    L0[h, h-1] (0 for h = 0). */
int hpadi_plan_export_factor(hpadi_plan plan, int j, int axis, double* buf, size_t len);

/* G = T_x F T_y^T (Sec. 3.2): F_dev is Nleg_x x Nleg_y (ldf), G_dev is
 * N_x x N_y (ldg), both FP64 device memory. */
int hpadi_load(hpadi_plan plan, const double* F_dev, int ldf, double* G_dev, int ldg);

/* hpadi_load for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same G, computed in
 * column blocks through a fixed 16 MiB scratch array that every GPU the library runs
 * on holds until the process ends; no hipMalloc, hipFree or allocating library call.
 * hpadi_load instead allocates an Nleg_x x N_y intermediate on its first call.
 * Limit: Nleg_x <= 32768 (a block must hold at least 64 columns), else EINVAL.
 * All calls on one GPU share its scratch: calls that overlap in time on one GPU
 * (different streams, or host threads) race and must be serialised by the caller.
 * Stream-ordered on the plan's stream; the device is the one current at the call. */
int hpadi_load_noalloc(hpadi_plan plan, const double* F_dev, int ldf, double* G_dev, int ldg);

/* Solve A_Y^x U M^y + M^x U A_Y^y = G (Alg. 2).  G_dev and U_dev are FP64
 * N_x x N_y device arrays.  FP64: J ADI iterations in FP64 (relative error
 * <= tol in the norm of the ADI lemma, Sec. 5.1).  MIXED: iterative
 * refinement on the FP64 residual, every round an ADI solve with the plan's
 * shift family (tolerance inner_tol): the first fp32_rounds rounds with FP32
 * storage between half-sweeps, the later ones in FP64; the solve stops after
 * an FP64 round once the bound of the ADI lemma (Sec. 5.1) on the relative error,
 * f ||delta|| / (| ||U_old|| - ||delta|| | - f ||delta||) with f = eps/(1-eps),
 * delta the round's correction and U_old the iterate before it, all in the
 * lemma's norm ||V X L^T||_F (M^x = V^T V, M^y = L^T L), is <= tol
 * (stats->est_rel_err).  The bound covers the truncation error of the ADI
 * rounds; FP64 rounding adds its own, below 1e-11 relative in every test, and the
 * estimate is never below 16 unit roundoffs (1.8e-15): a tolerance below that ends
 * ENOCONV.
 * stats may be NULL.  ENOCONV if the
 * round limit is reached (U holds the last iterate).  Synchronises the stream
 * in MIXED mode (one scalar read-back per FP64 round). */
int hpadi_solve(hpadi_plan plan, const double* G_dev, int ldg, double* U_dev, int ldu,
                hpadi_stats* stats);

/* Y = A_Y^x U M^y + M^x U A_Y^y in FP64 (device arrays, N_x x N_y). */
int hpadi_apply(hpadi_plan plan, const double* U_dev, int ldu, double* Y_dev, int ldy);

void hpadi_plan_destroy(hpadi_plan plan);

/* ---- Batches of independent solves ------------------------------------- */

/* count independent problems A_Y^x U M^y + M^x U A_Y^y = G (operators xs[i],
 * ys[i], omega2[i]; any sizes, degrees and boundary conditions) solved to the
 * relative error tol, replayed as one HIP graph.  Each instance has a MIXED plan
 * and a fixed schedule of one round with FP32 storage and one FP64 round.  The
 * instances advance in lock step: every ADI iteration is a few grouped launches,
 * one per (direction, chain length p/2, lines per workgroup) present, each running
 * that half-sweep for all instances in it (a device task table maps workgroups to
 * instances); transforms and final solves likewise; residuals per instance.  The
 * launches of one step touch disjoint instances and are captured as parallel
 * branches over four streams (the origin and three of the batch's own, default
 * priority), joined before the next step.  Both rounds use one shift family (3e-6).
 * autotune != 0: for every distinct (n_x, p_x, n_y, p_y, boundary conditions) the
 * lines per workgroup (4 or 8) is chosen by timing both on the instance (this runs
 * solves and overwrites U[i]).  When the environment variable HPADI_TUNE_CACHE names
 * a file, choices found there for this GPU architecture are used without timing and
 * new ones are appended (text, one line per key); an unreadable or unwritable file
 * only disables the cache.  G[i], U[i]: FP64 device arrays N_x x N_y (ld ldg[i],
 * ldu[i]) bound to the graph: later solves read and write these same arrays.
 * nstreams: reserved, pass 0.  hip_stream: the stream the graph is launched on (a
 * hipStream_t, or NULL for a stream of the batch's own). */
typedef struct hpadi_batch_s* hpadi_batch;
int hpadi_batch_create(int count, const hpadi_op1d* xs, const hpadi_op1d* ys, const double* omega2, double tol,
                       const double* const* G, const int* ldg, double* const* U, const int* ldu, int autotune,
                       int nstreams, void* hip_stream, hpadi_batch* out);
/* Launch the graph and wait for it; then, per instance, the ADI lemma bound of
 * its FP64 round (as in hpadi_solve); instances above tol get further FP64
 * rounds outside the graph (*n_extra counts them; may be NULL).  stats: host
 * array of count entries or NULL.  ENOCONV if an instance stays above tol. */
int hpadi_batch_solve(hpadi_batch b, hpadi_stats* stats, int* n_extra);
/* Tuned lines per workgroup and J of instance i; stream_index is 0 (any pointer may be NULL). */
int hpadi_batch_info(hpadi_batch b, int i, int* lines_per_block, int* J, int* stream_index);
void hpadi_batch_destroy(hpadi_batch b);

/* ---- Variable coefficient and ADI-preconditioned CG (Sec. 7) ----------- */

/* -div(a grad u) = f with the same bases and boundary conditions as the plans:
 * the Galerkin form sum_e sum_(i,j) w_i w_j a(x_i, y_j) grad u . grad v is
 * evaluated with q = p + 2 Gauss-Legendre points per element and dimension
 * (exact for a polynomial a of degree <= 3 per variable).  Sec. 7 solves such
 * a problem by CG preconditioned with the constant-coefficient ADI solve at a
 * loose tolerance. */
typedef struct hpadi_varcoef_s* hpadi_varcoef;

/* Quadrature grid of one axis, host: x[e q + i] physical Gauss point i of
 * element e, w[e q + i] its weight including the Jacobian delta_e / 2, q = p + 2.
 * len >= n q.  Either pointer may be NULL. */
int hpadi_varcoef_grid(hpadi_op1d op, double* x, double* w, int len);
/* Operator for the coefficient a_dev[(e_x q_x + i) * lda + e_y q_y + j] =
 * a(x_i of e_x, y_j of e_y): FP64 device memory, (n_x q_x) x (n_y q_y), copied
 * (the caller may free it afterwards).  EINVAL when (p_x+1)(p_y+1) + (p_x+2)(p_y+1)
 * + (p_x+2)(p_y+2) + (p_y+1)(p_y+2) doubles exceed 160 KiB (p up to about 80). */
int hpadi_varcoef_create(hpadi_op1d x, hpadi_op1d y, const double* a_dev, int lda, void* hip_stream,
                         hpadi_varcoef* out);
/* The operator of -div(a grad u) + c u (Sec. 7: the paper's example is
 * (-Laplace - 10 log r) u = 1, a = 1 and a potential c): a_dev as above or NULL
 * for a = 1; c_dev the potential on the same Gauss grid (ldc), or NULL for none;
 * both copied.  Terms on a = 1 and the potential run as separable passes along
 * each axis (any p); a variable a uses the element kernel (the p limit above).
 * Host arrays hold the combined quadrature weights of each term. */
int hpadi_varcoef_create_ex(hpadi_op1d x, hpadi_op1d y, const double* a_dev, int lda, const double* c_dev, int ldc,
                            void* hip_stream, hpadi_varcoef* out);
/* Y = A_a U (FP64 device arrays N_x x N_y, row-major), stream-ordered. */
int hpadi_varcoef_apply(hpadi_varcoef vc, const double* U_dev, int ldu, double* Y_dev, int ldy);
void hpadi_varcoef_destroy(hpadi_varcoef vc);

typedef struct {
    int iters;            /* Krylov iterations (operator applications) */
    int status;           /* HPADI_OK, HPADI_ENOCONV or HPADI_ENOTSPD */
    int precond_calls;    /* preconditioner applications */
    int corrections;      /* learned corrections accepted (0 without a network) */
    double rel_res;       /* ||r_k|| / ||b|| of the recurrence residual at exit */
    double true_rel_res;  /* ||b - A_a x|| / ||b||, recomputed in FP64 at exit */
    double t_ms;          /* host wall time of the call */
    int fallback_iters;   /* iterations of plain ADI-PCG after the learned correction was given up */
    int reserved_i;
    double reserved[2];
} hpadi_krylov_stats;

/* ---- Learned correction (an addition to Sec. 7's ADI-preconditioned CG) -- */

/* A small convolutional network on the coefficient image: per dimension the
 * coefficients are laid out element by element (the element's left-vertex hat,
 * then W_0 .. W_{p-2}; one trailing slot for the last vertex), an image of
 * (n_x p_x + 1) x (n_y p_y + 1) pixels.  Channels 3 -> 32 -> 32 -> 32 -> 1, 3x3
 * convolutions with zero padding, tanh-form GELU after the hidden layers; BF16
 * activations and weights on the matrix cores with FP32 accumulation, FP32
 * master parameters.  Inside the Krylov loop the preconditioned residual z is
 * corrected by c = s_z NN([z/s_z, (z/s_z)/a, log a]) (s_z: root-mean-square value of z):
 * z <- z + (beta/alpha) c with alpha z + beta c the energy-optimal combination
 * (it minimises ||v - e||_A over span{z, c} for the error e of the iterate, which
 * needs A z and A c: two extra operator applications per iteration); a
 * degenerate or non-finite combination falls back to the plain z. */
typedef struct hpadi_net_s* hpadi_net;

/* Number of FP32 parameters: W0[3][3][3][32] b0[32] W1[3][3][32][32] b1[32]
 * W2[3][3][32][32] b2[32] W3[3][3][32][1] b3[1], in that order (W[dy][dx][c_in][c_out]). */
int hpadi_net_num_params(void);
/* params: host array of hpadi_net_num_params() floats, or NULL for a seeded
 * initialisation (normal, std sqrt(2 / fan_in), last layer scaled by 1/10,
 * zero biases).  hip_stream: a hipStream_t or NULL. */
int hpadi_net_create(const float* params, unsigned long long seed, void* hip_stream, hpadi_net* out);
int hpadi_net_get_params(hpadi_net net, float* params);
int hpadi_net_set_params(hpadi_net net, const float* params);
/* How the correction c enters the Krylov loop: omega = 0 (the default) combines z
 * and c energy-optimally (two extra operator applications and two host round trips
 * per iteration); omega > 0 uses z <- z + omega c, with the scale s_z kept on the
 * device (no operator application, no host round trip).  EINVAL for omega < 0. */
int hpadi_net_set_damping(hpadi_net net, double omega);
/* Apply the correction at Krylov iterations 0, period, 2 period, ... only (period >= 1,
 * default 1); the other iterations use the plain preconditioned residual.  EINVAL for
 * period < 1. */
int hpadi_net_set_period(hpadi_net net, int period);
/* out = NN(x): x FP32 device [B][H][W][3], out FP32 device [B][H][W]. */
int hpadi_net_forward(hpadi_net net, const float* x_dev, int B, int H, int W, float* out_dev);
/* Loss of a batch and its gradient with respect to the parameters (host copy),
 * without updating:  L = (1/B) sum_b sum_p w (zn + NN(x) - t)^2 / sum_p w t^2.
 * x [B][H][W][3], zn, t, w [B][H][W]: FP32 device.  W must be a multiple of 16.
 * grad may be NULL. */
int hpadi_net_loss_grad(hpadi_net net, const float* x_dev, const float* zn_dev, const float* t_dev,
                        const float* w_dev, int B, int H, int W, double* loss, float* grad);
/* Adam training (beta 0.9, 0.999, eps 1e-8) on npairs crops of c x c pixels
 * (arrays laid out as for hpadi_net_loss_grad with B = npairs): steps steps of
 * batch crops drawn uniformly with a counter-based generator from seed.
 * loss_hist (host, may be NULL) receives the loss of each step. */
int hpadi_net_train(hpadi_net net, const float* X_dev, const float* ZN_dev, const float* T_dev, const float* W_dev,
                    int npairs, int c, int batch, int steps, double lr, unsigned long long seed, float* loss_hist);
/* Training pairs from the method: plain preconditioned CG (truncation 0) on
 * A_a x = b from x = 0; after the preconditioner of iteration k the images
 * [z/s_z, (z/s_z)/a, log a], zn = z/s_z, t = (xstar - x_k)/s_z and the slot weights
 * w = a (diag K_x diag M_y + diag M_x diag K_y), the diagonal of the energy form,
 * are formed and crops_per_iter
 * random c x c crops of them are appended to X (3 ch), ZN, T, Wt (FP32 device,
 * capacity cap crops).  xstar: the converged solution (device, ldxs).  Stops
 * after max_iters iterations, at convergence (tol) or when cap crops are
 * stored; *count = crops stored. */
int hpadi_net_pairs(hpadi_varcoef vc, hpadi_plan precond, const double* b_dev, int ldb, const double* xstar_dev,
                    int ldxs, double tol, int max_iters, int c, int crops_per_iter, unsigned long long seed,
                    float* X_dev, float* ZN_dev, float* T_dev, float* W_dev, int cap, int* count);
void hpadi_net_destroy(hpadi_net net);

/* Solve A_a x = b from x = 0 until ||r_k||_2 / ||b||_2 <= tol (FP64 vectors).
 * truncation = 0: preconditioned CG; 1..4: flexible CG keeping that many
 * previous directions (each new direction is the preconditioned residual made
 * A_a-orthogonal to them; alpha = d.r / d.A d).  precond: an ADI plan whose
 * solve is the preconditioner (its N_x, N_y must match; typically omega2 = 0,
 * tol 1e-4), or NULL for none.  net: a learned correction applied after each
 * preconditioner application (NULL for none; use truncation >= 1 with it, the
 * corrected preconditioner is not a fixed linear map).  Plain ADI-PCG is the
 * correction's fallback: the corrected run is given up on a non-finite or
 * non-positive curvature d.A d, on divergence (the residual 100 times its best),
 * on stagnation (ten iterations without halving the residual) or after maxit / 2
 * iterations, and PCG with the same preconditioner continues
 * from the last iterate (from x = 0 if that is not finite or its residual exceeds
 * ||b||) for the remaining iterations (stats->fallback_iters).  res_hist (host, may be
 * NULL) receives the relative recurrence residual of iterates
 * 0..min(iters, hist_len-1).  Synchronises the stream once per dot product.
 * ENOCONV after maxit iterations (x holds the last iterate); ENOTSPD if
 * d.A d <= 0. */
int hpadi_fcg_solve(hpadi_varcoef vc, hpadi_plan precond, hpadi_net net, const double* b_dev, int ldb, double* x_dev,
                    int ldx, double tol, int maxit, int truncation, double* res_hist, int hist_len,
                    hpadi_krylov_stats* stats);

/* ---- Grid transforms and the Burgers time-stepper (Sec. 6) ------------- */

/* The grid of one axis (host): on every element the m = p + 1 Chebyshev points of the
 * first kind t_k = sin(pi (m - 2k - 1) / (2m)), k = 0..m-1 (descending; Sec. 6 counts
 * them from 1), mapped to the element: x[e m + k] = x_e + (1 + t_k) delta_e / 2.
 * len >= n m.  Values on a 2D grid are stored element-major along each axis: entry
 * (e_x m_x + k, e_y m_y + j), an (n_x m_x) x (n_y m_y) array (n m = Nleg). */
int hpadi_grid(hpadi_op1d op, double* x, int len);

/* Host copy of one reference-element table of degree p, row-major (p+1) x (p+1), for
 * tests: which = 0 the transform F_p (Legendre coefficient k from value i), 1 its inverse
 * (P_k(t_i)), 2 the local basis at the points (columns: left hat, right hat, W_0..W_{p-2}),
 * 3 their t-derivatives.  Host-only. */
int hpadi_transform_export(int p, int which, double* buf, int len);

typedef struct hpadi_transform_s* hpadi_transform;
/* Reference-element tables of both axes on the device, and an intermediate array of
 * max(Nleg_x, N_x) x Nleg_y doubles.  hip_stream: the stream of every call on the handle.
 * The operators are copied.  EINVAL for p > 239 on an axis (a workgroup stages the p + 1
 * inputs of 64 lines of an element in LDS). */
int hpadi_transform_create(hpadi_op1d x, hpadi_op1d y, void* hip_stream, hpadi_transform* out);
/* F = F_x V F_y^T (Sec. 6, the transform F_p on every element along each axis): the
 * piecewise Legendre coefficients (Nleg_x x Nleg_y, degree-major) of the interpolant of
 * the grid values V (element-major).  FP64 device arrays; V and F must not overlap. */
int hpadi_values_to_legendre(hpadi_transform t, const double* V_dev, int ldv, double* F_dev, int ldf);
/* V = F_x^{-1} F F_y^{-T}: the piecewise Legendre series F evaluated on the grid. */
int hpadi_legendre_to_values(hpadi_transform t, const double* F_dev, int ldf, double* V_dev, int ldv);
/* Grid values of u = Q_x U Q_y^T (deriv_x = 0), i.e. F_x^{-1} R_x U R_y^T F_y^{-T}, or of
 * du/dx (deriv_x = 1), F_x^{-1} D_x U R_y^T F_y^{-T} (Sec. 6).  U_dev: N_x x N_y
 * coefficients in the hat+bubble basis; V_dev: (n_x m_x) x (n_y m_y). */
int hpadi_q_to_values(hpadi_transform t, int deriv_x, const double* U_dev, int ldu, double* V_dev, int ldv);
void hpadi_transform_destroy(hpadi_transform t);

/* u_t + u u_x = eps Laplace(u) on the rectangle of the operators, with their (zero)
 * boundary conditions, by the splitting of Sec. 6: implicit Euler for the viscous part,
 * (I - dt eps Laplace) u_{k+1/2} = u_k, solved by the ADI plan of the screened problem with
 * omega^2 = 1 / (dt eps) and right-hand side omega^2 u_k; then explicit Euler for the
 * convection at the grid points, u_{k+1} = u_{k+1/2} - dt u_{k+1/2} d/dx u_{k+1/2} (the
 * sign of the equation as written), and back to Legendre coefficients by F_p.  tol,
 * precision, opts: those of the plan (hpadi_plan_create_ex).  EINVAL unless eps > 0 and
 * dt > 0. */
typedef struct hpadi_burgers_s* hpadi_burgers;
int hpadi_burgers_create(hpadi_op1d x, hpadi_op1d y, double eps, double dt, double tol, int precision,
                         const hpadi_options* opts, void* hip_stream, hpadi_burgers* out);
/* Advance F_dev (Nleg_x x Nleg_y piecewise Legendre coefficients of u, FP64 device, in place)
 * by nsteps steps.  stats: the last step's solve (may be NULL).  ENOCONV when a solve
 * missed its tolerance: F then holds the step that used it, and no further step is taken. */
int hpadi_burgers_step(hpadi_burgers b, double* F_dev, int ldf, int nsteps, hpadi_stats* stats);
void hpadi_burgers_destroy(hpadi_burgers b);

/* ---- Measurement ------------------------------------------------------- */

/* Kernel timing for roofline measurement: while enabled, HIP events are
 * recorded on the plan's stream around every half-sweep launch.  enable = 1
 * clears the totals and starts recording, 0 stops.  At most 65536 launches are
 * recorded per enable; later launches run untimed. */
int hpadi_plan_timing(hpadi_plan plan, int enable);
/* Totals since the last enable, by kind: 0 = full column half-sweeps of the
 * ADI loop, 1 = full row half-sweeps, 2 = the others: the transforms into the
 * mass-balanced coordinates, the last column half-sweep of each solve (a solve
 * only) and the final mass solve back to U; kinds 3, 4, 5 are the same for
 * sweeps whose iterate storage is FP64 (FP64 plans and the FP64 rounds of mixed
 * plans), kinds 0-2 then hold the FP32-storage sweeps.  ms[k]: summed kernel
 * durations; bytes[k]: summed algorithmic HBM bytes of those launches (every
 * array entry read or written once: input, G~ and output of a fused sweep);
 * count[k]: launches.  Any pointer may be NULL.  Synchronises the stream. */
int hpadi_plan_timing_read(hpadi_plan plan, double ms[6], double bytes[6], int count[6]);

const char* hpadi_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* HPADI_H */
