/*
 * sdbie: regularised boundary-integral Stokes-Darcy solver for one GPU (gfx950).
 *
 * C ABI.  Every pointer argument named as device memory must point to memory
 * on the current HIP device (for example a torch tensor's data); every
 * floating-point array is IEEE double, contiguous, and vector fields are
 * component-major "SoA": element (c, j) of a 3-vector field lives at
 * v[c * n + j].  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  All work is enqueued on that stream; outputs are valid once the
 * stream has reached the end of the call (the caller synchronises).  Solves
 * synchronise the stream internally (the Krylov least-squares step runs on
 * the host) and return only after their outputs are written.
 *
 * Ownership: the library never allocates or frees device memory.  The caller
 * passes a workspace of sdbie_workspace_bytes() bytes to sdbie_plan_create();
 * a plan refers to that workspace (and copies the node data into it) until
 * sdbie_plan_destroy().  Calls on one plan must not overlap in time; plans
 * with separate workspaces are independent.
 *
 * Errors: every function returns an int status.  0 = SDBIE_OK; 1 =
 * SDBIE_NOT_CONVERGED (outputs hold the last iterate, `info` is filled);
 * negative values are errors and leave outputs unspecified.  A message for
 * the last error of the calling thread is returned by sdbie_last_error().
 * No C++ exception crosses this interface.
 *
 * Paper: S. Tlupova, "A domain decomposition solution of the Stokes-Darcy
 * system in 3D based on boundary integrals" (arXiv 2110.10749).
 */
#ifndef SDBIE_H
#define SDBIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDBIE_OK 0
#define SDBIE_NOT_CONVERGED 1
#define SDBIE_ERR_ARG (-1)       /* invalid argument (null pointer, size, parameter range) */
#define SDBIE_ERR_NONFINITE (-2) /* NaN or Inf in the node data or in an iterate */
#define SDBIE_ERR_DEVICE (-3)    /* a HIP call or kernel launch failed */
#define SDBIE_ERR_WORKSPACE (-4) /* workspace missing, too small or misaligned */

/* Arithmetic of the pair sums.  SDBIE_FP64: every pair in double.
 * SDBIE_MIXED: pair geometry, smoothing and kernel values in float,
 * per-tile partial sums added into double accumulators per target; solves
 * recover double accuracy by iterative refinement with double residuals. */
typedef enum { SDBIE_FP64 = 0, SDBIE_MIXED = 1 } sdbie_precision;

/* Which layer sum (section "High-order regularization of kernels on the
 * surface"; every sum includes j = i with the finite rho -> 0 limits):
 *   SDBIE_SL     single layer:  Laplace  S_L[g]_i = -(1/4pi) sum_j w_j g_j s1(r/d)/r
 *                               Stokes   V[f]_i   = (1/(8 pi mu)) sum_j w_j [f_j s1/r + D (D.f_j) s3/r^3]
 *   SDBIE_DL_RAW double layer:  Laplace  D_L[p]_i = -(1/4pi) sum_j w_j p_j (D.n_j) s2/r^3
 *                               Stokes   D_S[u]_i = -(3/4pi) sum_j w_j (u_j.D)(D.n_j) D s4/r^5
 *   SDBIE_DL_SUB double layer with the singularity subtracted, eqs. (H_subtr) and (K_subtr):
 *                               Laplace  A_D[p]_i = (1/4pi) sum_j w_j (p_j-p_i)(D.n_j) s2/r^3  (= p/2 - H p)
 *                               Stokes   A_S[u]_i = u_i - (3/4pi) sum_j w_j ((u_j-u_i).D)(D.n_j) D s4/r^5 (= u/2 - K u)
 * with D = x_i - x_j, r = |D|, d = delta and the smoothing functions s1..s4
 * of the paper.  No completion term is added by the layer applies. */
typedef enum { SDBIE_SL = 0, SDBIE_DL_RAW = 1, SDBIE_DL_SUB = 2 } sdbie_layer;

/* Node set of a closed surface (section "Quadrature", eq. (Quadrature)):
 * points x, unit normals nrm pointing out of the porous body into the fluid,
 * quadrature weights w >= 0 (device memory, [3][n], [3][n], [n]), and the
 * regularisation width delta > 0 (the paper uses delta = 3h).  Accepted
 * range: |coordinates| <= 1e15 and 1e-15 <= delta <= 1e15 (every squared
 * pair distance is then a normal number in float and double). */
typedef struct {
    int64_t n;
    const double* x;
    const double* nrm;
    const double* w;
    double delta;
} sdbie_surface;

/* Physical parameters: viscosity mu > 0, permeability K > 0 (the paper's
 * kappa), slip coefficient alpha >= 0 (the paper's gamma); the slip
 * traction is beta * (u - (u.n) n) with beta = alpha * mu / sqrt(K). */
typedef struct {
    double mu;
    double K;
    double alpha;
} sdbie_params;

typedef struct {
    double tol_gmres;   /* local solves: stop at ||r||_2 <= tol ||b||_2 */
    double tol_ddm;     /* interface loop: residual of eq. (DDM_residual) (relaxation) or
                           relative GMRES residual of the interface equation (outer = 1) */
    double theta;       /* relaxation parameter of eq. (q_update), 0 < theta < 1 */
    int maxit_gmres;    /* per local solve */
    int restart;        /* GMRES restart length, 1 <= restart <= the plan's max_restart */
    int maxit_ddm;      /* interface iterations (relaxation) or outer GMRES iterations */
    int outer;          /* 0: relaxation (section "Algorithm"); 1: GMRES on the interface unknown */
    int slip;           /* 0: slip traction implicit in the Stokes solve; 1: lagged by one
                           interface iteration as printed in the algorithm */
    int prec;           /* sdbie_precision of the pair sums in the solves */
    double tol_mixed;   /* SDBIE_MIXED: mixed_mode 0 and 1: relative tolerance of each float-pair
                           correction solve; mixed_mode 2: relative residual below which the
                           GMRES products of a local solve at tol_gmres switch to float pairs (a
                           local solve at a looser tolerance tol, an inexact interface product,
                           switches at min(1, tol_mixed * tol / tol_gmres)) */
    int refine_max;     /* SDBIE_MIXED, mixed_mode 0 and 1: maximum refinement steps */
    int mixed_mode;     /* SDBIE_MIXED: 0 = iterative refinement of every local solve (double
                           residual, float-pair correction solves); 1 = (outer = 1 only) refinement
                           of the coupled system (double residual of both equations, float-pair
                           D-N corrections); 2 = relaxed GMRES in every local solve (double-pair
                           products until the residual reaches tol_mixed, float pairs after it,
                           convergence decided by a double-pair true residual) */
    int relax_outer;    /* outer = 1: 1 = inexact interface products (local solves of an interface
                           GMRES step loosened in proportion to the interface residual reached,
                           float pairs throughout once loose enough with SDBIE_MIXED; convergence
                           decided by the true interface residual of full-accuracy final solves);
                           0 = every local solve to tol_gmres */
    int local_solver;   /* 0 = GMRES; 1 = successive approximations of eqs. (Darcy_BIEM_iter),
                           (Stokes_BIEM_iter): x <- x + (b - A x) with the completed operator,
                           double pairs, until the relative change ||dx|| / ||x|| <= tol_gmres
                           (converges only while the spectral radius of I - A is below 1: no
                           or weak slip); maxit_gmres bounds the sweeps */
    int recycle;        /* SDBIE_FP64: 1 = the Stokes local solves of ddm_solve after the first
                           deflate the last GMRES cycle of that first solve (its Krylov basis V
                           and Arnoldi relation A V_k = V_{k+1} H, H = QR: U = V_k R^-1,
                           C = V_{k+1} Q with A U = C; the initial residual is projected off C
                           and every new Krylov vector orthogonalised against C); 0 = plain
                           GMRES.  Not used with float pairs. */
} sdbie_opts;

typedef struct {
    int ddm_iters;          /* interface iterations (relaxation) or outer GMRES iterations */
    int gmres_iters;        /* inner GMRES iterations, all local solves */
    int refine_steps;       /* SDBIE_MIXED refinement steps */
    int64_t applies_fp64;   /* layer-sum kernel passes, double pairs */
    int64_t applies_mixed;  /* layer-sum kernel passes, float pairs */
    double pairs;           /* (target, source) pair evaluations, all passes */
    double ddm_res;         /* final interface residual */
    double relres;          /* final relative residual of the last local solve */
} sdbie_info;

typedef struct sdbie_plan_s* sdbie_plan;

/* Fill `o` with the defaults: tol_gmres 1e-10, tol_ddm 1e-8, theta 0.5,
 * maxit_gmres 500, restart 50, maxit_ddm 200, outer 1, slip 0, prec FP64,
 * tol_mixed 1e-4, refine_max 8, mixed_mode 2, relax_outer 1, local_solver 0, recycle 1. */
void sdbie_default_opts(sdbie_opts* o);

/* Bytes of device workspace a plan for n nodes (1 <= n <= 2^23) and GMRES
 * restart length up to max_restart (1..1000) needs (0 if the arguments are
 * invalid).  Roughly (120 max_restart + 1185 + 96 S) n bytes plus
 * (n/256)^2 * 3471, with S the source splits of a pair pass (a multiple of 8
 * up to 64: 64 at n = 4096, 16 at n = 68166, 8 from n = 131072 on); the
 * quadratic term is the tile masks and the work lists and partial sums of the
 * symmetric far field (sdbie_plan_set_symmetric): 0.84 GB at n = 68166,
 * 9.4 GB at n = 351866 with max_restart = 50.  Above n = 524288 a plan holds
 * no symmetric lists (the quadratic term drops to the masks, (n/256)^2 * 2)
 * and runs every pass one direction at a time. */
size_t sdbie_workspace_bytes(int64_t n, int max_restart);

/* Stage a surface: spatial (Morton) ordering, double and float copies of the
 * node data, tile bounds.  `ws` (device, 256-byte aligned, ws_bytes >=
 * sdbie_workspace_bytes(s->n, max_restart)) must stay valid until the plan is
 * destroyed; the node arrays of `s` are copied and may be freed afterwards.
 * Synchronises `stream`.  Errors: ERR_ARG (also coordinates or delta out of
 * the accepted range), ERR_WORKSPACE, ERR_NONFINITE (non-finite node data or
 * weights), ERR_DEVICE. */
int sdbie_plan_create(sdbie_plan* plan, const sdbie_surface* s, int max_restart,
                      void* ws, size_t ws_bytes, void* stream);
int sdbie_plan_destroy(sdbie_plan plan);
int64_t sdbie_plan_n(sdbie_plan plan);

/* Target-source symmetric far field (section "Numerical Results", local
 * problems: the paper's code evaluates each pair of nodes once for both
 * directions).  `families` is a mask of SDBIE_SYM_LAPLACE and SDBIE_SYM_STOKES
 * (the Laplace or Stokes passes with float pairs) and SDBIE_SYM_LAPLACE_F64
 * and SDBIE_SYM_STOKES_F64 (the same with double pairs): in every later layer
 * sum and solve on the plan (the transposed sums of ddm_adjoint excepted) a
 * pass of a selected kind evaluates each tile pair whose node pairs all lie
 * beyond the smoothing cutoff once, adding its contributions to the targets
 * of both tiles; near tile pairs stay one pass per direction.  Same sums up to
 * rounding.  0: every ordered pair in its own pass.  Plans of more than 524288
 * nodes have no room for the symmetric lists and keep every pass
 * one-directional whatever the mask.  The default, SDBIE_SYM_DEFAULT, selects
 * every kind: each is at least as fast symmetric on gfx950.  ERR_ARG for a
 * null plan or unknown bits. */
#define SDBIE_SYM_LAPLACE 1
#define SDBIE_SYM_STOKES 2
#define SDBIE_SYM_LAPLACE_F64 4
#define SDBIE_SYM_STOKES_F64 8
#define SDBIE_SYM_ALL 15
#define SDBIE_SYM_DEFAULT (SDBIE_SYM_LAPLACE | SDBIE_SYM_STOKES | SDBIE_SYM_LAPLACE_F64 | SDBIE_SYM_STOKES_F64)
int sdbie_plan_set_symmetric(sdbie_plan plan, int families);

/* out = layer sum of `dens` (device, [n] for Laplace, [3][n] for Stokes, in
 * the caller's node order) at every node.  out must not alias dens.
 * Stokes single layer uses viscosity mu > 0 (ignored by the double layers). */
int laplace_layer_apply(sdbie_plan plan, sdbie_layer layer, const double* dens, double* out,
                        sdbie_precision prec, void* stream);
int stokes_layer_apply(sdbie_plan plan, double mu, sdbie_layer layer, const double* dens,
                       double* out, sdbie_precision prec, void* stream);

/* Allocation-free Stokes layer sum, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the same sums as stokes_layer_apply (same kernels) for
 * a surface given directly, staged on every call into a fixed device array
 * of the library (24 MiB per device the library runs on, held until the
 * process ends) instead of a plan's workspace.  No device memory is
 * allocated or freed.  Surfaces of 1 <= s->n <= SDBIE_NOALLOC_MAX_NODES
 * nodes; larger ones return SDBIE_ERR_ARG (use a plan).  dens, out: device
 * [3][n] in the caller's node order (out must not alias dens).  Staging
 * synchronises `stream` (it reads back the finiteness check and the weight
 * sum).  The array is shared by every call on a device and keeps the last
 * call's contents: calls that overlap in time on one device race.  Errors as
 * for sdbie_plan_create and stokes_layer_apply. */
#define SDBIE_NOALLOC_MAX_NODES 32768
int stokes_layer_apply_noalloc(const sdbie_surface* s, double mu, sdbie_layer layer, const double* dens,
                               double* out, sdbie_precision prec, void* stream);

/* Darcy problem, eq. (Darcy_final): given v = u.n on the nodes (device [n]),
 * solve (1/2 - H) p = b_D with b_D = -L dp/dn, dp/dn = -(mu/K) v, as
 * (A_D + w^T p/|S|) p = -S_L[dp/dn] by GMRES (the rank-one term fixes the
 * constant null vector of A_D), then remove the weighted mean of p.
 * p (device [n]) holds the initial guess on entry (zero it for none). */
int darcy_solve(sdbie_plan plan, const sdbie_params* prm, const double* vn, double* p,
                const sdbie_opts* opts, sdbie_info* info, void* stream);

/* Stokes problem, eq. (Stokes_final), with traction eq. (f) read as
 * f = -p n + beta (u - (u.n) n) + f_extra:
 *   (A_S + n (w n)^T/|S|) u + V[beta P_tau u] = U - V[-p n + f_extra]   (slip = 0), or
 *   (A_S + n (w n)^T/|S|) u = U - V[f(p, u_prev)]                       (slip = 1, u_prev = entry u).
 * U: host double[3] far-field velocity; p: device [n]; f_extra: device
 * [3][n] or NULL; u: device [3][n], initial guess on entry. */
int stokes_solve(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* p,
                 const double* f_extra, double* u, const sdbie_opts* opts, sdbie_info* info,
                 void* stream);

/* Coupled problem by the Dirichlet-Neumann iteration (sections "The
 * Dirichlet-Neumann iterative method" and "Algorithm"): Darcy solve with
 * the normal velocity, Stokes solve with the traction from p_D, relaxed
 * update of the interface unknown (outer = 0) or GMRES on the affine
 * interface map (outer = 1).  Outputs p (device [n]), u (device [3][n])
 * and the drag (host double[3]) by eq. (drag_int), D = sum_j w_j f_j.
 * f_extra (device [3][n] or NULL) is a prescribed extra traction (the
 * paper's benchmark adds the exact viscous traction of its test problem).
 * NOT_CONVERGED when the interface residual or a final local solve misses
 * its tolerance (with inexact interface products, relax_outer = 1, the
 * local solves inside the products only make the products inexact: the
 * final solves and the true interface residual decide). */
int ddm_solve(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* f_extra,
              double* p, double* u, double drag[3], const sdbie_opts* opts, sdbie_info* info,
              void* stream);

/* Adjoint of ddm_solve (not in the paper): gradient of J = dJ_ddrag . drag
 * with respect to the node coordinates (device [3][n], normals and weights
 * held fixed: the derivative of the discrete map), log K and alpha (host
 * doubles).  p, u (device [n], [3][n], caller order) are the converged
 * outputs of ddm_solve for the same plan, parameters, U and f_extra; only they
 * are needed (no Krylov history).  The transposed coupled system is solved by
 * the transposed interface iteration (interface GMRES to opts->tol_ddm, local
 * GMRES to opts->tol_gmres; with opts->relax_outer the inexact interface
 * products and true-residual correction cycles of ddm_solve); with
 * opts->prec = SDBIE_MIXED the transposed local solves use the relaxed scheme
 * of the forward solves (float pairs below the switch point, double true
 * residuals), otherwise double pairs; then one position-gradient pass in
 * double.  Returns NOT_CONVERGED if a Krylov solve missed its tolerance. */
int ddm_adjoint(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* f_extra,
                const double* p, const double* u, const double dJ_ddrag[3], double* dJ_dx,
                double* dJ_dlogK, double* dJ_dalpha, const sdbie_opts* opts, sdbie_info* info,
                void* stream);

/* Spectrum of the Dirichlet-Neumann iteration (section "Discrete iteration
 * operator", eqs. (Discrete_iter_oper), (A_mat)).  With no far-field flow
 * the D-N map is linear, T_lin(v) = u(p(v)).n: p the Darcy solution for the
 * normal velocity v (weighted mean removed), u the Stokes solution for the
 * traction -p n (with the implicit slip term when prm->alpha > 0).  The
 * relaxed iteration's matrix is A~ = (1 - theta) I + theta T_lin, so its
 * eigenvalues are 1 - theta + theta lambda for the eigenvalues lambda of
 * T_lin.  m Arnoldi steps on T_lin from v0 (device [n], caller order,
 * nonzero), each product one Darcy and one Stokes solve to opts->tol_gmres
 * with opts->prec pairs (1 <= m <= the plan's max_restart); the Ritz values
 * (eigenvalues of the Hessenberg matrix, by the Francis QR iteration on the
 * host) approximate the eigenvalues of largest modulus first.  eig_re,
 * eig_im: host double[k] (1 <= k <= m) receive the k Ritz values of largest
 * modulus in decreasing modulus (NaN past the steps taken when the Krylov
 * space becomes invariant; info->ddm_iters = steps taken).  Returns
 * NOT_CONVERGED if a local solve missed its tolerance or the QR iteration
 * stalled (then the eigenvalues it did not reach are NaN, listed last). */
int ddm_dn_spectrum(sdbie_plan plan, const sdbie_params* prm, const double* v0, int m, int k, double* eig_re,
                    double* eig_im, const sdbie_opts* opts, sdbie_info* info, void* stream);

/* Eigenvalues of an upper Hessenberg matrix H (host, n x n, row-major; the
 * entries below the subdiagonal are ignored) by the Francis double-shift QR
 * iteration, the host step of ddm_dn_spectrum: eig_re, eig_im (host
 * double[n]) in no particular order, complex pairs adjacent.  NOT_CONVERGED
 * if 30 max(10, n) QR steps pass without a deflation (the eigenvalues not
 * reached are NaN); ERR_ARG for n < 1 or a null pointer. */
int sdbie_hessenberg_eigenvalues(int n, const double* H, double* eig_re, double* eig_im);

/* Kernel timing (diagnostics).  While enabled, every pair-sum kernel launch
 * records a HIP event pair around the kernel on the stream it runs on.
 * sdbie_profile_enable(1) clears old records and starts recording;
 * sdbie_profile_enable(0) clears and stops.  sdbie_profile_read() waits for
 * the recorded events and writes up to `max` per-variant summaries (count
 * receives the number of variants): launches, summed kernel milliseconds,
 * pair evaluations, and the algorithmic far-field flops per pair of that
 * variant (FMA = 2, add/mul = 1, rsqrt = 1).  Process-wide; not reentrant
 * with concurrent recording threads.  Errors: ERR_ARG (null count, or null
 * out with max > 0), ERR_DEVICE. */
typedef struct {
    char name[48];
    int64_t launches;
    double ms;
    double pairs;
    double flops_per_pair;
} sdbie_kernel_stat;
int sdbie_profile_enable(int on);
int sdbie_profile_read(sdbie_kernel_stat* out, int max, int* count);

/* Message describing the last error returned on the calling thread. */
const char* sdbie_last_error(void);

/* Library ABI version (incremented on incompatible changes). */
int sdbie_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SDBIE_H */
