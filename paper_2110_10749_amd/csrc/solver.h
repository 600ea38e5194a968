// Solver context: operators, GMRES, local solves and the interface loop.
#pragma once

#include <functional>
#include <vector>

#include "internal.h"

namespace sdbie {

// work-vector slots of Plan::vec (each 3n doubles)
enum : int {
    kVecV = 0,        // interface unknown v = u.n
    kVecVn,           // next interface iterate
    kVecT0,           // outer GMRES right-hand side
    kVecPl,           // pressure inside the outer operator
    kVecUl,           // velocity inside the outer operator
    kVecDarcyB,       // Darcy right-hand side
    kVecStokesB,      // Stokes right-hand side
    kVecTraction,     // traction f
    kVecRefR,         // refinement residual
    kVecRefC,         // refinement correction
    kVecGmresR,       // inner GMRES residual
    kVecGmresW,       // inner GMRES new Krylov vector
    kVecOuterR,       // outer GMRES residual
    kVecOuterW,       // outer GMRES new vector
    kVecP,            // sorted pressure (entry points)
    kVecU,            // sorted velocity (entry points)
    kVecFx,           // sorted extra traction
    kVecIn,           // sorted input density / misc
    kVecOut,          // sorted output / misc
    kVecCoupledP,     // mixed coupled refinement: pressure iterate
    kVecCoupledU,     // mixed coupled refinement: velocity iterate
    kVecCoupledR1,    // mixed coupled refinement: Darcy residual
    kVecCoupledR2,    // mixed coupled refinement: Stokes residual
    kVecCoupledDP,    // mixed coupled refinement: pressure correction
    kVecCoupledDU,    // mixed coupled refinement: velocity correction
    kVecCoupledV,     // mixed coupled refinement: u.n / projected pressure
    kVecImage,        // interface solve: (p, u, b_D, b_S) combined from the image basis (8n: three slots)
    kVecImage2,
    kVecImage3,
    kVecRecycle,      // device coefficients of the deflation corrections
    kVecSpare,
};
static_assert(kVecSpare < kNumVec, "work-vector slots exceed the workspace");

// device scalar slots of Plan::scal
enum : int {
    kScalCompD = 0,
    kScalCompS = 1,
    kScalMean = 2,
    kScalNorm = 3,
    kScalDrag = 4,   // 3 slots
    kScalStage = 16, // staging: finite flag (16), bounding box (18..23), weight sum (24), near-pair counts (26, 27)
    kScalGmres = 32, // inner and outer Hessenberg columns / coefficients
};

struct GmresWS {
    double* V = nullptr;
    double* r = nullptr;
    double* w = nullptr;
    double* dcol = nullptr;
    double* dy = nullptr;
    // optional image basis: the operator stores what it computed for basis
    // vector k at W2 + k ld2 (Ctx::krylov_index tells it k), and every cycle
    // adds W2 y to x2 with the same coefficients y as V y to x
    double* W2 = nullptr;
    int64_t ld2 = 0;
    double* x2 = nullptr;
};

// Deflation space carried from one local solve to later solves with the same
// operator: the last GMRES cycle's basis V (k + 1 vectors of length ld) and
// its Arnoldi relation A V_k = V_{k+1} H with H = Q R (the cycle's Givens
// rotations and triangle), so that U = V_k R^-1 and C = V_{k+1} Q satisfy
// A U = C with orthonormal C.  exact: the cycle used double products only.
struct Recycle {
    double* V = nullptr;
    int64_t ld = 0;
    int k = 0;
    bool exact = true;
    std::vector<double> cs, sn, R;  // R: k x k upper triangle, row-major
};

struct GmresOut {
    int iters = 0;
    int checks = 0;  // double-pair true residuals after cycles with float-pair products
    double relres = 0.0;
    bool conv = false;
};

struct Ctx {
    Plan& P;
    hipStream_t s;
    const sdbie_opts& o;
    sdbie_info info;
    bool converged = true;
    GmresWS inner, outer;
    // correction mode of the coupled refinement: every pass in float pairs,
    // local solves by plain GMRES to tol_corr
    bool corr = false;
    double tol_corr = 0.0;
    // inexact interface products: local solves to tol_local (0: tol_gmres);
    // loose32: every pass of the local solves (right-hand sides included) in float pairs
    double tol_local = 0.0;
    bool loose32 = false;
    // estimate_only: the relaxed GMRES of a local solve ends on its own
    // residual estimate, without the double-pair true residual (set for the
    // solves whose results only enter an interface product, when the final
    // solves and the true interface residual certify the answer)
    bool estimate_only = false;
    // in_product: the local solves of T(0) and of the interface products under
    // inexact products; the final solves and the true interface residual
    // decide convergence, so a product's local solve that misses its own
    // tolerance only makes the product inexact (and costs correction cycles)
    bool in_product = false;
    // index of the Krylov basis vector the operator is being applied to (-1: a residual)
    int krylov_index = -1;
    // deflation of the Stokes local solves (opts.recycle): rc_cur is set around
    // a solve that may use (or, while empty, fill) the space
    Recycle rc_stokes;
    Recycle* rc_cur = nullptr;

    Ctx(Plan& plan, hipStream_t st, const sdbie_opts& opts);
    void finish();

    double norm(const double* a, int64_t len);
    double dot(const double* a, const double* b, int64_t len);
    void copy(const double* a, double* b, int64_t len);

    void op_darcy(const double* p, double* out, bool mixed);
    void op_stokes(const double* u, double* out, double mu, double beta, bool mixed);
    void single_layer_laplace(const double* g, double scale, double* out, bool mixed);
    void single_layer_stokes(const double* f, double mu, double scale, const double* add, double* out, bool mixed);

    // operator with a precision flag (true: float pairs) and the relative
    // residual estimate of the iteration the product belongs to (0 for true
    // residuals, which need full accuracy)
    using GmresOp = std::function<void(const double*, double*, bool, double)>;
    // r = b - A x in double pairs, from one fused pass (the right-hand side's
    // single layer and the operator's double layer together); replaces the
    // separate right-hand-side pass of a warm-started solve
    using ResidualFn = std::function<void(const double*, double*)>;
    static constexpr double kAllFloat = __builtin_huge_val();
    // with res set, b is not read: residuals come from res, and bnorm (an
    // estimate of ||b|| good to a few digits) scales the tolerance
    GmresOut gmres(const GmresWS& ws, const GmresOp& op, const double* b, double* x, int64_t L, bool x_nonzero,
                   double tol, int restart, int maxit, double relax = 0.0, const ResidualFn* res = nullptr,
                   double bnorm = 0.0);
    void solve(const std::function<void(const double*, double*, bool)>& op, const double* b, double* x, int64_t L,
               bool x_nonzero, double* rbuf, double* cbuf, const ResidualFn* res = nullptr, double bnorm = 0.0);

    // v_zero: v is known to be zero (then, without an extra right-hand side,
    // b = 0 and its single-layer pass is skipped).  bnorm > 0 (with a warm
    // start p, no extra right-hand side): an estimate of ||b||; the residuals
    // then come from one fused pass each and b itself is never formed
    void darcy(const sdbie_params& prm, const double* v, double* p, bool p_nonzero, const double* extra_rhs,
               bool remove_mean = true, bool v_zero = false, double bnorm = 0.0);
    // p_zero: p is known to be zero (then, without fx or lagged slip, the
    // right-hand side is U itself and its single-layer pass is skipped).
    // bnorm: as for darcy()
    void stokes(const sdbie_params& prm, const double U[3], const double* p, const double* fx, double* u,
                bool u_nonzero, const double* extra_rhs, bool p_zero = false, double bnorm = 0.0);
    bool fused_residuals_ok(bool warm, const double* extra_rhs, double bnorm) const;
    void ddm(const sdbie_params& prm, const double U[3], const double* fx, double* p, double* u, double drag[3]);
    void ddm_outer(const sdbie_params& prm, const double U[3], const double* fx, const double* r1, const double* r2,
                   double* p, double* u, bool remove_mean, double tol);
    void coupled_residual(const sdbie_params& prm, const double U[3], const double* fx, const double* pt,
                          const double* u, double* r1, double* r2);
    void project_mean(const double* p, double* out);
    void ddm_refined(const sdbie_params& prm, const double U[3], const double* fx, double* p, double* u);
    void adjoint(const sdbie_params& prm, const double U[3], const double* fx, const double* p, const double* u,
                 const double e[3], double* grad, double* dlogK, double* dalpha);
    void compute_drag(const sdbie_params& prm, const double* p, const double* u, const double* fx, double drag[3]);
    // Arnoldi on the linear D-N map (spectrum.hip)
    int dn_arnoldi(const sdbie_params& prm, const double* v0, int m, std::vector<double>& H);
};

}  // namespace sdbie
