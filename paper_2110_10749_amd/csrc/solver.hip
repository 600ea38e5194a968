// Local solves and the Dirichlet-Neumann interface loop, on sorted device vectors.
//
// Operators (paper, sections "Boundary integral formulations" and
// "High-order regularization of kernels on the surface"), with the rank-one
// completions that remove the null vectors of the subtracted forms:
//   Darcy:   Abar_D p = A_D p + (sum_j w_j p_j / |S|) 1
//   Stokes:  Abar_S u = A_S u + (sum_j w_j n_j.u_j / |S|) n   [+ V[beta P_tau u]]
// Krylov solver: restarted GMRES, classical Gram-Schmidt with one
// re-orthogonalisation (CGS2) on the device, Hessenberg column and Givens
// rotations on the host (one device->host copy per iteration), all in double.
// Mixed precision: the solve is wrapped in iterative refinement
//   r = b - A64 x  (double pairs),  A32 c = r by GMRES (float pairs), x += c.
#include <cmath>
#include <cstring>
#include <vector>

#include "solver.h"

namespace sdbie {

namespace {
constexpr double kPi = 3.14159265358979323846;
}

// ------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------
double Ctx::norm(const double* a, int64_t len) {
    dev_dot(P, a, a, len, P.scal + kScalNorm, s);
    const double v = host_read_scalar(P.scal + kScalNorm, s);
    if (!std::isfinite(v)) throw Error(SDBIE_ERR_NONFINITE, "non-finite iterate");
    return std::sqrt(v);
}

double Ctx::dot(const double* a, const double* b, int64_t len) {
    dev_dot(P, a, b, len, P.scal + kScalNorm, s);
    return host_read_scalar(P.scal + kScalNorm, s);
}

void Ctx::copy(const double* a, double* b, int64_t len) {
    SDBIE_HIP(hipMemcpyAsync(b, a, len * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// ------------------------------------------------------------------------------
// operators
// ------------------------------------------------------------------------------
void Ctx::op_darcy(const double* p, double* out, bool mixed) {
    dev_dot(P, P.w, p, P.n, P.scal + kScalCompD, s);
    PassDesc d;
    d.dl = true;
    d.sub = true;
    d.c_dl = 1.0 / (4.0 * kPi);
    d.dl_dens = p;
    d.comp = P.scal + kScalCompD;
    d.comp_scale = 1.0 / P.area;
    d.out = out;
    d.mixed = mixed;
    launch_laplace_pass(P, d, s);
}

void Ctx::op_stokes(const double* u, double* out, double mu, double beta, bool mixed) {
    dev_dot(P, P.wn, u, 3 * P.n, P.scal + kScalCompS, s);
    PassDesc d;
    d.dl = true;
    d.sub = true;
    d.c_dl = -3.0 / (4.0 * kPi);
    d.dl_dens = u;
    d.base = u;
    d.base_scale = 1.0;
    if (beta != 0.0) {
        d.sl = true;
        d.c_sl = 1.0 / (8.0 * kPi * mu);
        d.slip_beta = beta;
        d.sl_dens = nullptr;
    }
    d.comp = P.scal + kScalCompS;
    d.comp_scale = 1.0 / P.area;
    d.out = out;
    d.mixed = mixed;
    launch_stokes_pass(P, d, s);
}

// out = scale * S_L[g] (+ base)
void Ctx::single_layer_laplace(const double* g, double scale, double* out, bool mixed) {
    PassDesc d;
    d.sl = true;
    d.c_sl = -scale / (4.0 * kPi);
    d.sl_dens = g;
    d.out = out;
    d.mixed = mixed;
    launch_laplace_pass(P, d, s);
}

// out = add + scale * V[f]
void Ctx::single_layer_stokes(const double* f, double mu, double scale, const double* add, double* out, bool mixed) {
    PassDesc d;
    d.sl = true;
    d.c_sl = scale / (8.0 * kPi * mu);
    d.sl_dens = f;
    d.add_const = add;
    d.out = out;
    d.mixed = mixed;
    launch_stokes_pass(P, d, s);
}

// ------------------------------------------------------------------------------
// GMRES
// ------------------------------------------------------------------------------
GmresOut Ctx::gmres(const GmresWS& ws, const std::function<void(const double*, double*)>& op, const double* b,
                    double* x, int64_t L, bool x_nonzero, double tol, int restart, int maxit) {
    GmresOut res;
    const double bnorm = norm(b, L);
    if (bnorm == 0.0) {
        dev_fill(0.0, x, L, s);
        res.conv = true;
        return res;
    }
    double* r = ws.r;
    double* w = ws.w;
    if (x_nonzero) {
        op(x, r);
        dev_axpby(1.0, b, -1.0, r, r, L, s);
    } else {
        dev_fill(0.0, x, L, s);
        copy(b, r, L);
    }
    double beta = norm(r, L);
    res.relres = beta / bnorm;
    const int m = restart;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), e(m + 1), col(2 * (m + 1) + 1), y(m);
    auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    while (res.relres > tol && res.iters < maxit) {
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(e.begin(), e.end(), 0.0);
        e[0] = beta;
        dev_scale(1.0 / beta, r, ws.V, L, s);
        int k_used = 0;
        for (int k = 0; k < m; ++k) {
            double* vk = ws.V + (int64_t)k * L;
            op(vk, w);
            res.iters++;
            double* h1 = ws.dcol;
            double* h2 = ws.dcol + (k + 1);
            double* hn = ws.dcol + 2 * (k + 1);
            dev_multidot(P, ws.V, L, k + 1, w, L, h1, s);
            dev_multi_axpy_sub(ws.V, L, k + 1, h1, w, L, s);
            dev_multidot(P, ws.V, L, k + 1, w, L, h2, s);
            dev_multi_axpy_sub(ws.V, L, k + 1, h2, w, L, s);
            dev_dot(P, w, w, L, hn, s);
            SDBIE_HIP(hipMemcpyAsync(col.data(), ws.dcol, (2 * (k + 1) + 1) * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
            SDBIE_HIP(hipStreamSynchronize(s));
            for (int j = 0; j <= k; ++j) Hat(j, k) = col[j] + col[k + 1 + j];
            const double hk1 = std::sqrt(col[2 * (k + 1)]);
            if (!std::isfinite(hk1)) throw Error(SDBIE_ERR_NONFINITE, "non-finite Krylov vector");
            Hat(k + 1, k) = hk1;
            if (hk1 > 0.0 && k + 1 < m + 1) dev_scale(1.0 / hk1, w, ws.V + (int64_t)(k + 1) * L, L, s);
            for (int j = 0; j < k; ++j) {
                const double t = cs[j] * Hat(j, k) + sn[j] * Hat(j + 1, k);
                Hat(j + 1, k) = -sn[j] * Hat(j, k) + cs[j] * Hat(j + 1, k);
                Hat(j, k) = t;
            }
            const double den = std::hypot(Hat(k, k), Hat(k + 1, k));
            cs[k] = Hat(k, k) / den;
            sn[k] = Hat(k + 1, k) / den;
            Hat(k, k) = den;
            Hat(k + 1, k) = 0.0;
            e[k + 1] = -sn[k] * e[k];
            e[k] = cs[k] * e[k];
            k_used = k + 1;
            res.relres = std::fabs(e[k + 1]) / bnorm;
            if (res.relres <= tol || res.iters >= maxit || hk1 == 0.0) break;
        }
        // back substitution H y = e on the k_used x k_used triangle
        for (int i = k_used - 1; i >= 0; --i) {
            double t = e[i];
            for (int j = i + 1; j < k_used; ++j) t -= Hat(i, j) * y[j];
            y[i] = t / Hat(i, i);
        }
        SDBIE_HIP(hipMemcpyAsync(ws.dy, y.data(), k_used * sizeof(double), hipMemcpyHostToDevice, s));
        dev_multi_axpy_add(ws.V, L, k_used, ws.dy, x, L, s);
        if (res.relres <= tol || res.iters >= maxit) break;
        // restart from the true residual
        op(x, r);
        dev_axpby(1.0, b, -1.0, r, r, L, s);
        beta = norm(r, L);
        res.relres = beta / bnorm;
    }
    res.conv = res.relres <= tol;
    SDBIE_HIP(hipStreamSynchronize(s));
    return res;
}

// Solve A x = b: plain GMRES with the double-pair operator, or iterative
// refinement (double residual, float-pair correction solves).
void Ctx::solve(const std::function<void(const double*, double*, bool)>& op, const double* b, double* x,
                int64_t L, bool x_nonzero, double* rbuf, double* cbuf) {
    const bool mixed = o.prec == SDBIE_MIXED;
    if (!mixed) {
        GmresOut g = gmres(inner, [&](const double* in, double* out) { op(in, out, false); }, b, x, L, x_nonzero,
                           o.tol_gmres, o.restart, o.maxit_gmres);
        info.gmres_iters += g.iters;
        info.relres = g.relres;
        if (!g.conv) converged = false;
        return;
    }
    const double bnorm = norm(b, L);
    if (bnorm == 0.0) {
        dev_fill(0.0, x, L, s);
        info.relres = 0.0;
        return;
    }
    bool have_x = x_nonzero;
    int step = 0;
    double rel = 1.0;
    for (;; ++step) {
        if (have_x) {
            op(x, rbuf, false);
            dev_axpby(1.0, b, -1.0, rbuf, rbuf, L, s);
        } else {
            copy(b, rbuf, L);
        }
        rel = norm(rbuf, L) / bnorm;
        if (rel <= o.tol_gmres || step >= o.refine_max) break;
        const double tol_c = std::max(o.tol_mixed, 0.5 * o.tol_gmres / rel);
        GmresOut g = gmres(inner, [&](const double* in, double* out) { op(in, out, true); }, rbuf, cbuf, L, false,
                           tol_c, o.restart, o.maxit_gmres);
        info.gmres_iters += g.iters;
        if (have_x) {
            dev_axpby(1.0, x, 1.0, cbuf, x, L, s);
        } else {
            copy(cbuf, x, L);
            have_x = true;
        }
    }
    info.refine_steps += step;
    info.relres = rel;
    if (rel > o.tol_gmres) converged = false;
}

// ------------------------------------------------------------------------------
// local problems
// ------------------------------------------------------------------------------
void Ctx::darcy(const sdbie_params& prm, const double* v, double* p, bool p_nonzero, const double* extra_rhs) {
    const int64_t n = P.n;
    double* b = P.vec(kVecDarcyB);
    // b = -S_L[g], g = dp/dn = -(mu/K) v   =>  b = (mu/K) S_L[v]
    single_layer_laplace(v, prm.mu / prm.K, b, false);
    if (extra_rhs) dev_axpby(1.0, b, 1.0, extra_rhs, b, n, s);
    solve([&](const double* in, double* out, bool mx) { op_darcy(in, out, mx); }, b, p, n, p_nonzero,
          P.vec(kVecRefR), P.vec(kVecRefC));
    // remove the weighted mean
    dev_dot(P, P.w, p, n, P.scal + kScalMean, s);
    dev_add_scaled_scalar(p, P.scal + kScalMean, -1.0 / P.area, n, s);
}

void Ctx::stokes(const sdbie_params& prm, const double U[3], const double* p, const double* fx, double* u,
                 bool u_nonzero, const double* extra_rhs) {
    const int64_t n = P.n;
    const double beta = prm.alpha * prm.mu / std::sqrt(prm.K);
    double* f = P.vec(kVecTraction);
    double* rhs = P.vec(kVecStokesB);
    const bool lagged = o.slip == 1 && beta != 0.0;
    // traction without the implicit slip term (lagged slip uses the entry u)
    dev_traction(P, p, lagged ? u : nullptr, lagged ? beta : 0.0, fx, f, s);
    single_layer_stokes(f, prm.mu, -1.0, U, rhs, false);
    if (extra_rhs) dev_axpby(1.0, rhs, 1.0, extra_rhs, rhs, 3 * n, s);
    const double b_impl = lagged ? 0.0 : beta;
    solve([&](const double* in, double* out, bool mx) { op_stokes(in, out, prm.mu, b_impl, mx); }, rhs, u, 3 * n,
          u_nonzero, P.vec(kVecRefR), P.vec(kVecRefC));
}

// ------------------------------------------------------------------------------
// Dirichlet-Neumann loop
// ------------------------------------------------------------------------------
void Ctx::ddm(const sdbie_params& prm, const double U[3], const double* fx, double* p, double* u, double drag[3]) {
    const int64_t n = P.n;
    double* v = P.vec(kVecV);
    double* vn = P.vec(kVecVn);
    if (o.outer == 0) {
        dev_fill(0.0, v, n, s);
        dev_fill(0.0, p, n, s);
        dev_fill(0.0, u, 3 * n, s);
        bool first = true;
        for (int k = 1; k <= o.maxit_ddm; ++k) {
            darcy(prm, v, p, !first, nullptr);
            stokes(prm, U, p, fx, u, !first, nullptr);
            first = false;
            dev_normal_component(P, u, vn, s);
            dev_axpby(1.0 - o.theta, v, o.theta, vn, vn, n, s);
            dev_axpby(1.0, vn, -1.0, v, v, n, s);  // v <- vn - v (difference)
            const double dn = norm(v, n);
            const double nv = norm(vn, n);
            copy(vn, v, n);
            info.ddm_iters = k;
            info.ddm_res = nv > 0.0 ? dn / nv : 0.0;
            if (info.ddm_res < o.tol_ddm) break;
        }
        if (!(info.ddm_res < o.tol_ddm)) converged = false;
    } else {
        const double zero[3] = {0.0, 0.0, 0.0};
        double* t0 = P.vec(kVecT0);
        double* pl = P.vec(kVecPl);
        double* ul = P.vec(kVecUl);
        // t0 = T(0): Stokes with p = 0
        dev_fill(0.0, pl, n, s);
        stokes(prm, U, pl, fx, ul, false, nullptr);
        dev_normal_component(P, ul, t0, s);
        auto op = [&](const double* y, double* out) {
            darcy(prm, y, pl, false, nullptr);
            stokes(prm, zero, pl, nullptr, ul, false, nullptr);
            dev_normal_component(P, ul, out, s);
            dev_axpby(1.0, y, -1.0, out, out, n, s);
        };
        GmresOut g = gmres(outer, op, t0, v, n, false, o.tol_ddm, o.restart, o.maxit_ddm);
        info.ddm_iters = g.iters;
        info.ddm_res = g.relres;
        if (!g.conv) converged = false;
        darcy(prm, v, p, false, nullptr);
        stokes(prm, U, p, fx, u, false, nullptr);
    }
    compute_drag(prm, p, u, fx, drag);
}

void Ctx::compute_drag(const sdbie_params& prm, const double* p, const double* u, const double* fx, double drag[3]) {
    const int64_t n = P.n;
    const double beta = prm.alpha * prm.mu / std::sqrt(prm.K);
    double* f = P.vec(kVecTraction);
    dev_traction(P, p, u, beta, fx, f, s);
    for (int c = 0; c < 3; ++c) dev_dot(P, P.w, f + c * n, n, P.scal + kScalDrag + c, s);
    double h[3];
    SDBIE_HIP(hipMemcpyAsync(h, P.scal + kScalDrag, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    SDBIE_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < 3; ++c) drag[c] = h[c];
}

Ctx::Ctx(Plan& plan, hipStream_t st, const sdbie_opts& opts) : P(plan), s(st), o(opts) {
    std::memset(&info, 0, sizeof(info));
    const int m = P.max_restart;
    inner.V = P.basis_in;
    inner.r = P.vec(kVecGmresR);
    inner.w = P.vec(kVecGmresW);
    inner.dcol = P.scal + kScalGmres;
    inner.dy = P.scal + kScalGmres + 2 * (m + 1) + 1;
    outer.V = P.basis_out;
    outer.r = P.vec(kVecOuterR);
    outer.w = P.vec(kVecOuterW);
    outer.dcol = P.scal + kScalGmres + 3 * (m + 2);
    outer.dy = P.scal + kScalGmres + 3 * (m + 2) + 2 * (m + 1) + 1;
    P.applies_fp64 = P.applies_mixed = 0;
    P.pairs = 0.0;
}

void Ctx::finish() {
    info.applies_fp64 = P.applies_fp64;
    info.applies_mixed = P.applies_mixed;
    info.pairs = P.pairs;
}

}  // namespace sdbie
