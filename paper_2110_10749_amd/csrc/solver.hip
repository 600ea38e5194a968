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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "solver.h"

namespace sdbie {

namespace {
constexpr double kPi = 3.14159265358979323846;

// SDBIE_DEBUG=1 prints solver progress to stderr
int debug_level() {
    static const int lvl = [] {
        const char* e = std::getenv("SDBIE_DEBUG");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}
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
// The operator takes a precision flag (true: float pairs).  relax = 0: every
// product in double pairs; relax = inf: every product in float pairs; else
// the Arnoldi products switch to float pairs once the residual estimate is
// at or below relax * ||b|| (relaxed inexact Krylov: the product error may
// grow as the residual shrinks), and a cycle that used float pairs ends with
// a double-pair true residual, which alone decides convergence (unless
// estimate_only is set: then the estimate decides, as in double GMRES).
GmresOut Ctx::gmres(const GmresWS& ws, const GmresOp& op, const double* b, double* x, int64_t L, bool x_nonzero,
                    double tol, int restart, int maxit, double relax, const ResidualFn* resfn, double bnorm_in) {
    GmresOut res;
    const double bnorm = resfn ? bnorm_in : norm(b, L);
    if (bnorm == 0.0) {
        dev_fill(0.0, x, L, s);
        res.conv = true;
        return res;
    }
    double* r = ws.r;
    double* w = ws.w;
    const bool all32 = std::isinf(relax);
    if (resfn && !all32) {
        if (!x_nonzero) dev_fill(0.0, x, L, s);
        krylov_index = -1;
        (*resfn)(x, r);
    } else if (x_nonzero) {
        krylov_index = -1;
        op(x, r, all32, 0.0);
        dev_axpby(1.0, b, -1.0, r, r, L, s);
    } else {
        dev_fill(0.0, x, L, s);
        copy(b, r, L);
    }
    const int m = restart;
    // deflation (Recycle): rc_use deflates this solve; rc_fill receives its last cycle
    // only a space from a cycle of double products (A U = C to double accuracy)
    Recycle* rc_use = rc_cur && rc_cur->k > 0 && rc_cur->ld == L && rc_cur->exact ? rc_cur : nullptr;
    Recycle* rc_fill = rc_cur && rc_cur->k == 0 ? rc_cur : nullptr;
    const int kr = rc_use ? rc_use->k : 0;
    std::vector<double> rh(kr + 1), rz(kr), Ecol((size_t)kr * m), G(kr + 1), SG(kr);
    // device coefficients of the two corrections (distinct regions of a work vector;
    // every reuse is preceded by a stream synchronisation)
    double* dG = P.vec(kVecRecycle);
    double* dSG = dG + kr + 1;
    // e = C^T w = Q^T V^T w (kr values in rh); then w -= C e = V (Q e)
    auto project_off = [&](double* wv) {
        dev_multidot(P, rc_use->V, L, kr + 1, wv, L, ws.dcol, s);
        SDBIE_HIP(hipMemcpyAsync(rh.data(), ws.dcol, (kr + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        SDBIE_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < kr; ++j) {
            const double t = rc_use->cs[j] * rh[j] + rc_use->sn[j] * rh[j + 1];
            rh[j + 1] = -rc_use->sn[j] * rh[j] + rc_use->cs[j] * rh[j + 1];
            rh[j] = t;
        }
        std::copy(rh.begin(), rh.begin() + kr, G.begin());
        G[kr] = 0.0;
        for (int j = kr - 1; j >= 0; --j) {
            const double t = rc_use->cs[j] * G[j] - rc_use->sn[j] * G[j + 1];
            G[j + 1] = rc_use->sn[j] * G[j] + rc_use->cs[j] * G[j + 1];
            G[j] = t;
        }
        SDBIE_HIP(hipMemcpyAsync(dG, G.data(), (kr + 1) * sizeof(double), hipMemcpyHostToDevice, s));
        dev_multi_axpy_sub(rc_use->V, L, kr + 1, dG, wv, L, s);
    };
    // x += sign U z with U = V_k R^-1: solve R t = z, x += sign V_k t
    auto add_U = [&](const double* z, double sign, double* xv) {
        for (int i = kr - 1; i >= 0; --i) {
            double t = z[i];
            for (int j = i + 1; j < kr; ++j) t -= rc_use->R[(size_t)i * kr + j] * rz[j];
            rz[i] = t / rc_use->R[(size_t)i * kr + i];
        }
        for (int i = 0; i < kr; ++i) SG[i] = sign * rz[i];
        SDBIE_HIP(hipMemcpyAsync(dSG, SG.data(), kr * sizeof(double), hipMemcpyHostToDevice, s));
        dev_multi_axpy_add(rc_use->V, L, kr, dSG, xv, L, s);
    };
    auto deflate_residual = [&]() {  // x += U C^T r, r -= C C^T r
        project_off(r);
        add_U(rh.data(), 1.0, x);
    };
    if (rc_use) deflate_residual();
    double beta = norm(r, L);
    res.relres = beta / bnorm;
    const double rel0 = res.relres;
    int n64 = 0;  // products with double pairs (diagnostics)
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), e(m + 1), col(2 * (m + 1) + 1), y(m);
    auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    int last_k = 0;
    bool last32 = false;
    while (res.relres > tol && res.iters < maxit) {
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(e.begin(), e.end(), 0.0);
        e[0] = beta;
        dev_scale(1.0 / beta, r, ws.V, L, s);
        int k_used = 0;
        bool cycle32 = false;
        for (int k = 0; k < m; ++k) {
            double* vk = ws.V + (int64_t)k * L;
            const bool m32 = all32 || res.relres <= relax;
            cycle32 = cycle32 || m32;
            n64 += !m32;
            krylov_index = k;
            op(vk, w, m32, res.relres);
            krylov_index = -1;
            res.iters++;
            if (rc_use) {
                project_off(w);
                std::copy(rh.begin(), rh.begin() + kr, Ecol.begin() + (size_t)k * kr);
            }
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
        if (ws.W2) dev_multi_axpy_add(ws.W2, ws.ld2, k_used, ws.dy, ws.x2, ws.ld2, s);
        if (rc_use) {
            // A (V y - U E y) = V_{m+1} H y: x -= U (E y)
            std::vector<double> ey(kr, 0.0);
            for (int j = 0; j < k_used; ++j)
                for (int i = 0; i < kr; ++i) ey[i] += Ecol[(size_t)j * kr + i] * y[j];
            add_U(ey.data(), -1.0, x);
        }
        last_k = k_used;
        last32 = cycle32;
        const bool verify = cycle32 && !all32 && !estimate_only;
        if (!verify && (res.relres <= tol || res.iters >= maxit)) break;
        // restart from (or verify with) the true residual
        krylov_index = -1;
        if (resfn && !all32) {
            (*resfn)(x, r);
        } else {
            op(x, r, all32, 0.0);
            dev_axpby(1.0, b, -1.0, r, r, L, s);
        }
        beta = norm(r, L);
        res.relres = beta / bnorm;
        if (verify) res.checks++;
        if (rc_use && res.relres > tol && res.iters < maxit) {
            deflate_residual();
            beta = norm(r, L);
            res.relres = beta / bnorm;
        }
    }
    if (rc_fill && last_k > 0) {
        // keep this solve's last cycle: V_0 .. V_k and the rotated Hessenberg
        SDBIE_HIP(hipMemcpyAsync(rc_fill->V, ws.V, (size_t)(last_k + 1) * L * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
        rc_fill->ld = L;
        rc_fill->k = last_k;
        rc_fill->exact = !last32;
        rc_fill->cs.assign(cs.begin(), cs.begin() + last_k);
        rc_fill->sn.assign(sn.begin(), sn.begin() + last_k);
        rc_fill->R.assign((size_t)last_k * last_k, 0.0);
        for (int i = 0; i < last_k; ++i)
            for (int j = i; j < last_k; ++j) rc_fill->R[(size_t)i * last_k + j] = Hat(i, j);
    }
    res.conv = res.relres <= tol;
    SDBIE_HIP(hipStreamSynchronize(s));
    if (debug_level() > 1)
        std::fprintf(stderr, "[sdbie] gmres L=%lld start %.1e iters=%d (double pairs %d) relres=%.3e tol=%.1e\n",
                     (long long)L, rel0, res.iters, n64, res.relres, tol);
    return res;
}

// Solve A x = b: plain GMRES with the double-pair operator, or iterative
// refinement (double residual, float-pair correction solves).
void Ctx::solve(const std::function<void(const double*, double*, bool)>& op3, const double* b, double* x,
                int64_t L, bool x_nonzero, double* rbuf, double* cbuf, const ResidualFn* resfn, double bnorm) {
    const GmresOp op = [&](const double* in, double* out, bool m32, double) { op3(in, out, m32); };
    if (corr) {
        const bool m32 = debug_level() < 10;  // SDBIE_DEBUG >= 10: double-pair corrections (diagnostics)
        GmresOut g = gmres(inner, op, b, x, L, x_nonzero, tol_corr, o.restart, o.maxit_gmres,
                           m32 ? kAllFloat : 0.0);
        info.gmres_iters += g.iters;
        return;
    }
    const double tol = tol_local > 0.0 ? tol_local : o.tol_gmres;
    if (resfn && (o.local_solver == 1 || loose32 || (o.prec == SDBIE_MIXED && o.mixed_mode != 2)))
        throw Error(SDBIE_ERR_ARG, "internal: a fused residual needs the GMRES local solver");
    if (o.local_solver == 1) {
        // successive approximations (eqs. Darcy_BIEM_iter, Stokes_BIEM_iter)
        // on the completed operator: x <- x + (b - A x) until the relative
        // change is at most tol; double pairs
        if (!x_nonzero) dev_fill(0.0, x, L, s);
        double ch = 0.0;
        int m = 0;
        while (m < o.maxit_gmres) {
            ++m;
            op3(x, rbuf, false);
            dev_axpby(1.0, b, -1.0, rbuf, rbuf, L, s);  // the change b - A x
            const double dn = norm(rbuf, L);
            dev_axpby(1.0, x, 1.0, rbuf, x, L, s);
            const double xn = norm(x, L);
            ch = xn > 0.0 ? dn / xn : 0.0;
            if (!std::isfinite(ch)) throw Error(SDBIE_ERR_NONFINITE, "successive approximations diverged");
            if (ch <= tol) break;
        }
        info.gmres_iters += m;
        info.relres = ch;
        if (ch > tol && !in_product) converged = false;
        return;
    }
    if (loose32) {
        // a loose inexact interface product: float pairs throughout, no double check
        GmresOut g = gmres(inner, op, b, x, L, x_nonzero, tol, o.restart, o.maxit_gmres, kAllFloat);
        info.gmres_iters += g.iters;
        return;
    }
    const bool mixed = o.prec == SDBIE_MIXED;
    if (!mixed || o.mixed_mode == 2) {
        // double pairs, or relaxed: double pairs until the residual reaches
        // the switch point, float pairs below it, double-pair true residual at
        // the end.  The error a product may carry grows with the tolerance
        // sought, so a looser local solve switches earlier: at tol_mixed for
        // tol_gmres, in proportion above it.
        const double relax = mixed ? std::min(1.0, o.tol_mixed * (tol / o.tol_gmres)) : 0.0;
        GmresOut g = gmres(inner, op, b, x, L, x_nonzero, tol, o.restart, o.maxit_gmres, relax, resfn, bnorm);
        if (mixed) info.refine_steps += g.checks;
        info.gmres_iters += g.iters;
        info.relres = g.relres;
        if (!g.conv && !in_product) converged = false;
        return;
    }
    const double b_norm = norm(b, L);
    if (b_norm == 0.0) {
        dev_fill(0.0, x, L, s);
        info.relres = 0.0;
        return;
    }
    // every step starts from a double-pair residual, and that residual alone
    // decides convergence (and is what info.relres reports)
    bool have_x = x_nonzero;
    int step = 0;
    double rel = 1.0;
    for (;; ++step) {
        if (have_x) {
            op3(x, rbuf, false);
            dev_axpby(1.0, b, -1.0, rbuf, rbuf, L, s);
        } else {
            copy(b, rbuf, L);
        }
        rel = norm(rbuf, L) / b_norm;
        if (rel <= tol || step >= o.refine_max) break;
        GmresOut g = gmres(inner, op, rbuf, cbuf, L, false, o.tol_mixed, o.restart, o.maxit_gmres, kAllFloat);
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
    if (rel > tol && !in_product) converged = false;
}

// ------------------------------------------------------------------------------
// local problems
// ------------------------------------------------------------------------------
// whether a warm-started local solve may take its residuals from fused passes
bool Ctx::fused_residuals_ok(bool warm, const double* extra_rhs, double bnorm) const {
    return warm && bnorm > 0.0 && !extra_rhs && !corr && !loose32 && o.local_solver == 0 &&
           (o.prec != SDBIE_MIXED || o.mixed_mode == 2);
}

void Ctx::darcy(const sdbie_params& prm, const double* v, double* p, bool p_nonzero, const double* extra_rhs,
                bool remove_mean, bool v_zero, double bnorm) {
    const int64_t n = P.n;
    double* b = P.vec(kVecDarcyB);
    const auto op = [&](const double* in, double* out, bool mx) { op_darcy(in, out, mx); };
    if (!v_zero && fused_residuals_ok(p_nonzero, extra_rhs, bnorm)) {
        // r = (mu/K) S_L[v] - Abar_D x: the single and subtracted double layer in one pass
        const ResidualFn res = [&](const double* xv, double* r) {
            dev_dot(P, P.w, xv, n, P.scal + kScalCompD, s);
            PassDesc d;
            d.dl = true;
            d.sub = true;
            d.c_dl = -1.0 / (4.0 * kPi);
            d.dl_dens = xv;
            d.sl = true;
            d.c_sl = -(prm.mu / prm.K) / (4.0 * kPi);
            d.sl_dens = v;
            d.comp = P.scal + kScalCompD;
            d.comp_scale = -1.0 / P.area;
            d.out = r;
            launch_laplace_pass(P, d, s);
        };
        solve(op, nullptr, p, n, true, P.vec(kVecRefR), P.vec(kVecRefC), &res, bnorm);
    } else {
        // b = -S_L[g], g = dp/dn = -(mu/K) v   =>  b = (mu/K) S_L[v]
        if (v_zero) dev_fill(0.0, b, n, s);
        else single_layer_laplace(v, prm.mu / prm.K, b, (corr && debug_level() < 10) || loose32);
        if (extra_rhs) dev_axpby(1.0, b, 1.0, extra_rhs, b, n, s);
        solve(op, b, p, n, p_nonzero, P.vec(kVecRefR), P.vec(kVecRefC));
    }
    if (remove_mean) {
        dev_dot(P, P.w, p, n, P.scal + kScalMean, s);
        dev_add_scaled_scalar(p, P.scal + kScalMean, -1.0 / P.area, n, s);
    }
}

void Ctx::stokes(const sdbie_params& prm, const double U[3], const double* p, const double* fx, double* u,
                 bool u_nonzero, const double* extra_rhs, bool p_zero, double bnorm) {
    const int64_t n = P.n;
    const double beta = prm.alpha * prm.mu / std::sqrt(prm.K);
    double* f = P.vec(kVecTraction);
    double* rhs = P.vec(kVecStokesB);
    const bool lagged = o.slip == 1 && beta != 0.0;
    if (!lagged && fused_residuals_ok(u_nonzero, extra_rhs, bnorm)) {
        // r = U - V[-p n + beta P_tau x + fx] - Abar_S x: the traction's single layer
        // and the subtracted stresslet in one pass
        const ResidualFn res = [&](const double* xv, double* r) {
            dev_traction(P, p, xv, beta, fx, f, s);
            dev_dot(P, P.wn, xv, 3 * n, P.scal + kScalCompS, s);
            PassDesc d;
            d.dl = true;
            d.sub = true;
            d.c_dl = 3.0 / (4.0 * kPi);
            d.dl_dens = xv;
            d.base = xv;
            d.base_scale = -1.0;
            d.sl = true;
            d.c_sl = -1.0 / (8.0 * kPi * prm.mu);
            d.sl_dens = f;
            d.comp = P.scal + kScalCompS;
            d.comp_scale = -1.0 / P.area;
            d.add_const = U;
            d.out = r;
            launch_stokes_pass(P, d, s);
        };
        Recycle* saved = rc_cur;
        if (o.recycle && !corr && o.prec == SDBIE_FP64) rc_cur = &rc_stokes;
        solve([&](const double* in, double* out, bool mx) { op_stokes(in, out, prm.mu, beta, mx); }, nullptr, u,
              3 * n, true, P.vec(kVecRefR), P.vec(kVecRefC), &res, bnorm);
        rc_cur = saved;
        return;
    }
    if (p_zero && !fx && !lagged) {
        // zero traction: V[f] = 0, so the right-hand side is the uniform U
        for (int c = 0; c < 3; ++c) dev_fill(U[c], rhs + c * n, n, s);
    } else {
        // traction without the implicit slip term (lagged slip uses the entry u)
        dev_traction(P, p, lagged ? u : nullptr, lagged ? beta : 0.0, fx, f, s);
        single_layer_stokes(f, prm.mu, -1.0, U, rhs, (corr && debug_level() < 10) || loose32);
    }
    if (extra_rhs) dev_axpby(1.0, rhs, 1.0, extra_rhs, rhs, 3 * n, s);
    const double b_impl = lagged ? 0.0 : beta;
    // every Stokes solve of one call has the same operator: the first fills the
    // deflation space, the later ones use it.  Double pairs only: with float
    // products the deflated operator and the space disagree at float level
    // and hard cases stall (sphere, h = 1/32, beta = 100: 1.5-2.5x the
    // iterations, against 0.71x in double)
    Recycle* saved = rc_cur;
    if (o.recycle && o.local_solver == 0 && !corr && o.prec == SDBIE_FP64) rc_cur = &rc_stokes;
    solve([&](const double* in, double* out, bool mx) { op_stokes(in, out, prm.mu, b_impl, mx); }, rhs, u, 3 * n,
          u_nonzero, P.vec(kVecRefR), P.vec(kVecRefC));
    rc_cur = saved;
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
            darcy(prm, v, p, !first, nullptr, true, first);           // first: v = 0
            stokes(prm, U, p, fx, u, !first, nullptr, first);  // first: v = 0, hence p = 0
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
    } else if (o.prec == SDBIE_MIXED && o.mixed_mode == 1) {
        ddm_refined(prm, U, fx, p, u);
    } else {
        ddm_outer(prm, U, fx, nullptr, nullptr, p, u, true, o.tol_ddm);
    }
    compute_drag(prm, p, u, fx, drag);
}

// Interface GMRES: the D-N map T(v) = u(p(v)).n is affine in v; solve
// (I - T_lin) v = T(0) and finish with one more Darcy and Stokes solve.
// r1, r2 (nullable) are extra right-hand sides of the Darcy and Stokes
// equations (used by the coupled refinement).
//
// Inexact products (relax_outer, not in the coupled refinement): a Krylov
// product taken when the interface residual estimate is rr ||T(0)|| only needs
// an error of order tol ||T(0)|| / rr, so its local solves run to
// clamp(kOuterSafety tol / rr, tol_gmres, kOuterLoosest), and with float
// pairs throughout once that is at least kLooseFloat.  The final solves are
// full-accuracy; their u.n - v is the true interface residual, and a cycle
// on the correction equation (I - T_lin) d = u.n - v follows when it is
// above tol.  The safety factor stands for the conditioning of the interface
// operator, which the residual bound needs and nothing here knows in
// advance: when a cycle ends with a true residual F times the one its GMRES
// predicted, the products were about F times too inexact, and the next cycle
// runs its local solves with the safety factor divided by F.
namespace {
constexpr double kOuterSafety = 1e-3;
constexpr double kOuterLoosest = 1e-2;
constexpr double kLooseFloat = 1e-5;  // float-pair operator error is ~1e-7 relative
constexpr int kOuterCycles = 4;
}  // namespace

void Ctx::ddm_outer(const sdbie_params& prm, const double U[3], const double* fx, const double* r1, const double* r2,
                    double* p, double* u, bool remove_mean, double tol) {
    const int64_t n = P.n;
    const double zero[3] = {0.0, 0.0, 0.0};
    double* v = P.vec(kVecV);
    double* t0 = P.vec(kVecT0);
    double* pl = P.vec(kVecPl);
    double* ul = P.vec(kVecUl);
    double* pp = P.vec(kVecCoupledV);
    double* dv = P.vec(kVecVn);
    const bool relax = o.relax_outer != 0 && !corr;
    // image basis: the local solutions and right-hand sides of every interface
    // product, combined with the GMRES coefficients into a warm start (p, u)
    // for the final solves and the norms of their right-hand sides (which
    // lets those solves take their residuals from fused passes)
    const bool image = !corr;
    static_assert(kVecImage2 == kVecImage + 1 && kVecImage3 == kVecImage + 2, "the image vector spans three slots");
    double* img = P.vec(kVecImage);  // [p (n) | u (3n) | b_D (n) | b_S (3n)]
    const int64_t ld_img = (int64_t)kImageStride * n;
    // t0 = T(0)
    if (r1) {
        dev_fill(0.0, v, n, s);
        darcy(prm, v, pl, false, r1, remove_mean, true);  // v = 0: b = r1
    } else {
        dev_fill(0.0, pl, n, s);
    }
    const double* pstk = pl;
    if (!remove_mean && r1) {
        project_mean(pl, pp);
        pstk = pp;
    }
    // The local solves of T(0) and of the interface products feed only the
    // interface GMRES: with float pairs below the switch point their relaxed
    // GMRES may stop on its residual estimate, whose gap to the true residual
    // is bounded by the float-pair error (about 3e-7) times the residual at
    // the switch (tol_mixed), well below what an interface product needs.
    // The final solves still end on double-pair residuals and the true
    // interface residual decides convergence, correction cycles included.
    const bool est_save = estimate_only, prod_save = in_product;
    estimate_only = relax && image && o.prec == SDBIE_MIXED && o.mixed_mode == 2;
    in_product = relax;
    stokes(prm, U, pstk, fx, ul, false, r2, r1 == nullptr);  // T(0): p = 0 without a Darcy source
    estimate_only = est_save;
    in_product = prod_save;
    dev_normal_component(P, ul, t0, s);
    const double t0n = relax ? norm(t0, n) : 0.0;
    if (image) {
        copy(pl, img, n);  // p(0): zero without an extra Darcy right-hand side
        copy(ul, img + n, 3 * n);
        if (r1) copy(P.vec(kVecDarcyB), img + 4 * n, n);
        else dev_fill(0.0, img + 4 * n, n, s);
        copy(P.vec(kVecStokesB), img + 5 * n, 3 * n);
        outer.W2 = P.image_out;
        outer.ld2 = ld_img;
        outer.x2 = img;
    }
    double tol_cyc = tol;  // relative tolerance of the current cycle
    double safety = kOuterSafety;
    int outer_steps = 0;
    auto op = [&](const double* y, double* out, bool, double rr) {
        const int kslot = krylov_index;  // the local solves below run GMRES of their own
        const double tl_save = tol_local;
        const bool l_save = loose32;
        if (relax && rr > 0.0) {
            const double tl = std::min(kOuterLoosest, std::max(o.tol_gmres, safety * tol_cyc / rr));
            tol_local = tl;
            loose32 = o.prec == SDBIE_MIXED && tl >= kLooseFloat;
        }
        if (debug_level() >= 1)
            std::fprintf(stderr, "[sdbie] interface step %d: residual %.3e, local tolerance %.1e%s\n",
                         ++outer_steps, rr, tol_local > 0.0 ? tol_local : o.tol_gmres,
                         loose32 ? " (float pairs)" : "");
        estimate_only = relax && image && o.prec == SDBIE_MIXED && o.mixed_mode == 2;
        in_product = relax;
        darcy(prm, y, pl, false, nullptr, remove_mean);
        double* slot = image && kslot >= 0 ? P.image_out + (int64_t)kslot * ld_img : nullptr;
        if (slot) {
            // the Darcy solution before its weighted mean was removed: the
            // solution of the completed equation, hence a warm start for it
            copy(pl, slot, n);
            dev_add_scaled_scalar(slot, P.scal + kScalMean, 1.0 / P.area, n, s);
            copy(P.vec(kVecDarcyB), slot + 4 * n, n);
        }
        const double* ps = pl;
        if (!remove_mean) {
            project_mean(pl, pp);
            ps = pp;
        }
        stokes(prm, zero, ps, nullptr, ul, false, nullptr);
        if (slot) {
            copy(ul, slot + n, 3 * n);
            copy(P.vec(kVecStokesB), slot + 5 * n, 3 * n);
        }
        dev_normal_component(P, ul, out, s);
        dev_axpby(1.0, y, -1.0, out, out, n, s);
        tol_local = tl_save;
        loose32 = l_save;
        estimate_only = est_save;
        in_product = prod_save;
    };
    auto finish = [&]() {
        double bD = 0.0, bS = 0.0;  // norms of the final right-hand sides, from the image basis
        if (image) {
            copy(img, p, n);
            copy(img + n, u, 3 * n);
            bD = norm(img + 4 * n, n);
            bS = norm(img + 5 * n, 3 * n);
        }
        darcy(prm, v, p, image, r1, remove_mean, false, bD);
        if (image) {  // keep the pre-mean-removal solution for a correction cycle
            copy(p, img, n);
            dev_add_scaled_scalar(img, P.scal + kScalMean, 1.0 / P.area, n, s);
        }
        const double* ps = p;
        if (!remove_mean) {
            project_mean(p, pp);
            ps = pp;
        }
        stokes(prm, U, ps, fx, u, image, r2, false, bS);
        if (image) copy(u, img + n, 3 * n);
    };
    GmresOut g = gmres(outer, op, t0, v, n, false, tol, o.restart, o.maxit_ddm);
    info.ddm_iters += g.iters;
    info.ddm_res = g.relres;
    bool conv = g.conv;
    double predicted = g.relres;  // the cycle's own estimate of the relative interface residual
    finish();
    for (int cyc = 1; relax && t0n > 0.0; ++cyc) {
        // true interface residual T(v) - v = u.n - v
        dev_normal_component(P, u, pl, s);
        dev_axpby(1.0, pl, -1.0, v, pl, n, s);
        const double rt = norm(pl, n) / t0n;
        info.ddm_res = rt;
        if (debug_level() >= 1) std::fprintf(stderr, "[sdbie] true interface residual %.3e\n", rt);
        conv = rt <= tol;
        if (conv || cyc >= kOuterCycles || info.ddm_iters >= o.maxit_ddm) break;
        if (predicted > 0.0 && rt > 10.0 * predicted) safety = std::max(safety * predicted / rt, 1e-12);
        // correction cycle: (I - T_lin) d = u.n - v, relative tolerance tol / rt
        copy(pl, t0, n);
        tol_cyc = std::min(0.5, tol / rt);
        GmresOut gc = gmres(outer, op, t0, dv, n, false, tol_cyc, o.restart, o.maxit_ddm - info.ddm_iters);
        info.ddm_iters += gc.iters;
        predicted = rt * gc.relres;
        dev_axpby(1.0, v, 1.0, dv, v, n, s);
        finish();
    }
    if (!conv && !corr) converged = false;
    outer.W2 = nullptr;
    outer.x2 = nullptr;
}

// out = p - (sum_j w_j p_j / |S|)
void Ctx::project_mean(const double* p, double* out) {
    copy(p, out, P.n);
    dev_dot(P, P.w, p, P.n, P.scal + kScalMean, s);
    dev_add_scaled_scalar(out, P.scal + kScalMean, -1.0 / P.area, P.n, s);
}

// Residual of the coupled system whose solution is the D-N fixed point.
// Unknowns: pt (Darcy pressure before its weighted mean is removed) and u.
//   r1 = -(Abar_D pt - (mu/K) S_L[u.n])
//   r2 = U - (Abar_S u + V[-(Pi pt) n + beta P_tau u + f_extra])
// Two fused double-pair passes (Laplace double + single layer, stresslet +
// Stokeslet).
void Ctx::coupled_residual(const sdbie_params& prm, const double U[3], const double* fx, const double* pt,
                           const double* u, double* r1, double* r2) {
    const int64_t n = P.n;
    const double beta = prm.alpha * prm.mu / std::sqrt(prm.K);
    double* vn = P.vec(kVecCoupledV);
    dev_normal_component(P, u, vn, s);
    dev_dot(P, P.w, pt, n, P.scal + kScalCompD, s);
    PassDesc d;
    d.dl = true;
    d.sub = true;
    d.c_dl = -1.0 / (4.0 * kPi);
    d.dl_dens = pt;
    d.sl = true;
    d.c_sl = -(prm.mu / prm.K) / (4.0 * kPi);
    d.sl_dens = vn;
    d.comp = P.scal + kScalCompD;
    d.comp_scale = -1.0 / P.area;
    d.out = r1;
    launch_laplace_pass(P, d, s);
    // projected pressure and the traction
    double* f = P.vec(kVecTraction);
    project_mean(pt, vn);
    dev_traction(P, vn, u, beta, fx, f, s);
    dev_dot(P, P.wn, u, 3 * n, P.scal + kScalCompS, s);
    PassDesc e;
    e.dl = true;
    e.sub = true;
    e.c_dl = 3.0 / (4.0 * kPi);
    e.dl_dens = u;
    e.base = u;
    e.base_scale = -1.0;
    e.sl = true;
    e.c_sl = -1.0 / (8.0 * kPi * prm.mu);
    e.sl_dens = f;
    e.comp = P.scal + kScalCompS;
    e.comp_scale = -1.0 / P.area;
    e.add_const = U;
    e.out = r2;
    launch_stokes_pass(P, e, s);
}

// Mixed-precision coupled solve: iterative refinement of the coupled system
// with double-pair residuals; each correction is a D-N solve (interface
// GMRES, local GMRES) with float-pair operators.  The local solves stop at
// tol_mixed; the interface GMRES at tol_mixed * min(1, K / (mu R^2)) with R
// the equivalent radius of the surface: the correction's Darcy equation sees
// the interface iterate v instead of the final u.n, and the Darcy residual
// it leaves behind is (mu/K) S_L[u.n - v], so the interface tolerance is
// scaled by K/mu to keep the contraction per step near tol_mixed.  Stops
// when ||r|| <= tol_ddm ||b|| (b: the right-hand side at u = p = 0).
void Ctx::ddm_refined(const sdbie_params& prm, const double U[3], const double* fx, double* p, double* u) {
    const int64_t n = P.n;
    double* pt = P.vec(kVecCoupledP);
    double* uu = P.vec(kVecCoupledU);
    double* r1 = P.vec(kVecCoupledR1);
    double* r2 = P.vec(kVecCoupledR2);
    double* dp = P.vec(kVecCoupledDP);
    double* du = P.vec(kVecCoupledDU);
    dev_fill(0.0, pt, n, s);
    dev_fill(0.0, uu, 3 * n, s);
    dev_fill(0.0, r1, n, s);
    if (fx) {
        single_layer_stokes(fx, prm.mu, -1.0, U, r2, false);
    } else {
        for (int c = 0; c < 3; ++c) dev_fill(U[c], r2 + c * n, n, s);
    }
    const double bnorm = std::sqrt(dot(r2, r2, 3 * n));
    const double target = o.tol_ddm;
    double rel = 1.0;
    int step = 0;
    for (;; ++step) {
        if (step > 0) coupled_residual(prm, U, fx, pt, uu, r1, r2);
        rel = bnorm > 0.0 ? std::sqrt(dot(r1, r1, n) + dot(r2, r2, 3 * n)) / bnorm : 0.0;
        if (debug_level() > 0)
            std::fprintf(stderr, "[sdbie] coupled refinement step %d: ||r||/||b|| = %.3e (r1 %.3e, r2 %.3e)\n", step,
                         rel, std::sqrt(dot(r1, r1, n)) / bnorm, std::sqrt(dot(r2, r2, 3 * n)) / bnorm);
        if (rel <= target || step >= o.refine_max) break;
        corr = true;
        tol_corr = o.tol_mixed;
        const double R2 = P.area / (4.0 * kPi);
        const double tol_if = tol_corr * std::min(1.0, prm.K / (prm.mu * R2));
        const double zero[3] = {0.0, 0.0, 0.0};
        ddm_outer(prm, zero, nullptr, r1, r2, dp, du, false, tol_if);
        corr = false;
        dev_axpby(1.0, pt, 1.0, dp, pt, n, s);
        dev_axpby(1.0, uu, 1.0, du, uu, 3 * n, s);
    }
    info.refine_steps += step;
    info.relres = rel;
    if (rel > target) converged = false;
    project_mean(pt, p);
    copy(uu, u, 3 * n);
}

// ------------------------------------------------------------------------------
// Adjoint of the coupled solve (gradient of J = e . drag)
// ------------------------------------------------------------------------------
// Forward (the D-N fixed point, unknowns pt and u):
//   F1 = Abar_D pt - (mu/K) S_L[N u] = 0,
//   F2 = (Abar_S + beta V P_tau) u - V[Nhat Pi pt] + V[f_extra] - U = 0,
//   J  = e . sum_j w_j f_j,  f = -(Pi pt) n + beta P_tau u + f_extra,
// with N u = u.n, Nhat p = p n, Pi = I - 1 w^T/|S|.  The adjoint system
//   Abar_D^T lam1 - Pi^T Nhat^T V^T lam2 = dJ/dpt = Pi^T (-w (e.n)),
//   -(mu/K) N^T S_L^T lam1 + (Abar_S + beta V P_tau)^T lam2 = dJ/du = beta w P_tau e,
// is solved by the transposed interface iteration on lam1 (GMRES on the affine
// map lam1 -> Abar_D^-T [dJ/dpt + Pi^T Nhat^T V^T S^-T (dJ/du + (mu/K) N^T S_L^T lam1)]).
// Transposed sums: S_L^T l = w (.) S~[l] and V^T l = w (.) V~[l] (unit source
// weights, target weight); A_D^T l = -(1/4pi) w (.) n.sum l_s D K2 + l (.) D_L[1];
// A_S^T l = l - M l + (3/4pi) w (.) sum (D.l_s)(D.n_t) D K4 with the stresslet
// moment M_t = -(3/4pi) sum_s w_s (D.n_s) K4 D D^T.  Then
//   dJ/dx    = -lam^T dF/dx   (position-gradient pass; normals and weights fixed)
//   dJ/dlogK = -(beta/2) e.sum w P_tau u - lam1.(mu/K) S_L[u.n] + (beta/2) lam2.V[P_tau u]
//   dJ/dalpha = (beta/alpha) [e.sum w P_tau u - lam2.V[P_tau u]]
// p (= Pi pt) replaces pt throughout: every term sees pt only through
// differences pt_j - pt_i or through Pi pt.
void Ctx::adjoint(const sdbie_params& prm, const double U[3], const double* fx, const double* p, const double* u,
                  const double e[3], double* grad, double* dlogK, double* dalpha) {
    (void)U;
    const int64_t n = P.n;
    const double mu = prm.mu, K = prm.K;
    const double beta = prm.alpha * mu / std::sqrt(K);
    double* lam1 = P.vec(kVecV);
    double* dl1 = P.vec(kVecVn);
    double* t0 = P.vec(kVecT0);
    double* tD = P.vec(kVecPl);      // n-vector temporaries
    double* tE = P.vec(kVecUl);      // 3n rhs of the transposed Stokes solve
    double* tA = P.vec(kVecDarcyB);  // transposed Darcy operator temp
    double* tB = P.vec(kVecStokesB); // transposed stresslet temp
    double* tC = P.vec(kVecTraction);// transposed Stokeslet temp (follows tB)
    static_assert(kVecTraction == kVecStokesB + 1, "the fused transposed pass writes tB and tC as one [6][n] block");
    double* x2 = P.vec(kVecIn);
    double* tG = P.vec(kVecOut);
    double* x1 = P.vec(kVecCoupledV);
    double* m0 = P.vec(kVecCoupledP);
    double* m1 = P.vec(kVecCoupledU);
    double* m2 = P.vec(kVecCoupledR1);
    double* gp = P.vec(kVecCoupledR2);
    double* gu = P.vec(kVecCoupledDP);
    double* lam2 = P.vec(kVecCoupledDU);
    double* mneg[3] = {m0, m1, m2};

    // diagonal terms: D_L[1] and -M e_c (subtracted stresslet with zero source density)
    dev_fill(1.0, tD, n, s);
    {
        PassDesc d;
        d.dl = true;
        d.c_dl = -1.0 / (4.0 * kPi);
        d.dl_dens = tD;
        d.out = dl1;
        launch_laplace_pass(P, d, s);
    }
    dev_fill(0.0, tE, 3 * n, s);
    for (int c = 0; c < 3; ++c) {
        dev_fill(0.0, tG, 3 * n, s);
        dev_fill(1.0, tG + c * n, n, s);
        PassDesc d;
        d.dl = true;
        d.sub = true;
        d.c_dl = -3.0 / (4.0 * kPi);
        d.dl_dens = tE;
        d.dl_target = tG;
        d.out = mneg[c];
        launch_stokes_pass(P, d, s);
    }
    // transposed operators (m32: float pairs for the transposed sums; the
    // diagonal terms dl1 and M above stay double)
    auto opDT = [&](const double* l, double* out, bool m32) {
        PassDesc d;
        d.dl = true;
        d.target_normal = true;
        d.unit_src_weight = true;
        d.target_weight = true;
        d.c_dl = -1.0 / (4.0 * kPi);
        d.dl_dens = l;
        d.out = tA;
        d.mixed = m32;
        launch_laplace_pass(P, d, s);
        dev_dot(P, l, nullptr, n, P.scal + kScalCompD, s);
        dev_adj_darcy(P, tA, l, dl1, P.scal + kScalCompD, out, s);
    };
    auto opST = [&](const double* l, double* out, bool m32) {
        PassDesc d;
        d.dl = true;
        d.target_normal = true;
        d.unit_src_weight = true;
        d.target_weight = true;
        d.c_dl = 3.0 / (4.0 * kPi);
        d.dl_dens = l;
        d.out = tB;
        d.mixed = m32;
        if (beta != 0.0) {
            // with slip, the transposed Stokeslet of the same density comes
            // from the same pass, target-weighted, into tC = tB + 3n
            d.sl = true;
            d.c_sl = 1.0 / (8.0 * kPi * mu);
            d.sl_dens = l;
        }
        launch_stokes_pass(P, d, s);
        dev_normal_component(P, l, tD, s);
        dev_dot(P, tD, nullptr, n, P.scal + kScalCompS, s);
        dev_adj_stokes(P, l, m0, m1, m2, tB, beta != 0.0 ? tC : nullptr, P.scal + kScalCompS, beta, out, s);
    };
    // transposed local solves: double pairs, or with float pairs the relaxed
    // GMRES of the forward solves (float products below the switch point,
    // double true residuals decide convergence).  Inside an inexact interface
    // product they run to tl_adj, all in float pairs when l32_adj.
    const bool mixed = o.prec == SDBIE_MIXED;
    double tl_adj = o.tol_gmres;
    bool l32_adj = false;
    auto solve_T = [&](const std::function<void(const double*, double*, bool)>& op, const double* b, double* x,
                       int64_t L) {
        const double relax = l32_adj ? kAllFloat : (mixed ? std::min(1.0, o.tol_mixed * (tl_adj / o.tol_gmres)) : 0.0);
        GmresOut g = gmres(inner, [&](const double* in, double* out, bool m32, double) { op(in, out, m32); }, b, x,
                           L, false, tl_adj, o.restart, o.maxit_gmres, relax);
        info.gmres_iters += g.iters;
        if (mixed) info.refine_steps += g.checks;
        info.relres = g.relres;
        if (!g.conv) converged = false;
    };
    // transposed single layers: out = w (.) S~[l] (scaled) / w (.) V~[l]
    auto SLT = [&](const double* l, double scale, double* out) {
        PassDesc d;
        d.sl = true;
        d.unit_src_weight = true;
        d.target_weight = true;
        d.c_sl = -scale / (4.0 * kPi);
        d.sl_dens = l;
        d.out = out;
        d.mixed = l32_adj;
        launch_laplace_pass(P, d, s);
    };
    auto VT = [&](const double* l, double* out) {
        PassDesc d;
        d.sl = true;
        d.unit_src_weight = true;
        d.target_weight = true;
        d.c_sl = 1.0 / (8.0 * kPi * mu);
        d.sl_dens = l;
        d.out = out;
        d.mixed = l32_adj;
        launch_stokes_pass(P, d, s);
    };
    // Pi^T g = g - w (sum g)/|S|   (in place)
    auto PiT = [&](double* g) {
        dev_dot(P, g, nullptr, n, P.scal + kScalMean, s);
        dev_axpy_w(P, g, P.scal + kScalMean, -1.0 / P.area, s);
    };
    // y -> Abar_D^-T [base + Pi^T Nhat^T V^T S^-T (rhs3)],  rhs3 in tE
    // the transposed Stokes solves share one operator: with double pairs the
    // first fills the deflation space and the later ones use it (as in ddm_solve)
    const bool rc_on = o.recycle && o.prec == SDBIE_FP64;
    auto solve_ST = [&](const double* b, double* x) {
        rc_cur = rc_on ? &rc_stokes : nullptr;
        solve_T(opST, b, x, 3 * n);
        rc_cur = nullptr;
    };
    auto chain = [&](const double* base, double* out) {
        solve_ST(tE, x2);               // x2 = S^-T rhs3
        VT(x2, tG);                     // tG = V^T x2
        dev_normal_component(P, tG, tD, s);
        PiT(tD);
        if (base) dev_axpby(1.0, tD, 1.0, base, tD, n, s);
        solve_T(opDT, tD, out, n);
    };

    dev_adj_rhs(P, e, beta, gp, gu, s);
    PiT(gp);
    // t0 = T'(0)
    copy(gu, tE, 3 * n);
    chain(gp, t0);
    // the transposed interface equation, with the inexact products and
    // correction cycles of the forward interface GMRES (relax_outer)
    const bool relax = o.relax_outer != 0;
    double tol_cyc = o.tol_ddm;
    double safety = kOuterSafety;
    auto opOuter = [&](const double* y, double* out, bool, double rr) {
        if (relax && rr > 0.0) {
            tl_adj = std::min(kOuterLoosest, std::max(o.tol_gmres, safety * tol_cyc / rr));
            l32_adj = mixed && tl_adj >= kLooseFloat;
        }
        SLT(y, 1.0, tA);                          // S_L^T y
        dev_scalar_normal(P, tA, mu / K, tE, s);  // (mu/K) N^T S_L^T y
        chain(nullptr, x1);
        dev_axpby(1.0, y, -1.0, x1, out, n, s);
        tl_adj = o.tol_gmres;
        l32_adj = false;
    };
    GmresOut g = gmres(outer, opOuter, t0, lam1, n, false, o.tol_ddm, o.restart, o.maxit_ddm);
    info.ddm_iters = g.iters;
    info.ddm_res = g.relres;
    bool conv = g.conv;
    if (relax) {
        // true residual t0 - (I - T'_lin) lam1 with full-accuracy local solves;
        // correction cycles while it is above tol_ddm
        double* rt_v = P.vec(kVecImage);
        double* dlam = P.vec(kVecImage2);
        const double t0n = norm(t0, n);
        double predicted = g.relres;
        for (int cyc = 1; t0n > 0.0; ++cyc) {
            opOuter(lam1, rt_v, false, 0.0);
            dev_axpby(1.0, t0, -1.0, rt_v, rt_v, n, s);
            const double rt = norm(rt_v, n) / t0n;
            info.ddm_res = rt;
            if (debug_level() >= 1) std::fprintf(stderr, "[sdbie] adjoint: true interface residual %.3e\n", rt);
            conv = rt <= o.tol_ddm;
            if (conv || cyc >= kOuterCycles || info.ddm_iters >= o.maxit_ddm) break;
            if (predicted > 0.0 && rt > 10.0 * predicted) safety = std::max(safety * predicted / rt, 1e-12);
            tol_cyc = std::min(0.5, o.tol_ddm / rt);
            GmresOut gc = gmres(outer, opOuter, rt_v, dlam, n, false, tol_cyc, o.restart, o.maxit_ddm - info.ddm_iters);
            info.ddm_iters += gc.iters;
            dev_axpby(1.0, lam1, 1.0, dlam, lam1, n, s);
            predicted = rt * gc.relres;
        }
    }
    if (!conv) converged = false;
    // lam2 = S^-T (gu + (mu/K) N^T S_L^T lam1)
    SLT(lam1, 1.0, tA);
    dev_scalar_normal(P, tA, mu / K, tE, s);
    dev_axpby(1.0, tE, 1.0, gu, tE, 3 * n, s);
    solve_ST(tE, lam2);

    // position gradient
    double* v = P.vec(kVecRefR);
    double* f = P.vec(kVecRefC);
    dev_normal_component(P, u, v, s);
    dev_traction(P, p, u, beta, fx, f, s);
    GradDesc gd;
    gd.mu = mu;
    gd.K = K;
    gd.p = p;
    gd.v = v;
    gd.u = u;
    gd.f = f;
    gd.lam1 = lam1;
    gd.lam2 = lam2;
    gd.out = grad;
    launch_grad_pass(P, gd, s);

    // parameter derivatives
    double* tu = tC;
    dev_traction(P, nullptr, u, 1.0, nullptr, tu, s);  // P_tau u
    double ewtu = 0.0;
    for (int c = 0; c < 3; ++c) ewtu += e[c] * dot(P.w, tu + c * n, n);
    single_layer_laplace(v, 1.0, tA, false);             // S_L[u.n]
    single_layer_stokes(tu, mu, 1.0, nullptr, tG, false); // V[P_tau u]
    const double l1S = dot(lam1, tA, n);
    const double l2V = dot(lam2, tG, 3 * n);
    *dlogK = -(beta / 2.0) * ewtu - (mu / K) * l1S + (beta / 2.0) * l2V;
    const double sa = mu / std::sqrt(K);
    *dalpha = sa * (ewtu - l2V);
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
    rc_stokes.V = P.basis_rc;
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
