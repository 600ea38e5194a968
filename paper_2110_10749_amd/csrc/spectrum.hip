// Spectrum of the Dirichlet-Neumann iteration (section "Discrete iteration
// operator", eqs. (Discrete_iter_oper) and (A_mat)).
//
// With no far-field flow the D-N map is linear: T_lin(v) = u(p(v)).n, p the
// Darcy solution for the flux v (mean removed), u the Stokes solution for the
// traction -p n (+ the implicit slip term).  The relaxed iteration multiplies
// the interface unknown by A~ = (1 - theta) I + theta T_lin, so the
// eigenvalues of A~ are 1 - theta + theta lambda for the eigenvalues lambda of
// T_lin.  The matrix is never formed: m steps of Arnoldi on T_lin (every
// product a Darcy and a Stokes solve on the device, classical Gram-Schmidt
// with one re-orthogonalisation as in the GMRES of solver.hip) give an upper
// Hessenberg matrix whose eigenvalues, the Ritz values, approximate the
// eigenvalues of T_lin of largest modulus first.  The Hessenberg eigenvalue
// problem (m <= 1000) is solved on the host by the Francis double-shift QR
// iteration.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <vector>

#include "solver.h"

namespace sdbie {

// Eigenvalues of an upper Hessenberg matrix A (n x n, row-major; overwritten)
// by the Francis double-shift QR iteration (Golub and Van Loan, "Matrix
// Computations", section 7.5): each step chases the bulge of the implicit
// double shift down the active window with Householder reflectors of three
// elements (two at the end), applied only inside the window since only the
// eigenvalues are wanted; a subdiagonal entry below DBL_EPSILON times the
// larger of its two diagonal neighbours' sum and the largest entry of the
// matrix deflates the window, and 1x1 and 2x2 trailing blocks
// give their eigenvalues in closed form.  A real pair of shifts is replaced by
// the one closer to the last diagonal entry, taken twice, and ad hoc shifts
// after 10 and 20 steps without deflation break cycles (both as in LAPACK's
// small-matrix QR).  Returns false if one eigenvalue needs more than 100
// steps.
bool hessenberg_eigenvalues(int n, double* A, double* wr, double* wi) {
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    double hmax = 0.0;  // largest entry: the scale of the normwise deflation test
    for (int i = 0; i < n; ++i)
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) hmax = std::fmax(hmax, std::fabs(a(i, j)));
    int hi = n - 1, its = 0;
    while (hi >= 0) {
        // deflation: the lowest l > 0 in the window with a negligible a(l, l-1),
        // below DBL_EPSILON times its diagonal neighbours or times the largest
        // entry (normwise backward stable; the copies of one eigenvalue in a
        // cluster leave subdiagonals a few ulps of that eigenvalue in size)
        int l = hi;
        for (; l > 0; --l) {
            const double sc = std::fmax(std::fabs(a(l - 1, l - 1)) + std::fabs(a(l, l)), hmax);
            if (std::fabs(a(l, l - 1)) <= DBL_EPSILON * sc) {
                a(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {  // a 1x1 block
            wr[hi] = a(hi, hi);
            wi[hi] = 0.0;
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {  // a 2x2 block [[p, q], [r, s]]
            const double p = a(hi - 1, hi - 1), q = a(hi - 1, hi), r = a(hi, hi - 1), s = a(hi, hi);
            const double mid = 0.5 * (p + s), half = 0.5 * (p - s);
            const double disc = half * half + q * r;
            if (disc >= 0.0) {
                const double root = std::sqrt(disc);
                const double l1 = mid + (mid >= 0.0 ? root : -root);  // the one of larger modulus
                const double l2 = l1 != 0.0 ? (p * s - q * r) / l1 : mid - root;
                wr[hi - 1] = l1;
                wr[hi] = l2;
                wi[hi - 1] = wi[hi] = 0.0;
            } else {
                const double root = std::sqrt(-disc);
                wr[hi - 1] = wr[hi] = mid;
                wi[hi - 1] = root;
                wi[hi] = -root;
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (its >= 100) return false;
        // the double shift (sum s and product t of the two shifts): the
        // eigenvalues of the trailing 2x2 block when they are complex; when
        // they are real, twice the one closer to a(hi, hi).  The trailing
        // block's own pair would annihilate the first column of the step
        // whenever a block higher in the window has the same eigenvalues, as
        // the copies of one eigenvalue that Arnoldi on a symmetric surface
        // produces do; a repeated real shift does not.  Steps 10 and 20 take
        // an ad hoc complex pair near a(hi, hi) instead.
        double s, t;
        const double p = a(hi - 1, hi - 1), q = a(hi - 1, hi), r = a(hi, hi - 1), d = a(hi, hi);
        if (its == 10 || its == 20) {
            const double x = std::fabs(a(hi, hi - 1)) + std::fabs(a(hi - 1, hi - 2));
            const double c = d + 0.75 * x;
            s = 2.0 * c;
            t = c * c + 0.4375 * x * x;
        } else {
            const double mid = 0.5 * (p + d), half = 0.5 * (p - d), disc = half * half + q * r;
            if (disc >= 0.0) {
                const double root = std::sqrt(disc);
                const double sig = std::fabs(mid + root - d) <= std::fabs(mid - root - d) ? mid + root : mid - root;
                s = 2.0 * sig;
                t = sig * sig;
            } else {
                s = p + d;
                t = p * d - q * r;
            }
        }
        ++its;
        // first column of (A - s1 I)(A - s2 I) = A^2 - s A + t I (rows l .. l+2)
        double v[3];
        v[0] = a(l, l) * a(l, l) + a(l, l + 1) * a(l + 1, l) - s * a(l, l) + t;
        v[1] = a(l + 1, l) * (a(l, l) + a(l + 1, l + 1) - s);
        v[2] = a(l + 1, l) * a(l + 2, l + 1);
        for (int k = l; k < hi; ++k) {
            const int len = hi - k + 1 < 3 ? hi - k + 1 : 3;
            if (k > l)
                for (int i = 0; i < len; ++i) v[i] = a(k + i, k - 1);
            // reflector I - beta u u^T mapping v onto a multiple of e_1
            double nv = 0.0;
            for (int i = 0; i < len; ++i) nv += v[i] * v[i];
            nv = std::sqrt(nv);
            if (nv == 0.0) continue;
            const double alpha = v[0] >= 0.0 ? -nv : nv;
            double u[3] = {v[0] - alpha, len > 1 ? v[1] : 0.0, len > 2 ? v[2] : 0.0};
            double uu = 0.0;
            for (int i = 0; i < len; ++i) uu += u[i] * u[i];
            if (uu == 0.0) continue;
            const double beta = 2.0 / uu;
            // from the left: rows k .. k+len-1, columns from the bulge's column to hi
            for (int j = (k > l ? k - 1 : l); j <= hi; ++j) {
                double dot = 0.0;
                for (int i = 0; i < len; ++i) dot += u[i] * a(k + i, j);
                dot *= beta;
                for (int i = 0; i < len; ++i) a(k + i, j) -= dot * u[i];
            }
            if (k > l) {  // the reflector zeroed the bulge below a(k, k-1)
                a(k, k - 1) = alpha;
                for (int i = 1; i < len; ++i) a(k + i, k - 1) = 0.0;
            }
            // from the right: columns k .. k+len-1, rows l .. min(k+3, hi)
            const int rmax = k + 3 < hi ? k + 3 : hi;
            for (int i = l; i <= rmax; ++i) {
                double dot = 0.0;
                for (int j = 0; j < len; ++j) dot += a(i, k + j) * u[j];
                dot *= beta;
                for (int j = 0; j < len; ++j) a(i, k + j) -= dot * u[j];
            }
        }
    }
    return true;
}

// m Arnoldi steps on T_lin from v0 (sorted order, nonzero); H receives the
// (m+1) x m Hessenberg matrix (row-major, m columns).  Returns the steps taken
// (fewer than m when the Krylov space is invariant).
int Ctx::dn_arnoldi(const sdbie_params& prm, const double* v0, int m, std::vector<double>& H) {
    const int64_t n = P.n;
    const double zero[3] = {0.0, 0.0, 0.0};
    double* V = P.basis_out;
    double* w = P.vec(kVecOuterW);
    double* pl = P.vec(kVecPl);
    double* ul = P.vec(kVecUl);
    const double b = norm(v0, n);
    if (b == 0.0) throw Error(SDBIE_ERR_ARG, "the start vector is zero");
    dev_scale(1.0 / b, v0, V, n, s);
    H.assign((size_t)(m + 1) * m, 0.0);
    std::vector<double> col(2 * (m + 1) + 1);
    int used = 0;
    for (int k = 0; k < m; ++k) {
        const double* vk = V + (int64_t)k * n;
        darcy(prm, vk, pl, false, nullptr, true);
        stokes(prm, zero, pl, nullptr, ul, false, nullptr);
        dev_normal_component(P, ul, w, s);
        double* h1 = outer.dcol;
        double* h2 = outer.dcol + (k + 1);
        double* hn = outer.dcol + 2 * (k + 1);
        dev_multidot(P, V, n, k + 1, w, n, h1, s);
        dev_multi_axpy_sub(V, n, k + 1, h1, w, n, s);
        dev_multidot(P, V, n, k + 1, w, n, h2, s);
        dev_multi_axpy_sub(V, n, k + 1, h2, w, n, s);
        dev_dot(P, w, w, n, hn, s);
        SDBIE_HIP(hipMemcpyAsync(col.data(), outer.dcol, (2 * (k + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                 s));
        SDBIE_HIP(hipStreamSynchronize(s));
        double cn = 0.0;
        for (int j = 0; j <= k; ++j) {
            H[(size_t)j * m + k] = col[j] + col[k + 1 + j];
            cn += H[(size_t)j * m + k] * H[(size_t)j * m + k];
        }
        const double hk1 = std::sqrt(col[2 * (k + 1)]);
        if (!std::isfinite(hk1)) throw Error(SDBIE_ERR_NONFINITE, "non-finite Arnoldi vector");
        H[(size_t)(k + 1) * m + k] = hk1;
        used = k + 1;
        if (hk1 <= 1e-14 * std::sqrt(cn + hk1 * hk1)) break;  // invariant subspace
        if (k + 1 < m) dev_scale(1.0 / hk1, w, V + (int64_t)(k + 1) * n, n, s);
    }
    return used;
}

}  // namespace sdbie
