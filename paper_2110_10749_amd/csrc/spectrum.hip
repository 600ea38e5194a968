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

// The double shift of one QR step from a 2x2 block [[h11, h12], [h21, h22]]:
// its eigenvalues when they are complex (sh = re, im, re, -im); when they are
// real, twice the one closer to h22 (a trailing block's own pair of real
// shifts would annihilate the first column of the step whenever a block
// higher in the window has the same eigenvalues, as the copies of one
// eigenvalue that Arnoldi on a symmetric surface produces do).  The block is
// scaled to unit size first.
static void double_shift(double h11, double h12, double h21, double h22, double sh[4]) {
    const double sc = std::fabs(h11) + std::fabs(h12) + std::fabs(h21) + std::fabs(h22);
    if (sc == 0.0) {
        sh[0] = sh[1] = sh[2] = sh[3] = 0.0;
        return;
    }
    h11 /= sc;
    h12 /= sc;
    h21 /= sc;
    h22 /= sc;
    const double tr = 0.5 * (h11 + h22);
    const double det = (h11 - tr) * (h22 - tr) - h12 * h21;
    const double rt = std::sqrt(std::fabs(det));
    if (det >= 0.0) {
        sh[0] = sh[2] = tr * sc;
        sh[1] = rt * sc;
        sh[3] = -rt * sc;
    } else {
        const double r1 = tr + rt, r2 = tr - rt;
        sh[0] = sh[2] = (std::fabs(r1 - h22) <= std::fabs(r2 - h22) ? r1 : r2) * sc;
        sh[1] = sh[3] = 0.0;
    }
}

// Eigenvalues of an upper Hessenberg matrix A (n x n, row-major; overwritten)
// by the Francis double-shift QR iteration (Golub and Van Loan, "Matrix
// Computations", section 7.5), with the safeguards of LAPACK's small-matrix
// QR: only the active window is transformed, since only the eigenvalues are
// wanted; a subdiagonal entry deflates when it is negligible against its
// diagonal neighbours in the sense of Ahues and Tisseur; the first column of
// the double-shift polynomial is formed from the shifts themselves,
// (a00 - s1)(a00 - s2) + a01 a10, never from their sum and product (for a
// cluster of nearly equal eigenvalues a00^2 - s a00 + t cancels to noise and
// the iteration stalls); a step starts below the top of the window where two
// consecutive subdiagonal entries are small enough; ad hoc shifts every 10
// steps without deflation break cycles; 1x1 and 2x2 blocks give their
// eigenvalues in closed form.  Returns false if 30 max(10, n) steps pass
// without a deflation; the eigenvalues not reached by then are NaN.
bool hessenberg_eigenvalues(int n, double* A, double* wr, double* wi) {
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    const double ulp = DBL_EPSILON, tiny = DBL_MIN;
    const int itmax = 30 * (n > 10 ? n : 10);
    int hi = n - 1;
    while (hi >= 0) {
        int l = hi, kdefl = 0;
        for (int its = 0;; ++its) {
            // the lowest l > 0 with a negligible a(l, l-1), or 0
            for (l = hi; l > 0; --l) {
                const double sub = std::fabs(a(l, l - 1));
                if (sub <= tiny) break;
                double tst = std::fabs(a(l - 1, l - 1)) + std::fabs(a(l, l));
                if (tst == 0.0) {
                    if (l >= 2) tst += std::fabs(a(l - 1, l - 2));
                    if (l + 1 <= hi) tst += std::fabs(a(l + 1, l));
                }
                if (sub <= ulp * tst) {
                    const double up = std::fabs(a(l - 1, l));
                    const double ab = std::fmax(sub, up), ba = std::fmin(sub, up);
                    const double dd = std::fabs(a(l - 1, l - 1) - a(l, l));
                    const double aa = std::fmax(std::fabs(a(l, l)), dd), bb = std::fmin(std::fabs(a(l, l)), dd);
                    const double sc = aa + ab;
                    if (ba * (ab / sc) <= std::fmax(tiny, ulp * (bb * (aa / sc)))) break;
                }
            }
            if (l > 0) a(l, l - 1) = 0.0;
            if (l >= hi - 1) break;  // a 1x1 or 2x2 block has split off
            if (its >= itmax) {
                for (int i = 0; i <= hi; ++i) wr[i] = wi[i] = NAN;
                return false;
            }
            ++kdefl;
            double sh[4];
            if (kdefl % 20 == 0) {  // ad hoc shift from the top of the window
                const double x = std::fabs(a(l + 1, l)) + std::fabs(a(l + 2, l + 1));
                const double c = 0.75 * x + a(l, l);
                double_shift(c, -0.4375 * x, x, c, sh);
            } else if (kdefl % 10 == 0) {  // from the bottom
                const double x = std::fabs(a(hi, hi - 1)) + std::fabs(a(hi - 1, hi - 2));
                const double c = 0.75 * x + a(hi, hi);
                double_shift(c, -0.4375 * x, x, c, sh);
            } else {
                double_shift(a(hi - 1, hi - 1), a(hi - 1, hi), a(hi, hi - 1), a(hi, hi), sh);
            }
            // first column of (A - s1 I)(A - s2 I) at rows m .. m+2, scaled; the
            // step starts at the lowest m whose a(m, m-1) it would barely touch
            double v[3];
            int m = hi - 2;
            for (;; --m) {
                const double h21 = a(m + 1, m);
                double sc = std::fabs(a(m, m) - sh[2]) + std::fabs(sh[3]) + std::fabs(h21);
                const double h21s = sc != 0.0 ? h21 / sc : 0.0;
                if (sc == 0.0) sc = 1.0;
                v[0] = h21s * a(m, m + 1) + (a(m, m) - sh[0]) * ((a(m, m) - sh[2]) / sc) - sh[1] * (sh[3] / sc);
                v[1] = h21s * (a(m, m) + a(m + 1, m + 1) - sh[0] - sh[2]);
                v[2] = h21s * a(m + 2, m + 1);
                const double sv = std::fabs(v[0]) + std::fabs(v[1]) + std::fabs(v[2]);
                if (sv != 0.0)
                    for (double& x : v) x /= sv;
                if (m == l) break;
                const double h00 = std::fabs(a(m - 1, m - 1)) + std::fabs(a(m, m)) + std::fabs(a(m + 1, m + 1));
                if (std::fabs(a(m, m - 1)) * (std::fabs(v[1]) + std::fabs(v[2])) <= ulp * std::fabs(v[0]) * h00) break;
            }
            // chase the bulge down the window with reflectors I - tau w w^T,
            // w = (1, w1, w2), each mapping its vector onto beta e1
            for (int k = m; k < hi; ++k) {
                const int len = hi - k + 1 < 3 ? hi - k + 1 : 3;
                if (k > m)
                    for (int i = 0; i < len; ++i) v[i] = a(k + i, k - 1);
                double xn = 0.0;
                for (int i = 1; i < len; ++i) xn += v[i] * v[i];
                xn = std::sqrt(xn);
                double tau = 0.0, beta = v[0], w[3] = {1.0, 0.0, 0.0};
                if (xn != 0.0) {
                    beta = -std::copysign(std::hypot(v[0], xn), v[0]);
                    tau = (beta - v[0]) / beta;
                    for (int i = 1; i < len; ++i) w[i] = v[i] / (v[0] - beta);
                }
                if (k > m) {
                    a(k, k - 1) = beta;
                    for (int i = 1; i < len; ++i) a(k + i, k - 1) = 0.0;
                } else if (m > l) {
                    a(k, k - 1) *= 1.0 - tau;
                }
                if (tau == 0.0) continue;
                for (int j = k; j <= hi; ++j) {  // from the left: rows k .. k+len-1
                    double dot = 0.0;
                    for (int i = 0; i < len; ++i) dot += w[i] * a(k + i, j);
                    dot *= tau;
                    for (int i = 0; i < len; ++i) a(k + i, j) -= dot * w[i];
                }
                const int rmax = k + 3 < hi ? k + 3 : hi;
                for (int i = l; i <= rmax; ++i) {  // from the right: columns k .. k+len-1
                    double dot = 0.0;
                    for (int j = 0; j < len; ++j) dot += a(i, k + j) * w[j];
                    dot *= tau;
                    for (int j = 0; j < len; ++j) a(i, k + j) -= dot * w[j];
                }
            }
        }
        if (l == hi) {  // a 1x1 block
            wr[hi] = a(hi, hi);
            wi[hi] = 0.0;
            hi -= 1;
            continue;
        }
        // a 2x2 block [[p, q], [r, s]]
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
