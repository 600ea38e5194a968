/*
 * Plain FP64 CPU oracle for the regularised layer sums of the Stokes-Darcy
 * boundary-integral method.  TEST INFRASTRUCTURE ONLY: it is linked by the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark,
 * never by the product library.  It shares no code with the HIP path.
 *
 * Notation (paper, section "High-order regularization of kernels on the
 * surface" and section "Boundary integral formulations"):
 *   target i, source j, d = x_i - x_j (the paper's yhat = y - x with y the
 *   target), r = |d|, rho = r / delta.
 *   The smoothed kernels replace 1/r^p by s_k(r/delta)/r^p with
 *     s1 = erf(rho) - (2/(3 sqrt(pi))) rho (2 rho^2 - 5) e^{-rho^2}
 *     s2 = erf(rho) + (2/(3 sqrt(pi))) rho (2 rho^2 - 3) e^{-rho^2}
 *     s3 = erf(rho) - (2/(3 sqrt(pi))) rho (4 rho^4 - 14 rho^2 + 3) e^{-rho^2}
 *     s4 = erf(rho) - (2/(9 sqrt(pi))) rho (8 rho^6 - 36 rho^4 + 6 rho^2 + 9) e^{-rho^2}
 *   (the four smoothing functions of that section).  The oracle evaluates
 *   the even entire functions F1 = s1/rho, F2 = s2/rho^3, F3 = s3/rho^3,
 *   F4 = s4/rho^5, so that s1/r = F1/delta, s2/r^3 = F2/delta^3,
 *   s3/r^3 = F3/delta^3, s4/r^5 = F4/delta^5, and every sum runs over all j
 *   including j = i (the rho -> 0 limits are finite).
 *
 * Operators (sums over the quadrature of eq. (Quadrature), weights w_j):
 *   LSL   S_L[g]_i = -(1/4pi) sum_j w_j g_j F1/delta                      (Laplace single layer, G = -1/(4 pi r))
 *   LDL   D_L[p]_i = -(1/4pi) sum_j w_j p_j (d.n_j) F2/delta^3            (Laplace double layer, raw)
 *   LDLS  A_D[p]_i = +(1/4pi) sum_j w_j (p_j - p_i)(d.n_j) F2/delta^3     (1/2 p - H p with H of eq. (H_subtr))
 *   SSL   V[f]_i   = (1/(8 pi mu)) sum_j w_j [f_j F1/delta + d (d.f_j) F3/delta^3]   (Stokeslet)
 *   SDL   D_S[u]_i = -(3/4pi) sum_j w_j (u_j.d)(d.n_j) d F4/delta^5       (stresslet, raw)
 *   SDLS  A_S[u]_i = u_i - (3/4pi) sum_j w_j ((u_j-u_i).d)(d.n_j) d F4/delta^5   (1/2 u - K u with K of eq. (K_subtr))
 *
 * Small-rho branch.  The formulas for s_k cancel catastrophically as
 * rho -> 0 (s4 ~ rho^5 from terms of size rho).  Below RHO_SERIES the oracle
 * sums the Taylor series of F_k instead.  Its coefficients follow from the
 * series erf(rho) = (2/sqrt(pi)) sum_n (-1)^n rho^{2n+1} / (n! (2n+1)) and
 * e^{-rho^2} = sum_n (-1)^n rho^{2n} / n!: collecting the coefficient of
 * rho^{2n+1} in each s_k and dividing by rho^p gives, with c = 2/sqrt(pi),
 *   F1 = c sum_m (-1)^m 4 (m+1)(m+2) / (3 (2m+1) m!) rho^{2m}
 *   F2 = c sum_m (-1)^m 4 (m+3)      / (3 (2m+3) m!) rho^{2m}
 *   F3 = c sum_m (-1)^m 8 (m+2)(m+3) / (3 (2m+3) m!) rho^{2m}
 *   F4 = c sum_m (-1)^m 16 (m+3)(m+4)/ (9 (2m+5) m!) rho^{2m}
 * (e.g. F1(0) = 16/(3 sqrt(pi)), F4(0) = 128/(15 sqrt(pi))).
 *
 * Radial derivatives (for the position derivatives of the adjoint):
 *   G_k(rho) = -F_k'(rho)/rho, also even and entire.  Differentiating the
 *   definitions gives G1 = F3 and G3 = 3 F4 (from s3 = s1 - rho s1' and
 *   s4 = s3 - rho s3'/3), and
 *   G2 = 3 s2/rho^5 - c e^{-rho^2} (4 - 4 rho^2/3) / rho^2
 *   G4 = 5 s4/rho^7 - (16 c/9) (rho^4 - 8 rho^2 + 12) e^{-rho^2} / rho^2
 *   with series G_k = -sum_{m>=1} 2 m a_{k,m} rho^{2m-2}.
 *
 * Layouts: points, normals and vector densities are component-major
 * [3][n] (SoA); scalars [n].  Dense matrices are row-major with the same
 * component-major ordering of rows and columns.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define PI 3.14159265358979323846
#define RHO_SERIES 0.6
#define RHO_SERIES_G 1.0

enum { LSL = 0, LDL = 1, LDLS = 2 };
enum { SSL = 0, SDL = 1, SDLS = 2 };

/* rational part R_k(m) of the series coefficient a_{k,m} = c (-1)^m R_k(m)/m! */
static double series_ratio(int k, double m)
{
    switch (k) {
    case 1: return 4.0 * (m + 1) * (m + 2) / (3.0 * (2 * m + 1));
    case 2: return 4.0 * (m + 3) / (3.0 * (2 * m + 3));
    case 3: return 8.0 * (m + 2) * (m + 3) / (3.0 * (2 * m + 3));
    default: return 16.0 * (m + 3) * (m + 4) / (9.0 * (2 * m + 5));
    }
}

/* F_k series: c sum_m (-1)^m R_k(m) rho^{2m}/m!  (deriv = 0);
 * G_k series: -sum_{m>=1} 2m a_{k,m} rho^{2m-2} = c sum_q (-1)^q 2 R_k(q+1) rho^{2q}/q!  (deriv = 1) */
static double series_sum(int k, double rho, int deriv)
{
    const double c = 2.0 / sqrt(PI);
    const double x = rho * rho;
    double pw = 1.0; /* x^m / m! */
    double sum = 0.0;
    for (int m = 0; m < 200; ++m) {
        double term = pw * (deriv ? 2.0 * series_ratio(k, m + 1) : series_ratio(k, m));
        if (m & 1) term = -term;
        sum += term;
        if (m > 2 && fabs(term) < 1e-19 * fabs(sum)) break;
        pw = pw * x / (m + 1);
    }
    return c * sum;
}

/* s_k from the paper's formulas */
static double smooth_s(int k, double rho)
{
    const double c = 2.0 / sqrt(PI);
    const double E = exp(-rho * rho);
    const double r2 = rho * rho;
    const double ef = erf(rho);
    switch (k) {
    case 1: return ef - (c / 3.0) * rho * (2.0 * r2 - 5.0) * E;
    case 2: return ef + (c / 3.0) * rho * (2.0 * r2 - 3.0) * E;
    case 3: return ef - (c / 3.0) * rho * (4.0 * r2 * r2 - 14.0 * r2 + 3.0) * E;
    default: return ef - (c / 9.0) * rho * (8.0 * r2 * r2 * r2 - 36.0 * r2 * r2 + 6.0 * r2 + 9.0) * E;
    }
}

double oracle_s(int k, double rho) { return smooth_s(k, rho); }

double oracle_F(int k, double rho)
{
    if (rho < RHO_SERIES) return series_sum(k, rho, 0);
    const double s = smooth_s(k, rho);
    switch (k) {
    case 1: return s / rho;
    case 2: return s / (rho * rho * rho);
    case 3: return s / (rho * rho * rho);
    default: return s / (rho * rho * rho * rho * rho);
    }
}

double oracle_G(int k, double rho)
{
    if (k == 1) return oracle_F(3, rho);
    if (k == 3) return 3.0 * oracle_F(4, rho);
    if (rho < RHO_SERIES_G) return series_sum(k, rho, 1);
    const double c = 2.0 / sqrt(PI);
    const double E = exp(-rho * rho);
    const double r2 = rho * rho;
    if (k == 2)
        return 3.0 * smooth_s(2, rho) / (r2 * r2 * rho) - c * E * (4.0 - 4.0 * r2 / 3.0) / r2;
    return 5.0 * smooth_s(4, rho) / (r2 * r2 * r2 * rho) - (16.0 * c / 9.0) * (r2 * r2 - 8.0 * r2 + 12.0) * E / r2;
}

/* ------------------------------------------------------------------------ */
/* matrix-free sums over all sources for a list of targets                   */
/* ------------------------------------------------------------------------ */

/* tidx: target indices (NULL = all n targets); out has nt rows (Laplace: [nt],
 * Stokes: [3][nt]). */
void oracle_laplace_apply(int64_t n, const double* x, const double* nrm, const double* w,
                          double delta, int kind, const double* dens,
                          int64_t nt, const int64_t* tidx, double* out)
{
    const double* X = x; const double* Y = x + n; const double* Z = x + 2 * n;
    const double* NX = nrm; const double* NY = nrm + n; const double* NZ = nrm + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = tidx ? tidx[t] : t;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = X[i] - X[j], dy = Y[i] - Y[j], dz = Z[i] - Z[j];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double rho = r / delta;
            if (kind == LSL) {
                acc += w[j] * dens[j] * oracle_F(1, rho) / delta;
            } else {
                const double dn = dx * NX[j] + dy * NY[j] + dz * NZ[j];
                const double k2 = oracle_F(2, rho) / (delta * delta * delta);
                const double dens_j = (kind == LDLS) ? dens[j] - dens[i] : dens[j];
                acc += w[j] * dens_j * dn * k2;
            }
        }
        out[t] = (kind == LDLS ? 1.0 : -1.0) * acc / (4.0 * PI);
    }
}

void oracle_stokes_apply(int64_t n, const double* x, const double* nrm, const double* w,
                         double delta, double mu, int kind, const double* dens,
                         int64_t nt, const int64_t* tidx, double* out)
{
    const double* X = x; const double* Y = x + n; const double* Z = x + 2 * n;
    const double* NX = nrm; const double* NY = nrm + n; const double* NZ = nrm + 2 * n;
    const double* UX = dens; const double* UY = dens + n; const double* UZ = dens + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = tidx ? tidx[t] : t;
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = X[i] - X[j], dy = Y[i] - Y[j], dz = Z[i] - Z[j];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double rho = r / delta;
            if (kind == SSL) {
                const double k1 = oracle_F(1, rho) / delta;
                const double k3 = oracle_F(3, rho) / (delta * delta * delta);
                const double df = dx * UX[j] + dy * UY[j] + dz * UZ[j];
                ax += w[j] * (UX[j] * k1 + dx * df * k3);
                ay += w[j] * (UY[j] * k1 + dy * df * k3);
                az += w[j] * (UZ[j] * k1 + dz * df * k3);
            } else {
                double ux = UX[j], uy = UY[j], uz = UZ[j];
                if (kind == SDLS) { ux -= UX[i]; uy -= UY[i]; uz -= UZ[i]; }
                const double ud = ux * dx + uy * dy + uz * dz;
                const double dn = dx * NX[j] + dy * NY[j] + dz * NZ[j];
                const double k4 = oracle_F(4, rho) / (delta * delta * delta * delta * delta);
                const double c = w[j] * ud * dn * k4;
                ax += c * dx; ay += c * dy; az += c * dz;
            }
        }
        if (kind == SSL) {
            const double s = 1.0 / (8.0 * PI * mu);
            out[t] = s * ax; out[nt + t] = s * ay; out[2 * nt + t] = s * az;
        } else {
            const double s = -3.0 / (4.0 * PI);
            double bx = 0.0, by = 0.0, bz = 0.0;
            if (kind == SDLS) { bx = UX[i]; by = UY[i]; bz = UZ[i]; }
            out[t] = bx + s * ax; out[nt + t] = by + s * ay; out[2 * nt + t] = bz + s * az;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* dense assembly (brute force for small n): out = M dens                   */
/* ------------------------------------------------------------------------ */
void oracle_laplace_matrix(int64_t n, const double* x, const double* nrm, const double* w,
                           double delta, int kind, double* M)
{
    const double* X = x; const double* Y = x + n; const double* Z = x + 2 * n;
    const double* NX = nrm; const double* NY = nrm + n; const double* NZ = nrm + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double* row = M + i * n;
        double diag = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = X[i] - X[j], dy = Y[i] - Y[j], dz = Z[i] - Z[j];
            const double rho = sqrt(dx * dx + dy * dy + dz * dz) / delta;
            double v;
            if (kind == LSL) {
                v = -w[j] * oracle_F(1, rho) / delta / (4.0 * PI);
            } else {
                const double dn = dx * NX[j] + dy * NY[j] + dz * NZ[j];
                v = w[j] * dn * oracle_F(2, rho) / (delta * delta * delta) / (4.0 * PI);
                if (kind == LDL) v = -v;
            }
            row[j] = v;
            diag += v;
        }
        if (kind == LDLS) row[i] -= diag; /* the -p_i part of (p_j - p_i) */
    }
}

void oracle_stokes_matrix(int64_t n, const double* x, const double* nrm, const double* w,
                          double delta, double mu, int kind, double* M)
{
    const double* P[3] = {x, x + n, x + 2 * n};
    const double* Nn[3] = {nrm, nrm + n, nrm + 2 * n};
    const int64_t ld = 3 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double diag[3][3] = {{0}};
        for (int64_t j = 0; j < n; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = P[a][i] - P[a][j];
            const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / delta;
            double blk[3][3];
            if (kind == SSL) {
                const double k1 = oracle_F(1, rho) / delta;
                const double k3 = oracle_F(3, rho) / (delta * delta * delta);
                const double s = w[j] / (8.0 * PI * mu);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        blk[a][b] = s * ((a == b ? k1 : 0.0) + d[a] * d[b] * k3);
            } else {
                const double dn = d[0] * Nn[0][j] + d[1] * Nn[1][j] + d[2] * Nn[2][j];
                const double k4 = oracle_F(4, rho) / (delta * delta * delta * delta * delta);
                const double s = -3.0 / (4.0 * PI) * w[j] * dn * k4;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        blk[a][b] = s * d[a] * d[b];
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    M[(a * n + i) * ld + b * n + j] = blk[a][b];
                    diag[a][b] += blk[a][b];
                }
        }
        if (kind == SDLS) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    M[(a * n + i) * ld + b * n + i] += (a == b ? 1.0 : 0.0) - diag[a][b];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* position derivative of lambda^T F for the coupled system                 */
/* ------------------------------------------------------------------------ */
/* The coupled equations (unknowns pt, u; see oracle.py) are
 *   F1_i = [A_D pt]_i + mean_w(pt) - (mu/K) S_L[v]_i,               v = u.n
 *   F2_i = [A_S u]_i + (flux) n_i + V[f]_i - U,                      f = traction
 * and only the pair sums depend on the node positions (normals and weights
 * are held fixed).  With D = x_i - x_j the pair terms are
 *   T1_ij = (1/4pi) w_j (pt_j - pt_i)(D.n_j) K2 + (mu/K)(1/4pi) w_j v_j K1
 *   T2_ij = -(3/4pi) w_j ((u_j - u_i).D)(D.n_j) D K4 + (1/(8 pi mu)) w_j [f_j K1 + D (D.f_j) K3]
 * with K1 = F1/delta, K2 = F2/delta^3, K3 = F3/delta^3, K4 = F4/delta^5 and
 * grad_D K1 = -(F3/delta^3) D, grad_D K2 = -(G2/delta^5) D,
 * grad_D K3 = -(3 F4/delta^5) D, grad_D K4 = -(G4/delta^7) D.
 * With g_ij = grad_D [lam1_i T1_ij + lam2_i . T2_ij], the derivative of
 * -(lam1.F1 + lam2.F2) with respect to x_m is
 *   grad_m = -sum_j g_mj + sum_i g_im.
 * Arrays: x, nrm, u, f, lam2, grad are [3][n]; pt, v, lam1 are [n]. */
static void pair_grad(int64_t n, const double* x, const double* nrm, const double* w, double delta, double mu,
                      double K, const double* pt, const double* v, const double* u, const double* f,
                      const double* lam1, const double* lam2, int64_t i, int64_t j, double g[3])
{
    double d[3], nj[3], a[3], fj[3], lam[3];
    for (int c = 0; c < 3; ++c) {
        d[c] = x[c * n + i] - x[c * n + j];
        nj[c] = nrm[c * n + j];
        a[c] = u[c * n + j] - u[c * n + i];
        fj[c] = f[c * n + j];
        lam[c] = lam2[c * n + i];
    }
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double rho = r / delta;
    const double d3 = delta * delta * delta, d5 = d3 * delta * delta, d7 = d5 * delta * delta;
    const double K2 = oracle_F(2, rho) / d3, K3 = oracle_F(3, rho) / d3, K4 = oracle_F(4, rho) / d5;
    const double dK1 = -oracle_F(3, rho) / d3;      /* grad K1 = dK1 * D */
    const double dK2 = -oracle_G(2, rho) / d5;
    const double dK3 = -3.0 * oracle_F(4, rho) / d5;
    const double dK4 = -oracle_G(4, rho) / d7;
    const double wj = w[j];
    const double dn = d[0] * nj[0] + d[1] * nj[1] + d[2] * nj[2];
    const double ad = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
    const double ld = lam[0] * d[0] + lam[1] * d[1] + lam[2] * d[2];
    const double df = d[0] * fj[0] + d[1] * fj[1] + d[2] * fj[2];
    const double lf = lam[0] * fj[0] + lam[1] * fj[1] + lam[2] * fj[2];
    const double c_l = 1.0 / (4.0 * PI), c_s = -3.0 / (4.0 * PI), c_v = 1.0 / (8.0 * PI * mu);
    const double dp = pt[j] - pt[i];
    for (int c = 0; c < 3; ++c) {
        double t = 0.0;
        /* Laplace double layer and single layer (weighted by lam1_i) */
        t += lam1[i] * c_l * wj * dp * (nj[c] * K2 + dn * dK2 * d[c]);
        t += lam1[i] * (mu / K) * c_l * wj * v[j] * dK1 * d[c];
        /* stresslet (lam2_i .) */
        t += c_s * wj * (a[c] * dn * ld * K4 + nj[c] * ad * ld * K4 + lam[c] * ad * dn * K4 + ad * dn * ld * dK4 * d[c]);
        /* Stokeslet */
        t += c_v * wj * (lf * dK1 * d[c] + (lam[c] * df + fj[c] * ld) * K3 + ld * df * dK3 * d[c]);
        g[c] = t;
    }
}

void oracle_coupled_xgrad(int64_t n, const double* x, const double* nrm, const double* w, double delta,
                          double mu, double K, const double* pt, const double* v, const double* u,
                          const double* f, const double* lam1, const double* lam2, double* grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < n; ++m) {
        double acc[3] = {0.0, 0.0, 0.0};
        double g[3];
        for (int64_t j = 0; j < n; ++j) {          /* m as target */
            pair_grad(n, x, nrm, w, delta, mu, K, pt, v, u, f, lam1, lam2, m, j, g);
            for (int c = 0; c < 3; ++c) acc[c] -= g[c];
        }
        for (int64_t i = 0; i < n; ++i) {          /* m as source */
            pair_grad(n, x, nrm, w, delta, mu, K, pt, v, u, f, lam1, lam2, i, m, g);
            for (int c = 0; c < 3; ++c) acc[c] += g[c];
        }
        for (int c = 0; c < 3; ++c) grad[c * n + m] = acc[c];
    }
}

int oracle_abi_version(void) { return 1; }

/* threads the OpenMP loops above use */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
#else
int oracle_num_threads(void) { return 1; }
#endif
