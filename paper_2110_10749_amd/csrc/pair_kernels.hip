// Pair-sum kernels of the regularised layer potentials (gfx950).
//
// Each pass evaluates, for every target i (one per lane) and every source j
// (all nodes, including j = i), the smoothed Laplace or Stokes kernels of
// the paper's section "High-order regularization of kernels on the surface":
//   s1/r, s2/r^3 (Laplace single / double layer),
//   s1/r, s3/r^3 (Stokeslet), s4/r^5 (stresslet),
// weighted by the quadrature weights of eq. (Quadrature), with the
// singularity subtraction of eqs. (H_subtr), (K_subtr) when requested.
//
// Work decomposition: a block of 256 lanes owns 256 consecutive targets (in
// Morton order, so a wave's targets are spatial neighbours and the near-field
// branch is taken by few waves); the source range is cut into `nsplit` equal
// chunks, one per block, with split = blockIdx.x % nsplit so that the
// round-robin dispatch over the 8 XCDs gives each XCD a fixed subset of the
// source chunks (and its L2 only those sources).  Sources are staged through
// LDS in tiles of 256 (every lane then reads the same LDS word: a broadcast).
// Partial sums per split go to a scratch array and an epilogue kernel adds
// them in a fixed order (no atomics: results are bitwise reproducible).
//
// Precision: T = double evaluates everything in double.  T = float evaluates
// pair geometry, smoothing and kernel values in float; each tile's partial sum
// is then added into double accumulators.
//
// Smoothing: for rho = r/delta below SDBIE_RHO_SERIES_* the factors are Taylor
// series in rho^2 (the closed forms cancel there); between that and the far
// cutoff they are the paper's erf/exp formulas; beyond the cutoff every s_k
// equals 1 to within half an ulp of T and the plain 1/r^p kernels are used.
#include "internal.h"
#include "smoothing_coeffs.h"

namespace sdbie {
namespace {

constexpr double kTwoOverSqrtPi = 1.12837916709551257389615890312154517;  // 2/sqrt(pi)
constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ double rsq(double v) { return rsqrt(v); }
__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double erf_t(double v) { return erf(v); }
__device__ __forceinline__ float erf_t(float v) { return erff(v); }
__device__ __forceinline__ double exp_t(double v) { return exp(v); }
__device__ __forceinline__ float exp_t(float v) { return __expf(v); }

template <typename T, int N>
__device__ __forceinline__ T horner(const T (&c)[N], T x) {
    T a = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) a = a * x + c[i];
    return a;
}

__device__ __forceinline__ double ser_F1(double x) { return horner(kF1_F64, x); }
__device__ __forceinline__ double ser_F2(double x) { return horner(kF2_F64, x); }
__device__ __forceinline__ double ser_F3(double x) { return horner(kF3_F64, x); }
__device__ __forceinline__ double ser_F4(double x) { return horner(kF4_F64, x); }
__device__ __forceinline__ float ser_F1(float x) { return horner(kF1_F32, x); }
__device__ __forceinline__ float ser_F2(float x) { return horner(kF2_F32, x); }
__device__ __forceinline__ float ser_F3(float x) { return horner(kF3_F32, x); }
__device__ __forceinline__ float ser_F4(float x) { return horner(kF4_F32, x); }

template <typename T> struct Consts;
template <> struct Consts<double> {
    static constexpr double rho_s2 = SDBIE_RHO_SERIES_F64 * SDBIE_RHO_SERIES_F64;
    static constexpr double cut_lap = SDBIE_RHO_CUT_LAPLACE_F64;
    static constexpr double cut_sto = SDBIE_RHO_CUT_STOKES_F64;
};
template <> struct Consts<float> {
    static constexpr float rho_s2 = SDBIE_RHO_SERIES_F32 * SDBIE_RHO_SERIES_F32;
    static constexpr float cut_lap = SDBIE_RHO_CUT_LAPLACE_F32;
    static constexpr float cut_sto = SDBIE_RHO_CUT_STOKES_F32;
};

// Smoothed kernel factors inside the near field (r < rho_cut delta).
// In: r2 = r^2, inv_r = 1/r (inf at r = 0), id = 1/delta, id2 = id^2.
// Out (only those requested): k1 = s1/r, k2 = s2/r^3, k3 = s3/r^3, k4 = s4/r^5.
template <typename T, bool K1, bool K2, bool K3, bool K4>
__device__ __forceinline__ void near_factors(T r2, T inv_r, T id, T id2, T& k1, T& k2, T& k3, T& k4) {
    const T x = r2 * id2;  // rho^2
    if (x < Consts<T>::rho_s2) {
        const T id3 = id * id2;
        if (K1) k1 = ser_F1(x) * id;
        if (K2) k2 = ser_F2(x) * id3;
        if (K3) k3 = ser_F3(x) * id3;
        if (K4) k4 = ser_F4(x) * id3 * id2;
    } else {
        const T rho = r2 * inv_r * id;
        const T ef = erf_t(rho);
        const T cE = T(kTwoOverSqrtPi) * rho * exp_t(-x);
        const T ir2 = inv_r * inv_r;
        const T third = T(1.0 / 3.0);
        if (K1) k1 = (ef - cE * third * (T(2) * x - T(5))) * inv_r;
        if (K2) k2 = (ef + cE * third * (T(2) * x - T(3))) * inv_r * ir2;
        if (K3) k3 = (ef - cE * third * ((T(4) * x - T(14)) * x + T(3))) * inv_r * ir2;
        if (K4) k4 = (ef - cE * T(1.0 / 9.0) * (((T(8) * x - T(36)) * x + T(6)) * x + T(9))) * inv_r * ir2 * ir2;
    }
}

struct KArgs {
    int64_t n;          // real nodes (targets and sources)
    int64_t npad;       // ntiles * kTile
    int ntiles;
    int nsplit;         // far splits (and near splits)
    int tiles_per_split;
    const double* x;    // padded sorted coordinates [3][npad]
    const double* nrm;  // padded sorted normals [3][npad]
    const double* w;    // padded sorted weights [npad] (0 on padding)
    const float* x32;   // padded sorted coordinates, float [3][npad]
    const uint8_t* mask;  // [ntiles][ntiles] near-field tile pairs
    const double* dl_dens;  // sorted, stride n
    const double* sl_dens;  // sorted, stride n
    double c_dl, c_sl, slip_beta;
    double inv_delta;
    double rc2;         // (rho_cut * delta)^2
    double* partial;    // [2 nsplit][C][n]
    int unit_w;         // sources enter with weight 1 (transposed single layers)
    const double* dl_tgt;  // target density of the subtracted double layer (nullable: dl_dens)
    // position-gradient pass
    const double *g_p, *g_v, *g_u, *g_f, *g_l1, *g_l2;
    double g_mu, g_K;
};

template <typename T> __device__ __forceinline__ T load_x(const KArgs& a, int c, int64_t j);
template <> __device__ __forceinline__ double load_x<double>(const KArgs& a, int c, int64_t j) { return a.x[c * a.npad + j]; }
template <> __device__ __forceinline__ float load_x<float>(const KArgs& a, int c, int64_t j) { return a.x32[c * a.npad + j]; }

__device__ __forceinline__ double dens_at(const double* d, int64_t n, int c, int64_t j) {
    return j < n ? d[c * n + j] : 0.0;
}

__device__ __forceinline__ double src_weight(const KArgs& a, int64_t j) {
    return a.unit_w ? (j < a.n ? 1.0 : 0.0) : a.w[j];
}

// --------------------------------------------------------------------------
// Laplace: DL term c_dl * w_j (q_j - SUB q_i) (D.n_j) s2/r^3, SL term c_sl * w_j g_j s1/r
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB>
struct LaplaceOp {
    static constexpr int C = 1;
    static constexpr int TD = DL ? kTile : 1, TS = SL ? kTile : 1;
    struct Smem {
        T x[kTile], y[kTile], z[kTile];
        T nx[TD], ny[TD], nz[TD], q[TD];
        T g[TS];
    };
    T xi, yi, zi, qi;
    double acc = 0.0;
    T tacc = T(0);

    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        qi = (DL && SUB) ? T(dens_at(a.dl_dens, a.n, 0, i)) : T(0);
    }
    __device__ __forceinline__ void load(Smem& s, int t, int64_t j, const KArgs& a) const {
        s.x[t] = load_x<T>(a, 0, j);
        s.y[t] = load_x<T>(a, 1, j);
        s.z[t] = load_x<T>(a, 2, j);
        const double wj = src_weight(a, j);
        if (DL) {
            const double c = a.c_dl * wj;
            s.nx[t] = T(c * a.nrm[j]);
            s.ny[t] = T(c * a.nrm[a.npad + j]);
            s.nz[t] = T(c * a.nrm[2 * a.npad + j]);
            s.q[t] = T(dens_at(a.dl_dens, a.n, 0, j));
        }
        if (SL) s.g[t] = T(a.c_sl * wj * dens_at(a.sl_dens, a.n, 0, j));
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(const Smem& s, int jj, T id, T id2, T rc2) {
        const T dx = xi - s.x[jj], dy = yi - s.y[jj], dz = zi - s.z[jj];
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T inv_r = rsq(r2);
        T k1 = inv_r, k2 = inv_r * inv_r * inv_r, k3, k4;
        if (NEAR && r2 < rc2) near_factors<T, SL, DL, false, false>(r2, inv_r, id, id2, k1, k2, k3, k4);
        if (DL) {
            const T dn = dx * s.nx[jj] + dy * s.ny[jj] + dz * s.nz[jj];
            tacc += (s.q[jj] - qi) * dn * k2;
        }
        if (SL) tacc += s.g[jj] * k1;
    }
    __device__ __forceinline__ void flush() {
        acc += (double)tacc;
        tacc = T(0);
    }
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        a.partial[(int64_t)slot * a.n + i] = acc;
    }
};

// --------------------------------------------------------------------------
// Stokes: DL term c_dl w_j ((u_j - SUB u_i).D)(D.n_j) D s4/r^5,
//         SL term c_sl w_j [f_j s1/r + D (D.f_j) s3/r^3],
//         f_j = sl_dens_j, or beta (u_j - (u_j.n_j) n_j) when SLIP.
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB, bool SLIP>
struct StokesOp {
    static constexpr int C = 3;
    static constexpr int TD = DL ? kTile : 1, TS = SL ? kTile : 1;
    struct Smem {
        T x[kTile], y[kTile], z[kTile];
        T nx[TD], ny[TD], nz[TD], ux[TD], uy[TD], uz[TD];
        T fx[TS], fy[TS], fz[TS];
    };
    T xi, yi, zi, uix = T(0), uiy = T(0), uiz = T(0);
    double ax = 0.0, ay = 0.0, az = 0.0;
    T tx = T(0), ty = T(0), tz = T(0);

    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        if (DL && SUB) {
            const double* tg = a.dl_tgt ? a.dl_tgt : a.dl_dens;
            uix = T(dens_at(tg, a.n, 0, i));
            uiy = T(dens_at(tg, a.n, 1, i));
            uiz = T(dens_at(tg, a.n, 2, i));
        }
    }
    __device__ __forceinline__ void load(Smem& s, int t, int64_t j, const KArgs& a) const {
        const int64_t np = a.npad;
        s.x[t] = load_x<T>(a, 0, j);
        s.y[t] = load_x<T>(a, 1, j);
        s.z[t] = load_x<T>(a, 2, j);
        const double wj = src_weight(a, j);
        const double nx = a.nrm[j], ny = a.nrm[np + j], nz = a.nrm[2 * np + j];
        double ux = 0.0, uy = 0.0, uz = 0.0;
        if (DL || SLIP) {
            ux = dens_at(a.dl_dens, a.n, 0, j);
            uy = dens_at(a.dl_dens, a.n, 1, j);
            uz = dens_at(a.dl_dens, a.n, 2, j);
        }
        if (DL) {
            const double c = a.c_dl * wj;
            s.nx[t] = T(c * nx);
            s.ny[t] = T(c * ny);
            s.nz[t] = T(c * nz);
            s.ux[t] = T(ux);
            s.uy[t] = T(uy);
            s.uz[t] = T(uz);
        }
        if (SL) {
            double fx, fy, fz;
            if (SLIP) {
                const double un = ux * nx + uy * ny + uz * nz;
                fx = a.slip_beta * (ux - un * nx);
                fy = a.slip_beta * (uy - un * ny);
                fz = a.slip_beta * (uz - un * nz);
            } else {
                fx = dens_at(a.sl_dens, a.n, 0, j);
                fy = dens_at(a.sl_dens, a.n, 1, j);
                fz = dens_at(a.sl_dens, a.n, 2, j);
            }
            const double c = a.c_sl * wj;
            s.fx[t] = T(c * fx);
            s.fy[t] = T(c * fy);
            s.fz[t] = T(c * fz);
        }
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(const Smem& s, int jj, T id, T id2, T rc2) {
        const T dx = xi - s.x[jj], dy = yi - s.y[jj], dz = zi - s.z[jj];
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T inv_r = rsq(r2);
        const T ir2 = inv_r * inv_r;
        T k1 = inv_r, k2, k3 = inv_r * ir2, k4 = k3 * ir2;
        if (NEAR && r2 < rc2) near_factors<T, SL, false, SL, DL>(r2, inv_r, id, id2, k1, k2, k3, k4);
        if (DL) {
            const T ux = s.ux[jj] - uix, uy = s.uy[jj] - uiy, uz = s.uz[jj] - uiz;
            const T ud = ux * dx + uy * dy + uz * dz;
            const T dn = dx * s.nx[jj] + dy * s.ny[jj] + dz * s.nz[jj];
            const T c = ud * dn * k4;
            tx += c * dx;
            ty += c * dy;
            tz += c * dz;
        }
        if (SL) {
            const T fx = s.fx[jj], fy = s.fy[jj], fz = s.fz[jj];
            const T c = (dx * fx + dy * fy + dz * fz) * k3;
            tx += fx * k1 + c * dx;
            ty += fy * k1 + c * dy;
            tz += fz * k1 + c * dz;
        }
    }
    __device__ __forceinline__ void flush() {
        ax += (double)tx;
        ay += (double)ty;
        az += (double)tz;
        tx = ty = tz = T(0);
    }
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        double* o = a.partial + (int64_t)slot * 3 * a.n;
        o[i] = ax;
        o[a.n + i] = ay;
        o[2 * a.n + i] = az;
    }
};

// --------------------------------------------------------------------------
// Transposed double layers (adjoint): the double-layer kernel contracted with
// the TARGET's normal, sources weighted by c_dl (times w_j unless unit_w):
//   Laplace:  out_i = n_i . sum_j c_dl w_j q_j D s2/r^3
//   Stokes:   out_i = sum_j c_dl w_j (D.q_j)(D.n_i) D s4/r^5
// --------------------------------------------------------------------------
template <typename T>
struct LaplaceTNOp {
    static constexpr int C = 1;
    struct Smem {
        T x[kTile], y[kTile], z[kTile], q[kTile];
    };
    T xi, yi, zi, nxi, nyi, nzi;
    double acc = 0.0;
    T tacc = T(0);
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        nxi = T(a.nrm[i]);
        nyi = T(a.nrm[a.npad + i]);
        nzi = T(a.nrm[2 * a.npad + i]);
    }
    __device__ __forceinline__ void load(Smem& s, int t, int64_t j, const KArgs& a) const {
        s.x[t] = load_x<T>(a, 0, j);
        s.y[t] = load_x<T>(a, 1, j);
        s.z[t] = load_x<T>(a, 2, j);
        s.q[t] = T(a.c_dl * src_weight(a, j) * dens_at(a.dl_dens, a.n, 0, j));
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(const Smem& s, int jj, T id, T id2, T rc2) {
        const T dx = xi - s.x[jj], dy = yi - s.y[jj], dz = zi - s.z[jj];
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T inv_r = rsq(r2);
        T k1, k2 = inv_r * inv_r * inv_r, k3, k4;
        if (NEAR && r2 < rc2) near_factors<T, false, true, false, false>(r2, inv_r, id, id2, k1, k2, k3, k4);
        tacc += s.q[jj] * (dx * nxi + dy * nyi + dz * nzi) * k2;
    }
    __device__ __forceinline__ void flush() {
        acc += (double)tacc;
        tacc = T(0);
    }
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        a.partial[(int64_t)slot * a.n + i] = acc;
    }
};

template <typename T>
struct StokesTNOp {
    static constexpr int C = 3;
    struct Smem {
        T x[kTile], y[kTile], z[kTile], qx[kTile], qy[kTile], qz[kTile];
    };
    T xi, yi, zi, nxi, nyi, nzi;
    double ax = 0.0, ay = 0.0, az = 0.0;
    T tx = T(0), ty = T(0), tz = T(0);
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        nxi = T(a.nrm[i]);
        nyi = T(a.nrm[a.npad + i]);
        nzi = T(a.nrm[2 * a.npad + i]);
    }
    __device__ __forceinline__ void load(Smem& s, int t, int64_t j, const KArgs& a) const {
        s.x[t] = load_x<T>(a, 0, j);
        s.y[t] = load_x<T>(a, 1, j);
        s.z[t] = load_x<T>(a, 2, j);
        const double c = a.c_dl * src_weight(a, j);
        s.qx[t] = T(c * dens_at(a.dl_dens, a.n, 0, j));
        s.qy[t] = T(c * dens_at(a.dl_dens, a.n, 1, j));
        s.qz[t] = T(c * dens_at(a.dl_dens, a.n, 2, j));
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(const Smem& s, int jj, T id, T id2, T rc2) {
        const T dx = xi - s.x[jj], dy = yi - s.y[jj], dz = zi - s.z[jj];
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T inv_r = rsq(r2);
        const T ir2 = inv_r * inv_r;
        T k1, k2, k3, k4 = inv_r * ir2 * ir2;
        if (NEAR && r2 < rc2) near_factors<T, false, false, false, true>(r2, inv_r, id, id2, k1, k2, k3, k4);
        const T dq = dx * s.qx[jj] + dy * s.qy[jj] + dz * s.qz[jj];
        const T c = dq * (dx * nxi + dy * nyi + dz * nzi) * k4;
        tx += c * dx;
        ty += c * dy;
        tz += c * dz;
    }
    __device__ __forceinline__ void flush() {
        ax += (double)tx;
        ay += (double)ty;
        az += (double)tz;
        tx = ty = tz = T(0);
    }
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        double* o = a.partial + (int64_t)slot * 3 * a.n;
        o[i] = ax;
        o[a.n + i] = ay;
        o[2 * a.n + i] = az;
    }
};

// --------------------------------------------------------------------------
// Position gradient of lam^T F (adjoint), double only.  See GradDesc.
// G2/delta^5 = -(d/dr K2)/r and G4/delta^7 = -(d/dr K4)/r in the near field.
// --------------------------------------------------------------------------
__device__ __forceinline__ void near_G(double r2, double inv_r, double id, double id2, double& g2, double& g4) {
    const double x = r2 * id2;
    const double id5 = id * id2 * id2;
    if (x < Consts<double>::rho_s2) {
        g2 = horner(kG2_F64, x) * id5;
        g4 = horner(kG4_F64, x) * id5 * id2;
    } else {
        const double rho = r2 * inv_r * id;
        const double ef = erf(rho);
        const double E = exp(-x);
        const double cE = kTwoOverSqrtPi * rho * E;
        const double ir2 = inv_r * inv_r;
        const double s2 = ef + cE * (1.0 / 3.0) * (2.0 * x - 3.0);
        const double s4 = ef - cE * (1.0 / 9.0) * (((8.0 * x - 36.0) * x + 6.0) * x + 9.0);
        const double ir5 = ir2 * ir2 * inv_r;
        g2 = 3.0 * s2 * ir5 - kTwoOverSqrtPi * E * (4.0 - 4.0 * x / 3.0) * ir2 * id * id2;
        g4 = 5.0 * s4 * ir5 * ir2 - (16.0 * kTwoOverSqrtPi / 9.0) * ((x - 8.0) * x + 12.0) * E * ir2 * id5;
    }
}

struct GTgt { double x, y, z, p, ux, uy, uz, l1, lx, ly, lz; };
struct GSrc { double x, y, z, nx, ny, nz, w, p, v, ux, uy, uz, fx, fy, fz; };

__device__ __forceinline__ GTgt load_gtgt(const KArgs& a, int64_t i) {
    GTgt t;
    t.x = a.x[i];
    t.y = a.x[a.npad + i];
    t.z = a.x[2 * a.npad + i];
    t.p = dens_at(a.g_p, a.n, 0, i);
    t.ux = dens_at(a.g_u, a.n, 0, i);
    t.uy = dens_at(a.g_u, a.n, 1, i);
    t.uz = dens_at(a.g_u, a.n, 2, i);
    t.l1 = dens_at(a.g_l1, a.n, 0, i);
    t.lx = dens_at(a.g_l2, a.n, 0, i);
    t.ly = dens_at(a.g_l2, a.n, 1, i);
    t.lz = dens_at(a.g_l2, a.n, 2, i);
    return t;
}

__device__ __forceinline__ GSrc load_gsrc(const KArgs& a, int64_t j) {
    GSrc s;
    s.x = a.x[j];
    s.y = a.x[a.npad + j];
    s.z = a.x[2 * a.npad + j];
    s.nx = a.nrm[j];
    s.ny = a.nrm[a.npad + j];
    s.nz = a.nrm[2 * a.npad + j];
    s.w = a.w[j];
    s.p = dens_at(a.g_p, a.n, 0, j);
    s.v = dens_at(a.g_v, a.n, 0, j);
    s.ux = dens_at(a.g_u, a.n, 0, j);
    s.uy = dens_at(a.g_u, a.n, 1, j);
    s.uz = dens_at(a.g_u, a.n, 2, j);
    s.fx = dens_at(a.g_f, a.n, 0, j);
    s.fy = dens_at(a.g_f, a.n, 1, j);
    s.fz = dens_at(a.g_f, a.n, 2, j);
    return s;
}

template <bool NEAR>
__device__ __forceinline__ void grad_pair(const GTgt& t, const GSrc& s, const KArgs& a, double id, double id2,
                                          double rc2, double& gx, double& gy, double& gz) {
    const double dx = t.x - s.x, dy = t.y - s.y, dz = t.z - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double inv_r = rsqrt(r2);
    const double ir2 = inv_r * inv_r;
    double k1, k2 = inv_r * ir2, k3 = k2, k4 = k2 * ir2;
    double g2 = 3.0 * k4, g4 = 5.0 * k4 * ir2;
    if (NEAR && r2 < rc2) {
        near_factors<double, false, true, true, true>(r2, inv_r, id, id2, k1, k2, k3, k4);
        near_G(r2, inv_r, id, id2, g2, g4);
    }
    // grad_D K1 = -K3 D, grad_D K2 = -g2 D, grad_D K3 = -3 K4 D, grad_D K4 = -g4 D
    const double cl = 1.0 / (4.0 * kPiD), cs = -3.0 / (4.0 * kPiD), cv = 1.0 / (8.0 * kPiD * a.g_mu);
    const double dn = dx * s.nx + dy * s.ny + dz * s.nz;
    const double axv = s.ux - t.ux, ayv = s.uy - t.uy, azv = s.uz - t.uz;
    const double ad = axv * dx + ayv * dy + azv * dz;
    const double ld = t.lx * dx + t.ly * dy + t.lz * dz;
    const double df = dx * s.fx + dy * s.fy + dz * s.fz;
    const double lf = t.lx * s.fx + t.ly * s.fy + t.lz * s.fz;
    const double w = s.w;
    // coefficient of D (radial part) and of the vectors n_j, a, lam, f_j
    const double cD = t.l1 * cl * w * (s.p - t.p) * dn * (-g2) + t.l1 * (a.g_mu / a.g_K) * cl * w * s.v * (-k3) +
                      cs * w * ad * dn * ld * (-g4) + cv * w * (lf * (-k3) + ld * df * (-3.0 * k4));
    const double cN = t.l1 * cl * w * (s.p - t.p) * k2 + cs * w * ad * ld * k4;
    const double cA = cs * w * dn * ld * k4;
    const double cL = cs * w * ad * dn * k4 + cv * w * df * k3;
    const double cF = cv * w * ld * k3;
    gx += cD * dx + cN * s.nx + cA * axv + cL * t.lx + cF * s.fx;
    gy += cD * dy + cN * s.ny + cA * ayv + cL * t.ly + cF * s.fy;
    gz += cD * dz + cN * s.nz + cA * azv + cL * t.lz + cF * s.fz;
}

// SWAP = false: the lane is the target i and the tile holds sources j;
// SWAP = true: the lane is the source j and the tile holds targets i.
template <bool SWAP>
struct GradOp {
    static constexpr int C = 3;
    struct Smem {
        double f[SWAP ? 11 : 15][kTile];
    };
    GTgt t;
    GSrc s;
    double ax = 0.0, ay = 0.0, az = 0.0;
    const KArgs* ap;
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        ap = &a;
        if (SWAP) s = load_gsrc(a, i);
        else t = load_gtgt(a, i);
    }
    __device__ __forceinline__ void load(Smem& sm, int k, int64_t j, const KArgs& a) const {
        if (SWAP) {
            const GTgt q = load_gtgt(a, j);
            const double v[11] = {q.x, q.y, q.z, q.p, q.ux, q.uy, q.uz, q.l1, q.lx, q.ly, q.lz};
#pragma unroll
            for (int f = 0; f < 11; ++f) sm.f[f][k] = v[f];
        } else {
            const GSrc q = load_gsrc(a, j);
            const double v[15] = {q.x, q.y, q.z, q.nx, q.ny, q.nz, q.w, q.p, q.v, q.ux, q.uy, q.uz, q.fx, q.fy, q.fz};
#pragma unroll
            for (int f = 0; f < 15; ++f) sm.f[f][k] = v[f];
        }
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(const Smem& sm, int jj, double id, double id2, double rc2) {
        if (SWAP) {
            GTgt q;
            q.x = sm.f[0][jj]; q.y = sm.f[1][jj]; q.z = sm.f[2][jj]; q.p = sm.f[3][jj];
            q.ux = sm.f[4][jj]; q.uy = sm.f[5][jj]; q.uz = sm.f[6][jj]; q.l1 = sm.f[7][jj];
            q.lx = sm.f[8][jj]; q.ly = sm.f[9][jj]; q.lz = sm.f[10][jj];
            grad_pair<NEAR>(q, s, *ap, id, id2, rc2, ax, ay, az);
        } else {
            GSrc q;
            q.x = sm.f[0][jj]; q.y = sm.f[1][jj]; q.z = sm.f[2][jj];
            q.nx = sm.f[3][jj]; q.ny = sm.f[4][jj]; q.nz = sm.f[5][jj]; q.w = sm.f[6][jj];
            q.p = sm.f[7][jj]; q.v = sm.f[8][jj];
            q.ux = sm.f[9][jj]; q.uy = sm.f[10][jj]; q.uz = sm.f[11][jj];
            q.fx = sm.f[12][jj]; q.fy = sm.f[13][jj]; q.fz = sm.f[14][jj];
            grad_pair<NEAR>(t, q, *ap, id, id2, rc2, ax, ay, az);
        }
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        double* o = a.partial + (int64_t)slot * 3 * a.n;
        o[i] = ax;
        o[a.n + i] = ay;
        o[2 * a.n + i] = az;
    }
};

// Far-field pass: block (b, split) sums target tile b against every tile of
// its split's range whose pairs are all beyond the cutoff (mask 0).  No
// smoothing code is compiled in: every pair uses the plain 1/r^p kernels.
template <class Op, typename T>
__global__ __launch_bounds__(kTPB) void far_pairs(KArgs a) {
    __shared__ typename Op::Smem sm;
    const int split = blockIdx.x % a.nsplit;
    const int b = blockIdx.x / a.nsplit;
    const int64_t i = (int64_t)b * kTPB + threadIdx.x;  // < npad
    Op op;
    op.init(a, i);
    const T id = T(a.inv_delta), id2 = id * id, rc2 = T(a.rc2);
    const int t0 = split * a.tiles_per_split;
    const int t1 = t0 + a.tiles_per_split < a.ntiles ? t0 + a.tiles_per_split : a.ntiles;
    const uint8_t* row = a.mask + (int64_t)b * a.ntiles;
    for (int t = t0; t < t1; ++t) {
        if (row[t]) continue;  // block-uniform
        __syncthreads();
        op.load(sm, threadIdx.x, (int64_t)t * kTile + threadIdx.x, a);
        __syncthreads();
#pragma unroll 8
        for (int jj = 0; jj < kTile; ++jj) op.template pair<false>(sm, jj, id, id2, rc2);
        op.flush();
    }
    if (i < a.n) op.store(a, split, i);
}

// Near-field pass: block (b, split) walks the near tiles of row b (mask 1) in
// order, cut into units of kNearUnit sources, and takes every nsplit-th unit.
template <class Op, typename T>
__global__ __launch_bounds__(kTPB) void near_pairs(KArgs a) {
    __shared__ typename Op::Smem sm;
    const int split = blockIdx.x % a.nsplit;
    const int b = blockIdx.x / a.nsplit;
    const int64_t i = (int64_t)b * kTPB + threadIdx.x;
    Op op;
    op.init(a, i);
    const T id = T(a.inv_delta), id2 = id * id, rc2 = T(a.rc2);
    const uint8_t* row = a.mask + (int64_t)b * a.ntiles;
    constexpr int kUnits = kTile / kNearUnit;
    int rank = 0;
    const int lane = threadIdx.x & 63;
    for (int c0 = 0; c0 < a.ntiles; c0 += 64) {
        const bool f = (c0 + lane < a.ntiles) && row[c0 + lane];
        uint64_t bal = __ballot(f);  // identical in every wave of the block
        while (bal) {
            const int t = c0 + __ffsll((long long)bal) - 1;
            bal &= bal - 1;
            for (int q = 0; q < kUnits; ++q) {
                if ((rank * kUnits + q) % a.nsplit != split) continue;
                __syncthreads();
                if (threadIdx.x < kNearUnit)
                    op.load(sm, threadIdx.x, (int64_t)t * kTile + q * kNearUnit + threadIdx.x, a);
                __syncthreads();
                for (int jj = 0; jj < kNearUnit; ++jj) op.template pair<true>(sm, jj, id, id2, rc2);
                op.flush();
            }
            ++rank;
        }
    }
    if (i < a.n) op.store(a, a.nsplit + split, i);
}

// out_i = sum_s partial[s][c][i] + base_scale*base + comp_scale*(*comp)*vecfac + add[c]
template <int C>
__global__ void epilogue(int64_t n, int nslots, const double* __restrict__ partial,
                         const double* __restrict__ tw,
                         const double* __restrict__ base, double base_scale,
                         const double* __restrict__ comp, double comp_scale,
                         const double* __restrict__ nrm, double add0, double add1, double add2,
                         double* __restrict__ out, const int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cs = comp ? comp_scale * comp[0] : 0.0;
    const int64_t o = perm ? (int64_t)perm[i] : i;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double v = 0.0;
        for (int s = 0; s < nslots; ++s) v += partial[((int64_t)s * C + c) * n + i];
        if (tw) v *= tw[i];
        if (base) v += base_scale * base[c * n + i];
        if (comp) v += cs * (C == 3 ? nrm[c * n + i] : 1.0);
        v += (c == 0 ? add0 : (c == 1 ? add1 : add2));
        out[c * n + o] = v;
    }
}

KArgs make_args(const Plan& P, const PassDesc& d, int nsplit, double cut) {
    KArgs a;
    a.n = P.n;
    a.npad = P.npad;
    a.ntiles = P.ntiles;
    a.nsplit = nsplit;
    a.tiles_per_split = (P.ntiles + nsplit - 1) / nsplit;
    a.x = P.px;
    a.nrm = P.pn;
    a.w = P.pw;
    a.x32 = P.px32;
    a.mask = d.mixed ? P.mask32 : P.mask64;
    a.dl_dens = d.dl_dens;
    a.sl_dens = d.sl_dens;
    a.c_dl = d.c_dl;
    a.c_sl = d.c_sl;
    a.slip_beta = d.slip_beta;
    a.inv_delta = 1.0 / P.delta;
    a.rc2 = (cut * P.delta) * (cut * P.delta);
    a.partial = P.partial;
    a.unit_w = d.unit_src_weight ? 1 : 0;
    a.dl_tgt = d.dl_target;
    a.g_p = a.g_v = a.g_u = a.g_f = a.g_l1 = a.g_l2 = nullptr;
    a.g_mu = a.g_K = 1.0;
    return a;
}

template <class Op, typename T>
void launch_pair_kernels(const KArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.ntiles * a.nsplit));
    hipLaunchKernelGGL((far_pairs<Op, T>), grid, dim3(kTPB), 0, st, a);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL((near_pairs<Op, T>), grid, dim3(kTPB), 0, st, a);
    SDBIE_LAUNCHED();
}

}  // namespace

int choose_splits(int64_t n) {
    const int64_t tblocks = (n + kTPB - 1) / kTPB;
    int64_t s = 8 * ((2048 + 8 * tblocks - 1) / (8 * tblocks));
    if (s > kMaxSplit) s = kMaxSplit;
    while (s > 1 && n / s < 64) s /= 2;
    return (int)(s < 1 ? 1 : s);
}

// The smoothing cutoff rho_cut of a pass is the Stokes one (the larger) for
// both families, matching the tile masks built at staging.
void launch_laplace_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    const int S = choose_splits(P.n);
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_STOKES_F32 : SDBIE_RHO_CUT_STOKES_F64;
    const KArgs a = make_args(P, d, S, cut);
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0);
    if (d.target_normal) {
        if (!d.dl || d.sl || d.sub) throw Error(SDBIE_ERR_ARG, "transposed Laplace pass takes a double layer only");
        ProfScope prof(prof_variant(0, d.mixed, 16 | 1), (double)P.n * (double)P.n, st);
        if (d.mixed) launch_pair_kernels<LaplaceTNOp<float>, float>(a, st);
        else launch_pair_kernels<LaplaceTNOp<double>, double>(a, st);
    } else {
        ProfScope prof(prof_variant(0, d.mixed, d.sl && !d.dl ? 2 : code), (double)P.n * (double)P.n, st);
#define SDBIE_LAP(T, DL, SL, SUB) launch_pair_kernels<LaplaceOp<T, DL, SL, SUB>, T>(a, st)
        if (!d.mixed) {
            switch (code) {
                case 1: SDBIE_LAP(double, true, false, false); break;
                case 5: SDBIE_LAP(double, true, false, true); break;
                case 2: case 6: SDBIE_LAP(double, false, true, false); break;
                case 3: SDBIE_LAP(double, true, true, false); break;
                case 7: SDBIE_LAP(double, true, true, true); break;
                default: throw Error(SDBIE_ERR_ARG, "empty Laplace pass");
            }
        } else {
            switch (code) {
                case 1: SDBIE_LAP(float, true, false, false); break;
                case 5: SDBIE_LAP(float, true, false, true); break;
                case 2: case 6: SDBIE_LAP(float, false, true, false); break;
                case 3: SDBIE_LAP(float, true, true, false); break;
                case 7: SDBIE_LAP(float, true, true, true); break;
                default: throw Error(SDBIE_ERR_ARG, "empty Laplace pass");
            }
        }
#undef SDBIE_LAP
    }
    const double* add = d.add_const;
    hipLaunchKernelGGL((epilogue<1>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P.n, 2 * S,
                       (const double*)P.partial, d.target_weight ? (const double*)P.w : nullptr, d.base,
                       d.base_scale, d.comp, d.comp_scale,
                       (const double*)P.nrm, add ? add[0] : 0.0, 0.0, 0.0, d.out,
                       d.scatter ? (const int32_t*)P.perm : nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

void launch_stokes_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    const int S = choose_splits(P.n);
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_STOKES_F32 : SDBIE_RHO_CUT_STOKES_F64;
    const KArgs a = make_args(P, d, S, cut);
    const bool slip = d.sl && d.slip_beta != 0.0 && d.sl_dens == nullptr;
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0) | (slip ? 8 : 0);
    if (d.target_normal) {
        if (!d.dl || d.sl || d.sub) throw Error(SDBIE_ERR_ARG, "transposed Stokes pass takes a double layer only");
        ProfScope prof(prof_variant(1, d.mixed, 16 | 1), (double)P.n * (double)P.n, st);
        if (d.mixed) launch_pair_kernels<StokesTNOp<float>, float>(a, st);
        else launch_pair_kernels<StokesTNOp<double>, double>(a, st);
    } else {
        ProfScope prof(prof_variant(1, d.mixed, code), (double)P.n * (double)P.n, st);
#define SDBIE_STO(T, DL, SL, SUB, SLIP) launch_pair_kernels<StokesOp<T, DL, SL, SUB, SLIP>, T>(a, st)
        if (!d.mixed) {
            switch (code) {
                case 1: SDBIE_STO(double, true, false, false, false); break;
                case 5: SDBIE_STO(double, true, false, true, false); break;
                case 2: SDBIE_STO(double, false, true, false, false); break;
                case 7: SDBIE_STO(double, true, true, true, false); break;
                case 15: SDBIE_STO(double, true, true, true, true); break;
                default: throw Error(SDBIE_ERR_ARG, "unsupported Stokes pass");
            }
        } else {
            switch (code) {
                case 1: SDBIE_STO(float, true, false, false, false); break;
                case 5: SDBIE_STO(float, true, false, true, false); break;
                case 2: SDBIE_STO(float, false, true, false, false); break;
                case 7: SDBIE_STO(float, true, true, true, false); break;
                case 15: SDBIE_STO(float, true, true, true, true); break;
                default: throw Error(SDBIE_ERR_ARG, "unsupported Stokes pass");
            }
        }
#undef SDBIE_STO
    }
    const double* add = d.add_const;
    hipLaunchKernelGGL((epilogue<3>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P.n, 2 * S,
                       (const double*)P.partial, d.target_weight ? (const double*)P.w : nullptr, d.base,
                       d.base_scale, d.comp, d.comp_scale,
                       (const double*)P.nrm, add ? add[0] : 0.0, add ? add[1] : 0.0, add ? add[2] : 0.0,
                       d.out, d.scatter ? (const int32_t*)P.perm : nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

void launch_grad_pass(const Plan& P, const GradDesc& g, hipStream_t st) {
    const int S = choose_splits(P.n);
    PassDesc d;
    KArgs a = make_args(P, d, S, SDBIE_RHO_CUT_STOKES_F64);
    a.g_p = g.p;
    a.g_v = g.v;
    a.g_u = g.u;
    a.g_f = g.f;
    a.g_l1 = g.lam1;
    a.g_l2 = g.lam2;
    a.g_mu = g.mu;
    a.g_K = g.K;
    const unsigned eb = (unsigned)((P.n + 255) / 256);
    {
        ProfScope prof(prof_variant(2, false, 0), 2.0 * (double)P.n * (double)P.n, st);
        // node as target: A_m = sum_j g_mj
        launch_pair_kernels<GradOp<false>, double>(a, st);
        hipLaunchKernelGGL((epilogue<3>), dim3(eb), dim3(256), 0, st, P.n, 2 * S, (const double*)P.partial,
                           (const double*)nullptr, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0,
                           (const double*)P.nrm, 0.0, 0.0, 0.0, g.out, (const int32_t*)nullptr);
        SDBIE_LAUNCHED();
        // node as source: out = sum_i g_im - A_m
        launch_pair_kernels<GradOp<true>, double>(a, st);
    }
    hipLaunchKernelGGL((epilogue<3>), dim3(eb), dim3(256), 0, st, P.n, 2 * S, (const double*)P.partial,
                       (const double*)nullptr, (const double*)g.out, -1.0, (const double*)nullptr, 0.0,
                       (const double*)P.nrm, 0.0, 0.0, 0.0, g.out, (const int32_t*)nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    Pm.applies_fp64 += 2;
    Pm.pairs += 2.0 * (double)P.n * (double)P.n;
}

}  // namespace sdbie
