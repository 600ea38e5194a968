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
    int64_t n;
    int nsplit;
    int64_t chunk;
    const double* x;    // sorted [3][n]
    const double* nrm;  // sorted [3][n]
    const double* w;    // sorted [n]
    const float* x32;   // sorted [3][n]
    const double* dl_dens;
    const double* sl_dens;
    double c_dl, c_sl, slip_beta;
    double inv_delta;
    double rc2;         // (rho_cut * delta)^2
    double* partial;    // [nsplit][comps][n]
};

template <typename T> __device__ __forceinline__ T load_x(const KArgs& a, int c, int64_t j);
template <> __device__ __forceinline__ double load_x<double>(const KArgs& a, int c, int64_t j) { return a.x[c * a.n + j]; }
template <> __device__ __forceinline__ float load_x<float>(const KArgs& a, int c, int64_t j) { return a.x32[c * a.n + j]; }

// --------------------------------------------------------------------------
// Laplace: DL term c_dl * w_j (q_j - SUB q_i) (D.n_j) s2/r^3, SL term c_sl * w_j g_j s1/r
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB>
__global__ __launch_bounds__(kTPB) void laplace_pairs(KArgs a) {
    __shared__ T sx[kTile], sy[kTile], sz[kTile];
    __shared__ T snx[DL ? kTile : 1], sny[DL ? kTile : 1], snz[DL ? kTile : 1], sq[DL ? kTile : 1];
    __shared__ T sg[SL ? kTile : 1];

    const int split = blockIdx.x % a.nsplit;
    const int64_t i = (int64_t)(blockIdx.x / a.nsplit) * kTPB + threadIdx.x;
    const bool active = i < a.n;
    const int64_t ii = active ? i : a.n - 1;
    const T xi = load_x<T>(a, 0, ii), yi = load_x<T>(a, 1, ii), zi = load_x<T>(a, 2, ii);
    const T qi = (DL && SUB) ? T(a.dl_dens[ii]) : T(0);
    const T id = T(a.inv_delta), id2 = id * id;
    const T rc2 = T(a.rc2);

    double acc = 0.0;
    const int64_t j0 = (int64_t)split * a.chunk;
    const int64_t j1 = j0 + a.chunk < a.n ? j0 + a.chunk : a.n;
    for (int64_t base = j0; base < j1; base += kTile) {
        const int cnt = (int)((j1 - base) < kTile ? (j1 - base) : kTile);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kTPB) {
            const int64_t j = base + t;
            sx[t] = load_x<T>(a, 0, j);
            sy[t] = load_x<T>(a, 1, j);
            sz[t] = load_x<T>(a, 2, j);
            const double wj = a.w[j];
            if (DL) {
                const double s = a.c_dl * wj;
                snx[t] = T(s * a.nrm[j]);
                sny[t] = T(s * a.nrm[a.n + j]);
                snz[t] = T(s * a.nrm[2 * a.n + j]);
                sq[t] = T(a.dl_dens[j]);
            }
            if (SL) sg[t] = T(a.c_sl * wj * a.sl_dens[j]);
        }
        __syncthreads();
        T tacc = T(0);
        for (int jj = 0; jj < cnt; ++jj) {
            const T dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
            const T r2 = dx * dx + dy * dy + dz * dz;
            const T inv_r = rsq(r2);
            T k1 = inv_r, k2 = inv_r * inv_r * inv_r, k3, k4;
            if (r2 < rc2) near_factors<T, SL, DL, false, false>(r2, inv_r, id, id2, k1, k2, k3, k4);
            if (DL) {
                const T dn = dx * snx[jj] + dy * sny[jj] + dz * snz[jj];
                tacc += (sq[jj] - qi) * dn * k2;
            }
            if (SL) tacc += sg[jj] * k1;
        }
        acc += (double)tacc;
    }
    if (active) a.partial[(int64_t)split * a.n + i] = acc;
}

// --------------------------------------------------------------------------
// Stokes: DL term c_dl w_j ((u_j - SUB u_i).D)(D.n_j) D s4/r^5,
//         SL term c_sl w_j [f_j s1/r + D (D.f_j) s3/r^3],
//         f_j = sl_dens_j, or beta (u_j - (u_j.n_j) n_j) when SLIP.
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB, bool SLIP>
__global__ __launch_bounds__(kTPB) void stokes_pairs(KArgs a) {
    constexpr int TD = DL ? kTile : 1;
    constexpr int TS = SL ? kTile : 1;
    __shared__ T sx[kTile], sy[kTile], sz[kTile];
    __shared__ T snx[TD], sny[TD], snz[TD], sux[TD], suy[TD], suz[TD];
    __shared__ T sfx[TS], sfy[TS], sfz[TS];

    const int split = blockIdx.x % a.nsplit;
    const int64_t i = (int64_t)(blockIdx.x / a.nsplit) * kTPB + threadIdx.x;
    const bool active = i < a.n;
    const int64_t ii = active ? i : a.n - 1;
    const int64_t n = a.n;
    const T xi = load_x<T>(a, 0, ii), yi = load_x<T>(a, 1, ii), zi = load_x<T>(a, 2, ii);
    T uix = T(0), uiy = T(0), uiz = T(0);
    if (DL && SUB) {
        uix = T(a.dl_dens[ii]);
        uiy = T(a.dl_dens[n + ii]);
        uiz = T(a.dl_dens[2 * n + ii]);
    }
    const T id = T(a.inv_delta), id2 = id * id;
    const T rc2 = T(a.rc2);

    double ax = 0.0, ay = 0.0, az = 0.0;
    const int64_t j0 = (int64_t)split * a.chunk;
    const int64_t j1 = j0 + a.chunk < n ? j0 + a.chunk : n;
    for (int64_t base = j0; base < j1; base += kTile) {
        const int cnt = (int)((j1 - base) < kTile ? (j1 - base) : kTile);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kTPB) {
            const int64_t j = base + t;
            sx[t] = load_x<T>(a, 0, j);
            sy[t] = load_x<T>(a, 1, j);
            sz[t] = load_x<T>(a, 2, j);
            const double wj = a.w[j];
            const double nx = a.nrm[j], ny = a.nrm[n + j], nz = a.nrm[2 * n + j];
            double ux = 0.0, uy = 0.0, uz = 0.0;
            if (DL || SLIP) {
                ux = a.dl_dens[j];
                uy = a.dl_dens[n + j];
                uz = a.dl_dens[2 * n + j];
            }
            if (DL) {
                const double s = a.c_dl * wj;
                snx[t] = T(s * nx);
                sny[t] = T(s * ny);
                snz[t] = T(s * nz);
                sux[t] = T(ux);
                suy[t] = T(uy);
                suz[t] = T(uz);
            }
            if (SL) {
                double fx, fy, fz;
                if (SLIP) {
                    const double un = ux * nx + uy * ny + uz * nz;
                    fx = a.slip_beta * (ux - un * nx);
                    fy = a.slip_beta * (uy - un * ny);
                    fz = a.slip_beta * (uz - un * nz);
                } else {
                    fx = a.sl_dens[j];
                    fy = a.sl_dens[n + j];
                    fz = a.sl_dens[2 * n + j];
                }
                const double s = a.c_sl * wj;
                sfx[t] = T(s * fx);
                sfy[t] = T(s * fy);
                sfz[t] = T(s * fz);
            }
        }
        __syncthreads();
        T tx = T(0), ty = T(0), tz = T(0);
        for (int jj = 0; jj < cnt; ++jj) {
            const T dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
            const T r2 = dx * dx + dy * dy + dz * dz;
            const T inv_r = rsq(r2);
            const T ir2 = inv_r * inv_r;
            T k1 = inv_r, k2, k3 = inv_r * ir2, k4 = k3 * ir2;
            if (r2 < rc2) near_factors<T, SL, false, SL, DL>(r2, inv_r, id, id2, k1, k2, k3, k4);
            if (DL) {
                const T ux = sux[jj] - uix, uy = suy[jj] - uiy, uz = suz[jj] - uiz;
                const T ud = ux * dx + uy * dy + uz * dz;
                const T dn = dx * snx[jj] + dy * sny[jj] + dz * snz[jj];
                const T c = ud * dn * k4;
                tx += c * dx;
                ty += c * dy;
                tz += c * dz;
            }
            if (SL) {
                const T fx = sfx[jj], fy = sfy[jj], fz = sfz[jj];
                const T c = (dx * fx + dy * fy + dz * fz) * k3;
                tx += fx * k1 + c * dx;
                ty += fy * k1 + c * dy;
                tz += fz * k1 + c * dz;
            }
        }
        ax += (double)tx;
        ay += (double)ty;
        az += (double)tz;
    }
    if (active) {
        double* o = a.partial + (int64_t)split * 3 * n;
        o[i] = ax;
        o[n + i] = ay;
        o[2 * n + i] = az;
    }
}

// out_i = sum_s partial[s][c][i] + base_scale*base + comp_scale*(*comp)*vecfac + add[c]
template <int C>
__global__ void epilogue(int64_t n, int nsplit, const double* __restrict__ partial,
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
        for (int s = 0; s < nsplit; ++s) v += partial[((int64_t)s * C + c) * n + i];
        if (base) v += base_scale * base[c * n + i];
        if (comp) v += cs * (C == 3 ? nrm[c * n + i] : 1.0);
        v += (c == 0 ? add0 : (c == 1 ? add1 : add2));
        out[c * n + o] = v;
    }
}

KArgs make_args(const Plan& P, const PassDesc& d, int nsplit, double cut) {
    KArgs a;
    a.n = P.n;
    a.nsplit = nsplit;
    a.chunk = (P.n + nsplit - 1) / nsplit;
    a.x = P.x;
    a.nrm = P.nrm;
    a.w = P.w;
    a.x32 = P.x32;
    a.dl_dens = d.dl_dens;
    a.sl_dens = d.sl_dens;
    a.c_dl = d.c_dl;
    a.c_sl = d.c_sl;
    a.slip_beta = d.slip_beta;
    a.inv_delta = 1.0 / P.delta;
    a.rc2 = (cut * P.delta) * (cut * P.delta);
    a.partial = P.partial;
    return a;
}

}  // namespace

int choose_splits(int64_t n) {
    const int64_t tblocks = (n + kTPB - 1) / kTPB;
    int64_t s = 8 * ((2048 + 8 * tblocks - 1) / (8 * tblocks));
    if (s > kMaxSplit) s = kMaxSplit;
    while (s > 1 && n / s < 64) s /= 2;
    return (int)(s < 1 ? 1 : s);
}

void launch_laplace_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    const int S = choose_splits(P.n);
    const int64_t tblocks = (P.n + kTPB - 1) / kTPB;
    const dim3 grid((unsigned)(tblocks * S));
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_LAPLACE_F32 : SDBIE_RHO_CUT_LAPLACE_F64;
    const KArgs a = make_args(P, d, S, cut);
#define SDBIE_LAP(T, DL, SL, SUB) hipLaunchKernelGGL((laplace_pairs<T, DL, SL, SUB>), grid, dim3(kTPB), 0, st, a)
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0);
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
    SDBIE_LAUNCHED();
    const double* add = d.add_const;
    hipLaunchKernelGGL((epilogue<1>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P.n, S,
                       (const double*)P.partial, d.base, d.base_scale, d.comp, d.comp_scale,
                       (const double*)P.nrm, add ? add[0] : 0.0, 0.0, 0.0, d.out,
                       d.scatter ? (const int32_t*)P.perm : nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

void launch_stokes_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    const int S = choose_splits(P.n);
    const int64_t tblocks = (P.n + kTPB - 1) / kTPB;
    const dim3 grid((unsigned)(tblocks * S));
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_STOKES_F32 : SDBIE_RHO_CUT_STOKES_F64;
    const KArgs a = make_args(P, d, S, cut);
#define SDBIE_STO(T, DL, SL, SUB, SLIP) \
    hipLaunchKernelGGL((stokes_pairs<T, DL, SL, SUB, SLIP>), grid, dim3(kTPB), 0, st, a)
    const bool slip = d.sl && d.slip_beta != 0.0 && d.sl_dens == nullptr;
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0) | (slip ? 8 : 0);
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
    SDBIE_LAUNCHED();
    const double* add = d.add_const;
    hipLaunchKernelGGL((epilogue<3>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P.n, S,
                       (const double*)P.partial, d.base, d.base_scale, d.comp, d.comp_scale,
                       (const double*)P.nrm, add ? add[0] : 0.0, add ? add[1] : 0.0, add ? add[2] : 0.0,
                       d.out, d.scatter ? (const int32_t*)P.perm : nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

}  // namespace sdbie
