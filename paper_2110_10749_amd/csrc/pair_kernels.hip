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
// source chunks (and its L2 only those sources).  The float far-field kernel
// stages source tiles in LDS and reads them back as broadcast loads into
// VGPRs; the other kernels read source records at wave-uniform addresses
// through the scalar cache into SGPRs.
// Partial sums per split go to a scratch array and an epilogue kernel adds
// them in a fixed order (no atomics: results are bitwise reproducible).
//
// Precision: T = double evaluates everything in double.  T = float evaluates
// pair geometry, smoothing and kernel values in float; every 16 terms of a
// lane's sum are then added into its double accumulator.
//
// Smoothing: for rho = r/delta below SDBIE_RHO_SERIES_* the factors are Taylor
// series in rho^2 (the closed forms cancel there); between that and the far
// cutoff they are the paper's erf/exp formulas, with erf = 1 - exp(-rho^2)
// erfcx(rho) and erfcx from a fitted polynomial (no branches inside erf);
// beyond the cutoff every s_k equals 1 to within half an ulp of T and the
// plain 1/r^p kernels are used.
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "internal.h"
#include "smoothing_coeffs.h"

namespace sdbie {
namespace {

// Source records are read through a constant-address-space pointer: they do
// not change during a pass, and loads from that space at wave-uniform
// addresses always become scalar loads into SGPRs.
template <typename T>
using src_ptr = const __attribute__((address_space(4))) T*;

constexpr double kTwoOverSqrtPi = 1.12837916709551257389615890312154517;  // 2/sqrt(pi)
constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ double rsq(double v) { return rsqrt(v); }
__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
// 1/sqrt(v) for finite v > 0 away from the denormal range (far-field r^2):
// the hardware estimate y refined by the second-order expansion of
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - v y^2.  No special cases.
__device__ __forceinline__ double rsq_pos(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    const double e = fma(-v * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float rsq_pos(float v) { return __builtin_amdgcn_rsqf(v); }
// far-field pairs never reach r = 0; near-field pairs do (the self pair)
template <bool NEAR, typename T>
__device__ __forceinline__ T rsq_pair(T v) { return NEAR ? rsq(v) : rsq_pos(v); }
__device__ __forceinline__ float exp_neg(float x) { return __expf(-x); }
// 1/v for v in [1, 4] (no special cases): hardware estimate, two Newton steps in double
__device__ __forceinline__ double rcp_t(double v) {
    double y = __builtin_amdgcn_rcp(v);
    y = fma(fma(-v, y, 1.0), y, y);
    return fma(fma(-v, y, 1.0), y, y);
}
__device__ __forceinline__ float rcp_t(float v) { return __builtin_amdgcn_rcpf(v); }

template <typename T, int N>
__device__ __forceinline__ T horner(const T (&c)[N], T x) {
    T a = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) a = a * x + c[i];
    return a;
}

// Double polynomials: the coefficients are read at the point of use through
// the scalar cache and enter each Horner step as the SGPR addend of one
// v_fma_f64.  Left to itself the compiler keeps every double coefficient of
// the near-field code in VGPRs (about a hundred registers, which caps the
// double near-field kernels at two or three waves per SIMD) and copies each
// one into the accumulator of a v_fmac_f64 with a v_mov_b64, two
// instructions per step.  The empty asm makes the table address opaque, so
// the loads stay at the point of use instead of being hoisted out of the
// source loop into registers.
typedef const __attribute__((address_space(4))) double cdouble;
template <int N>
__device__ __forceinline__ double horner_s(const double (&tab)[N], double x) {
    cdouble* c = (cdouble*)tab;
    asm volatile("" : "+s"(c));
    double a = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) {
        double r;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(x), "s"(c[i]));
        a = r;
    }
    return a;
}

// e^{-x} in double for 0 <= x <= 700: Cody-Waite reduction x = n ln2 + r
// (ln2 split in a double and its remainder, both products taken by fma),
// |r| <= ln2/2, then the degree-13 Taylor polynomial of e^{-r} (truncation
// below 5e-18 relative) and a power-of-two scale.
__device__ static constexpr double kExpTaylor[14] = {
    1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320, 1.0 / 362880,
    1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0};
__device__ __forceinline__ double exp_neg(double x) {
    constexpr double kLog2e = 1.44269504088896340736;
    constexpr double kLn2Hi = 0.693147180559945309417;       // ln 2 rounded to double
    constexpr double kLn2Lo = 2.319046813846299558e-17;      // ln 2 - kLn2Hi
    const double n = rint(x * kLog2e);
    double r = fma(-n, kLn2Hi, x);
    r = fma(-n, kLn2Lo, r);
    return ldexp(horner_s(kExpTaylor, -r), -(int)n);
}

__device__ __forceinline__ double erfcx_fit(double t) { return horner_s(kERFCX_F64, t); }
__device__ __forceinline__ float erfcx_fit(float t) { return horner(kERFCX_F32, t); }
// erf(rho) for rho between the series branch point and the far cutoff, given
// E = exp(-rho^2): erf = 1 - E erfcx(rho), with erfcx from its fitted
// polynomial in t = 1/(1 + p rho) (branch-free; smoothing_coeffs.h)
template <typename T>
__device__ __forceinline__ T erf_near(T rho, T E) {
    const T t = rcp_t(fma(T(SDBIE_ERFCX_P), rho, T(1)));
    return fma(-E, erfcx_fit(t), T(1));
}
__device__ __forceinline__ double ser_F1(double x) { return horner_s(kF1_F64, x); }
__device__ __forceinline__ double ser_F2(double x) { return horner_s(kF2_F64, x); }
__device__ __forceinline__ double ser_F3(double x) { return horner_s(kF3_F64, x); }
__device__ __forceinline__ double ser_F4(double x) { return horner_s(kF4_F64, x); }
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
        const T E = exp_neg(x);
        const T ef = erf_near(rho, E);
        const T cE = T(kTwoOverSqrtPi) * rho * E;
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
    const float* x32;   // padded sorted coordinates, float, in their tile's frame [3][npad]
    const double* tboxes;  // [ntiles][6] tile boxes (min, max per axis); a tile's frame is its box centre
    const uint8_t* mask;  // [ntiles][ntiles] near-field tile pairs
    const double* dl_dens;  // sorted, stride n
    const double* sl_dens;  // sorted, stride n
    double c_dl, c_sl, slip_beta;
    double inv_delta;
    double rc2;         // (rho_cut * delta)^2
    double rcu2;        // (rho_cut * delta)^2 with the tile masks' relative margin (unit box test)
    const double* uboxes;  // [npad / kNearUnit][6] source unit boxes
    double* partial;    // [2 nsplit][C][n]
    void* rec;          // source records of the pass [npad][Op::R] (T)
    int unit_w;         // sources enter with weight 1 (transposed single layers)
    const double* dl_tgt;  // target density of the subtracted double layer (nullable: dl_dens)
    // position-gradient pass
    const double *g_p, *g_v, *g_u, *g_f, *g_l1, *g_l2;
    double g_mu, g_K;
};

template <typename T> __device__ __forceinline__ T load_x(const KArgs& a, int c, int64_t j);
template <> __device__ __forceinline__ double load_x<double>(const KArgs& a, int c, int64_t j) { return a.x[c * a.npad + j]; }
template <> __device__ __forceinline__ float load_x<float>(const KArgs& a, int c, int64_t j) { return a.x32[c * a.npad + j]; }

// Float coordinates are taken in the frame of a tile, the centre of its box: a
// source's in its own tile's (the records), a target's moved into the frame of
// each source tile it meets.  D = x_i - x_j is then formed from numbers about
// as large as the distance to the source tile's centre, not to the body's, so
// the float rounding of the coordinates (eps32 times their size) weighs less
// on the close pairs.  Double coordinates stay absolute.
__device__ __forceinline__ double tile_centre(const KArgs& a, int t, int c) {
    return 0.5 * (a.tboxes[6 * t + 2 * c] + a.tboxes[6 * t + 2 * c + 1]);
}
template <typename T, class Op>
__device__ __forceinline__ void own_frame(const Op& op, T (&x0)[3]) {
    if constexpr (sizeof(T) == 4) {
        x0[0] = op.xi;
        x0[1] = op.yi;
        x0[2] = op.zi;
    }
}
// x0: the target's float coordinates in its own tile's frame (tile tt)
template <typename T, class Op>
__device__ __forceinline__ void targets_to_frame(Op& op, const KArgs& a, const T (&x0)[3], int tt, int t) {
    if constexpr (sizeof(T) == 4) {
        op.xi = x0[0] + (float)(tile_centre(a, tt, 0) - tile_centre(a, t, 0));
        op.yi = x0[1] + (float)(tile_centre(a, tt, 1) - tile_centre(a, t, 1));
        op.zi = x0[2] + (float)(tile_centre(a, tt, 2) - tile_centre(a, t, 2));
    }
}

__device__ __forceinline__ double dens_at(const double* d, int64_t n, int c, int64_t j) {
    return j < n ? d[c * n + j] : 0.0;
}

__device__ __forceinline__ double src_weight(const KArgs& a, int64_t j) {
    return a.unit_w ? (j < a.n ? 1.0 : 0.0) : a.w[j];
}

// Source records.  Before the pair kernels of a pass, one thread per source
// packs what every pair with that source needs (coordinates, weighted normal,
// densities, premultiplied by the quadrature weight and the kernel constant)
// into a record of R elements of T.  The pair kernels read the records at
// wave-uniform addresses, so they arrive through the scalar cache in SGPRs
// and enter the vector ALU as scalar operands: no LDS, no barriers.
// U records (a power of two, at most 128 bytes) are read per unrolled step.
template <typename T, int R>
struct alignas(16) Record {
    T v[R];
};

// records per unrolled step: the largest power of two within 128 bytes (2 for
// the float Stokes matvec, 1 for the double one); for the double kernels 256
// and 512 bytes measured 1% faster and 3% slower
template <typename T, int R>
__host__ __device__ constexpr int unroll_of() {
    int u = 1;
    while (2 * u * R * (int)sizeof(T) <= (sizeof(T) == 8 ? SDBIE_GROUP_BYTES_F64 : SDBIE_GROUP_BYTES_F32)) u *= 2;
    return u;
}

// Pair terms a lane sums in T before it adds the sum into its double
// accumulator (flush()): 16 in float, so the float rounding of the running
// sums stays at the level of the rounding of the terms themselves; a whole
// tile or unit in double, where the running sums are double already.
template <typename T>
__host__ __device__ constexpr int block_terms() { return sizeof(T) == 4 ? 16 : kTile; }

// --------------------------------------------------------------------------
// Laplace: DL term c_dl * w_j (q_j - SUB q_i) (D.n_j) s2/r^3, SL term c_sl * w_j g_j s1/r
// record: x y z q | nx ny nz g   (SL only: x y z g); n and g carry c w_j
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB>
struct LaplaceOp {
    static constexpr int C = 1;
    static constexpr int R = DL ? 8 : 4;
    static constexpr int U = unroll_of<T, R>();
    static constexpr int Q = 3, NX = 4, NY = 5, NZ = 6, G = DL ? 7 : 3;
    T xi, yi, zi, qi;
    double acc = 0.0;
    T tacc = T(0);

    __device__ __forceinline__ static void pack(T* r, int64_t j, const KArgs& a) {
        r[0] = load_x<T>(a, 0, j);
        r[1] = load_x<T>(a, 1, j);
        r[2] = load_x<T>(a, 2, j);
        const double wj = src_weight(a, j);
        if (DL) {
            const double c = a.c_dl * wj;
            r[NX] = T(c * a.nrm[j]);
            r[NY] = T(c * a.nrm[a.npad + j]);
            r[NZ] = T(c * a.nrm[2 * a.npad + j]);
            r[Q] = T(dens_at(a.dl_dens, a.n, 0, j));
        }
        r[G] = SL ? T(a.c_sl * wj * dens_at(a.sl_dens, a.n, 0, j)) : T(0);
    }
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        qi = (DL && SUB) ? T(dens_at(a.dl_dens, a.n, 0, i)) : T(0);
    }
    template <bool NEAR, class P>
    __device__ __forceinline__ void pair(P r, T id, T id2, T rc2) {
        const T dx = xi - r[0], dy = yi - r[1], dz = zi - r[2];
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T inv_r = rsq_pair<NEAR>(r2);
        T k1 = inv_r, k2 = inv_r * inv_r * inv_r, k3, k4;
        if (NEAR && r2 < rc2) near_factors<T, SL, DL, false, false>(r2, inv_r, id, id2, k1, k2, k3, k4);
        if (DL) {
            const T dn = fma(dx, r[NX], fma(dy, r[NY], dz * r[NZ]));
            tacc = fma((r[Q] - qi) * dn, k2, tacc);
        }
        if (SL) tacc = fma(r[G], k1, tacc);
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
// record: x y z nx | ny nz ux uy | uz fx fy fz   (SL only: x y z fx | fy fz 0 0)
// The two terms along D share one coefficient: acc += f k1 + (cDL + cSL) D.
// --------------------------------------------------------------------------
template <typename T, bool DL, bool SL, bool SUB, bool SLIP>
struct StokesOp {
    static constexpr int C = 3;
    static constexpr int R = DL ? 12 : 8;
    static constexpr int U = unroll_of<T, R>();
    static constexpr int NX = 3, NY = 4, NZ = 5, UX = 6, UY = 7, UZ = 8;
    static constexpr int FX = DL ? 9 : 3, FY = FX + 1, FZ = FX + 2;
    T xi, yi, zi, uix = T(0), uiy = T(0), uiz = T(0);
    double ax = 0.0, ay = 0.0, az = 0.0;
    T tx = T(0), ty = T(0), tz = T(0);

    __device__ __forceinline__ static void pack(T* r, int64_t j, const KArgs& a) {
        const int64_t np = a.npad;
        r[0] = load_x<T>(a, 0, j);
        r[1] = load_x<T>(a, 1, j);
        r[2] = load_x<T>(a, 2, j);
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
            r[NX] = T(c * nx);
            r[NY] = T(c * ny);
            r[NZ] = T(c * nz);
            r[UX] = T(ux);
            r[UY] = T(uy);
            r[UZ] = T(uz);
        } else {
            r[6] = r[7] = T(0);  // padding of the single-layer record
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
            r[FX] = T(c * fx);
            r[FY] = T(c * fy);
            r[FZ] = T(c * fz);
        } else {
            r[FX] = r[FY] = r[FZ] = T(0);
        }
    }
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
    template <bool NEAR, class P>
    __device__ __forceinline__ void pair(P r, T id, T id2, T rc2) {
        const T dx = xi - r[0], dy = yi - r[1], dz = zi - r[2];
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T inv_r = rsq_pair<NEAR>(r2);
        const T ir2 = inv_r * inv_r;
        if constexpr (!NEAR && SL) {
            // unsmoothed kernels: 1/r comes out of the sum,
            //   acc += (1/r) [f + D (1/r^2) ((u.D)(D.n)/r^2 + D.f)]
            // two multiplies fewer per pair than with k1, k3, k4 apart
            const T fx = r[FX], fy = r[FY], fz = r[FZ];
            T c = fma(dx, fx, fma(dy, fy, dz * fz));
            if (DL) {
                const T ux = r[UX] - uix, uy = r[UY] - uiy, uz = r[UZ] - uiz;
                const T ud = fma(ux, dx, fma(uy, dy, uz * dz));
                const T dn = fma(dx, r[NX], fma(dy, r[NY], dz * r[NZ]));
                c = fma(ud * dn, ir2, c);
            }
            c *= ir2;
            tx = fma(fma(c, dx, fx), inv_r, tx);
            ty = fma(fma(c, dy, fy), inv_r, ty);
            tz = fma(fma(c, dz, fz), inv_r, tz);
            return;
        }
        T k1 = inv_r, k2, k3 = inv_r * ir2, k4 = k3 * ir2;
        if (NEAR && r2 < rc2) near_factors<T, SL, false, SL, DL>(r2, inv_r, id, id2, k1, k2, k3, k4);
        T cd = T(0);
        if (DL) {
            const T ux = r[UX] - uix, uy = r[UY] - uiy, uz = r[UZ] - uiz;
            const T ud = fma(ux, dx, fma(uy, dy, uz * dz));
            const T dn = fma(dx, r[NX], fma(dy, r[NY], dz * r[NZ]));
            cd = ud * dn * k4;
        }
        if (SL) {
            const T fx = r[FX], fy = r[FY], fz = r[FZ];
            cd = fma(fma(dx, fx, fma(dy, fy, dz * fz)), k3, cd);
            tx = fma(fx, k1, tx);
            ty = fma(fy, k1, ty);
            tz = fma(fz, k1, tz);
        }
        tx = fma(cd, dx, tx);
        ty = fma(cd, dy, ty);
        tz = fma(cd, dz, tz);
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
// Transposed double layers (adjoint): the normal is the target's and the
// density carries the source weight factor.
//   Laplace:  out_i = sum_j c w_j q_j (D.n_i) s2/r^3       record: x y z cwq
//   Stokes:   out_i = sum_j c w_j (q_j.D)(D.n_i) D s4/r^5  record: x y z cwqx | cwqy cwqz 0 0
// --------------------------------------------------------------------------
template <typename T>
struct LaplaceTNOp {
    static constexpr int C = 1;
    static constexpr int R = 4;
    static constexpr int U = unroll_of<T, R>();
    T xi, yi, zi, nxi, nyi, nzi;
    double acc = 0.0;
    T tacc = T(0);
    __device__ __forceinline__ static void pack(T* r, int64_t j, const KArgs& a) {
        r[0] = load_x<T>(a, 0, j);
        r[1] = load_x<T>(a, 1, j);
        r[2] = load_x<T>(a, 2, j);
        r[3] = T(a.c_dl * src_weight(a, j) * dens_at(a.dl_dens, a.n, 0, j));
    }
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        nxi = T(a.nrm[i]);
        nyi = T(a.nrm[a.npad + i]);
        nzi = T(a.nrm[2 * a.npad + i]);
    }
    template <bool NEAR, class P>
    __device__ __forceinline__ void pair(P r, T id, T id2, T rc2) {
        const T dx = xi - r[0], dy = yi - r[1], dz = zi - r[2];
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T inv_r = rsq_pair<NEAR>(r2);
        T k1, k2 = inv_r * inv_r * inv_r, k3, k4;
        if (NEAR && r2 < rc2) near_factors<T, false, true, false, false>(r2, inv_r, id, id2, k1, k2, k3, k4);
        const T dn = fma(dx, nxi, fma(dy, nyi, dz * nzi));
        tacc = fma(r[3] * dn, k2, tacc);
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
    static constexpr int R = 8;
    static constexpr int U = unroll_of<T, R>();
    T xi, yi, zi, nxi, nyi, nzi;
    double ax = 0.0, ay = 0.0, az = 0.0;
    T tx = T(0), ty = T(0), tz = T(0);
    __device__ __forceinline__ static void pack(T* r, int64_t j, const KArgs& a) {
        r[0] = load_x<T>(a, 0, j);
        r[1] = load_x<T>(a, 1, j);
        r[2] = load_x<T>(a, 2, j);
        const double c = a.c_dl * src_weight(a, j);
        r[3] = T(c * dens_at(a.dl_dens, a.n, 0, j));
        r[4] = T(c * dens_at(a.dl_dens, a.n, 1, j));
        r[5] = T(c * dens_at(a.dl_dens, a.n, 2, j));
        r[6] = r[7] = T(0);
    }
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        nxi = T(a.nrm[i]);
        nyi = T(a.nrm[a.npad + i]);
        nzi = T(a.nrm[2 * a.npad + i]);
    }
    template <bool NEAR, class P>
    __device__ __forceinline__ void pair(P r, T id, T id2, T rc2) {
        const T dx = xi - r[0], dy = yi - r[1], dz = zi - r[2];
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T inv_r = rsq_pair<NEAR>(r2);
        const T ir2 = inv_r * inv_r;
        T k1, k2, k3, k4 = inv_r * ir2 * ir2;
        if (NEAR && r2 < rc2) near_factors<T, false, false, false, true>(r2, inv_r, id, id2, k1, k2, k3, k4);
        const T dq = fma(dx, r[3], fma(dy, r[4], dz * r[5]));
        const T c = dq * fma(dx, nxi, fma(dy, nyi, dz * nzi)) * k4;
        tx = fma(c, dx, tx);
        ty = fma(c, dy, ty);
        tz = fma(c, dz, tz);
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

// Transposed stresslet and transposed Stokeslet of one density (the adjoint's
// transposed Stokes operator with slip), from one record and one rsqrt:
//   out_i  = sum_j c_dl (q_j.D)(D.n_i) D s4/r^5
//   out2_i = sum_j c_sl [q_j s1/r + D (D.q_j) s3/r^3]
// (unit source weights), stored as six components [out | out2].
template <typename T>
struct StokesTNSLOp {
    static constexpr int C = 6;
    static constexpr int R = 8;
    static constexpr int U = unroll_of<T, R>();
    T xi, yi, zi, nxi, nyi, nzi;
    double ax = 0.0, ay = 0.0, az = 0.0, bx = 0.0, by = 0.0, bz = 0.0, sl_scale = 0.0;
    T tx = T(0), ty = T(0), tz = T(0), sx = T(0), sy = T(0), sz = T(0);
    __device__ __forceinline__ static void pack(T* r, int64_t j, const KArgs& a) { StokesTNOp<T>::pack(r, j, a); }
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        xi = load_x<T>(a, 0, i);
        yi = load_x<T>(a, 1, i);
        zi = load_x<T>(a, 2, i);
        nxi = T(a.nrm[i]);
        nyi = T(a.nrm[a.npad + i]);
        nzi = T(a.nrm[2 * a.npad + i]);
        sl_scale = a.c_sl / a.c_dl;  // the record carries c_dl q
    }
    template <bool NEAR, class P>
    __device__ __forceinline__ void pair(P r, T id, T id2, T rc2) {
        const T dx = xi - r[0], dy = yi - r[1], dz = zi - r[2];
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T inv_r = rsq_pair<NEAR>(r2);
        const T ir2 = inv_r * inv_r;
        T k1 = inv_r, k2, k3 = inv_r * ir2, k4 = k3 * ir2;
        if (NEAR && r2 < rc2) near_factors<T, true, false, true, true>(r2, inv_r, id, id2, k1, k2, k3, k4);
        const T dq = fma(dx, r[3], fma(dy, r[4], dz * r[5]));
        const T c = dq * fma(dx, nxi, fma(dy, nyi, dz * nzi)) * k4;
        tx = fma(c, dx, tx);
        ty = fma(c, dy, ty);
        tz = fma(c, dz, tz);
        const T cs = dq * k3;
        sx = fma(r[3], k1, fma(cs, dx, sx));
        sy = fma(r[4], k1, fma(cs, dy, sy));
        sz = fma(r[5], k1, fma(cs, dz, sz));
    }
    __device__ __forceinline__ void flush() {
        ax += (double)tx;
        ay += (double)ty;
        az += (double)tz;
        bx += (double)sx;
        by += (double)sy;
        bz += (double)sz;
        tx = ty = tz = sx = sy = sz = T(0);
    }
    __device__ __forceinline__ void store(const KArgs& a, int slot, int64_t i) const {
        double* o = a.partial + (int64_t)slot * 6 * a.n;
        o[i] = ax;
        o[a.n + i] = ay;
        o[2 * a.n + i] = az;
        o[3 * a.n + i] = sl_scale * bx;
        o[4 * a.n + i] = sl_scale * by;
        o[5 * a.n + i] = sl_scale * bz;
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
        g2 = horner_s(kG2_F64, x) * id5;
        g4 = horner_s(kG4_F64, x) * id5 * id2;
    } else {
        const double rho = r2 * inv_r * id;
        const double E = exp_neg(x);
        const double ef = erf_near(rho, E);
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
    const double inv_r = rsq_pair<NEAR>(r2);
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

// SWAP = false: the lane is the target i and the records are sources j;
// SWAP = true: the lane is the source j and the records are targets i.
// record (double): the GSrc fields (15, padded to 16) or the GTgt fields (11, padded to 12)
template <bool SWAP>
struct GradOp {
    static constexpr int C = 3;
    static constexpr int R = SWAP ? 12 : 16;
    static constexpr int U = unroll_of<double, R>();
    GTgt t;
    GSrc s;
    double ax = 0.0, ay = 0.0, az = 0.0;
    const KArgs* ap;
    __device__ __forceinline__ static void pack(double* r, int64_t j, const KArgs& a) {
        if (SWAP) {
            const GTgt q = load_gtgt(a, j);
            const double v[12] = {q.x, q.y, q.z, q.p, q.ux, q.uy, q.uz, q.l1, q.lx, q.ly, q.lz, 0.0};
#pragma unroll
            for (int f = 0; f < 12; ++f) r[f] = v[f];
        } else {
            const GSrc q = load_gsrc(a, j);
            const double v[16] = {q.x, q.y, q.z, q.nx, q.ny, q.nz, q.w, q.p, q.v, q.ux, q.uy, q.uz,
                                  q.fx, q.fy, q.fz, 0.0};
#pragma unroll
            for (int f = 0; f < 16; ++f) r[f] = v[f];
        }
    }
    __device__ __forceinline__ void init(const KArgs& a, int64_t i) {
        ap = &a;
        if (SWAP) s = load_gsrc(a, i);
        else t = load_gtgt(a, i);
    }
    template <bool NEAR>
    __device__ __forceinline__ void pair(src_ptr<double> r, double id, double id2, double rc2) {
        if (SWAP) {
            GTgt q;
            q.x = r[0]; q.y = r[1]; q.z = r[2]; q.p = r[3];
            q.ux = r[4]; q.uy = r[5]; q.uz = r[6]; q.l1 = r[7];
            q.lx = r[8]; q.ly = r[9]; q.lz = r[10];
            grad_pair<NEAR>(q, s, *ap, id, id2, rc2, ax, ay, az);
        } else {
            GSrc q;
            q.x = r[0]; q.y = r[1]; q.z = r[2];
            q.nx = r[3]; q.ny = r[4]; q.nz = r[5]; q.w = r[6];
            q.p = r[7]; q.v = r[8];
            q.ux = r[9]; q.uy = r[10]; q.uz = r[11];
            q.fx = r[12]; q.fy = r[13]; q.fz = r[14];
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

static_assert(GradOp<false>::R * sizeof(double) <= kRecBytes, "record larger than its workspace slot");

// One thread per source (padding included): write the pass's source records.
template <class Op, typename T>
__global__ __launch_bounds__(256) void pack_sources(KArgs a) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.npad) return;
    Record<T, Op::R> rec;
    Op::pack(rec.v, j, a);
    reinterpret_cast<Record<T, Op::R>*>(a.rec)[j] = rec;
}

// NU consecutive records starting at r (wave-uniform address)
template <class Op, typename T, bool NEAR, int NU>
__device__ __forceinline__ void pair_group(Op& op, src_ptr<T> r, T id, T id2, T rc2) {
#pragma unroll
    for (int u = 0; u < NU; ++u) op.template pair<NEAR>(r + u * Op::R, id, id2, rc2);
}

// Far-field pass: block (b, split) sums target tile b against every tile of
// its split's range whose pairs are all beyond the cutoff (mask 0).  No
// smoothing code is compiled in: every pair uses the plain 1/r^p kernels.
template <class Op, typename T>
__device__ __forceinline__ void far_body(const KArgs& a, int blk) {
    static_assert(kTile % Op::U == 0, "unroll must divide the tile");
    const int split = blk % a.nsplit;
    const int b = blk / a.nsplit;
    const int64_t i = (int64_t)b * kTPB + threadIdx.x;  // < npad
    Op op;
    op.init(a, i);
    T x0[3] = {};
    own_frame<T>(op, x0);
    const T id = T(a.inv_delta), id2 = id * id, rc2 = T(a.rc2);
    const int t0 = split * a.tiles_per_split;
    const int t1 = t0 + a.tiles_per_split < a.ntiles ? t0 + a.tiles_per_split : a.ntiles;
    const uint8_t* row = a.mask + (int64_t)b * a.ntiles;
    const src_ptr<T> rec = (src_ptr<T>)a.rec;
    constexpr int B = block_terms<T>();
    static_assert(kTile % B == 0 && B % Op::U == 0, "blocks of whole unrolled steps");
    for (int t = t0; t < t1; ++t) {
        if (row[t]) continue;  // uniform
        targets_to_frame<T>(op, a, x0, b, t);
        const src_ptr<T> rt = rec + (int64_t)t * kTile * Op::R;
#pragma unroll 1
        for (int jb = 0; jb < kTile; jb += B) {
#pragma unroll 1
            for (int jj = jb; jj < jb + B; jj += Op::U)
                pair_group<Op, T, false, Op::U>(op, rt + jj * Op::R, id, id2, rc2);
            op.flush();
        }
    }
    if (i < a.n) op.store(a, split, i);
}

template <class Op, typename T>
__global__ __launch_bounds__(kTPB) void far_pairs(KArgs a) {
    far_body<Op, T>(a, blockIdx.x);
}

// Far-field pass in float: the block stages each source tile in LDS (one
// record per thread, coalesced; the next tile is loaded into registers while
// the current one is summed) and every wave reads the records back as
// broadcast LDS loads into VGPRs.  Float VALU instructions whose operands
// are all VGPRs issue at twice the rate of those that read an SGPR, so this
// form beats scalar-cache records once half the pair's instructions would
// read one.
template <class Op>
__device__ __forceinline__ void far_lds_body(const KArgs& a, int blk) {
    using T = float;
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int R = Op::R, Q = R / 4;
    static_assert(R % 4 == 0, "records of whole float4s");
    static_assert(kTile == kTPB, "one record per thread when staging a tile");
    static_assert(kTile % Op::U == 0, "unroll must divide the tile");
    __shared__ f4 tile[kTile * Q];
    const int split = blk % a.nsplit;
    const int b = blk / a.nsplit;
    const int64_t i = (int64_t)b * kTPB + threadIdx.x;  // < npad
    Op op;
    op.init(a, i);
    T x0[3] = {};
    own_frame<T>(op, x0);
    const T id = T(a.inv_delta), id2 = id * id, rc2 = T(a.rc2);
    const int t0 = split * a.tiles_per_split;
    const int t1 = t0 + a.tiles_per_split < a.ntiles ? t0 + a.tiles_per_split : a.ntiles;
    const uint8_t* row = a.mask + (int64_t)b * a.ntiles;
    const f4* rec = static_cast<const f4*>(a.rec);
    int t = t0;
    while (t < t1 && row[t]) ++t;  // uniform
    f4 pf[Q];
    const f4* g = rec + (int64_t)(t < t1 ? t : 0) * kTile * Q + threadIdx.x;
#pragma unroll
    for (int c = 0; c < Q; ++c) pf[c] = g[c * kTPB];
    while (t < t1) {
        __syncthreads();  // every wave is done with the previous tile
#pragma unroll
        for (int c = 0; c < Q; ++c) tile[threadIdx.x + c * kTPB] = pf[c];
        __syncthreads();
        int tn = t + 1;
        while (tn < t1 && row[tn]) ++tn;
        // the next tile's records (this one's again after the last)
        g = rec + (int64_t)(tn < t1 ? tn : t) * kTile * Q + threadIdx.x;
#pragma unroll
        for (int c = 0; c < Q; ++c) pf[c] = g[c * kTPB];
        targets_to_frame<T>(op, a, x0, b, t);
        constexpr int B = block_terms<T>();
        static_assert(kTile % B == 0 && B % Op::U == 0, "blocks of whole unrolled steps");
#pragma unroll 1
        for (int jb = 0; jb < kTile; jb += B) {
#pragma unroll 1
            for (int jj = jb; jj < jb + B; jj += Op::U) {
#pragma unroll
                for (int u = 0; u < Op::U; ++u) {
                    T r[R];
#pragma unroll
                    for (int c = 0; c < Q; ++c) {
                        const f4 v = tile[(jj + u) * Q + c];
                        r[4 * c] = v[0];
                        r[4 * c + 1] = v[1];
                        r[4 * c + 2] = v[2];
                        r[4 * c + 3] = v[3];
                    }
                    op.template pair<false>(static_cast<const T*>(r), id, id2, rc2);
                }
            }
            op.flush();
        }
        t = tn;
    }
    if (i < a.n) op.store(a, split, i);
}

template <class Op>
__global__ __launch_bounds__(kTPB) void far_pairs_lds(KArgs a) {
    far_lds_body<Op>(a, blockIdx.x);
}

// Near-field pass: the tiles of the target tile's mask row, cut into units of
// kNearUnit sources dealt round-robin to the splits.  A (wave, unit) pair
// whose boxes are at least the cutoff apart (and which holds no padding node)
// runs the plain far-field body; every other pair takes the smoothing branch
// when r < rho_cut delta.
template <class Op, typename T>
__device__ __forceinline__ void near_body(const KArgs& a, int blk) {
    // the double smoothing branch is long: one record per step keeps its registers in bounds
    constexpr int NU = sizeof(T) == 8 ? 1 : Op::U;
    // far units: half the far kernel's unroll (the near kernel holds more scalars)
    constexpr int FU = Op::U > 1 ? Op::U / 2 : 1;
    static_assert(kNearUnit % NU == 0 && kNearUnit % FU == 0, "unroll must divide the near unit");
    static_assert(kNearUnit == 64, "one wave of targets per unit test");
    constexpr int B = block_terms<T>() < kNearUnit ? block_terms<T>() : kNearUnit;
    static_assert(kNearUnit % B == 0 && B % NU == 0 && B % FU == 0, "blocks of whole unrolled steps");
    const int split = blk % a.nsplit;
    const int b = blk / a.nsplit;
    const int64_t i = (int64_t)b * kTPB + threadIdx.x;
    Op op;
    op.init(a, i);
    T x0[3] = {};
    own_frame<T>(op, x0);
    const T id = T(a.inv_delta), id2 = id * id, rc2 = T(a.rc2);
    // bounding box of the wave's 64 targets (equal in every lane)
    const int64_t w0 = (int64_t)b * kTPB + (threadIdx.x & ~63);
    const bool wave_full = w0 + 64 <= a.n;
    double wb[6];
    for (int c = 0; c < 3; ++c) {
        double lo = a.x[c * a.npad + i], hi = lo;
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off));
            hi = fmax(hi, __shfl_xor(hi, off));
        }
        wb[2 * c] = lo;
        wb[2 * c + 1] = hi;
    }
    const uint8_t* row = a.mask + (int64_t)b * a.ntiles;
    const src_ptr<T> rec = (src_ptr<T>)a.rec;
    constexpr int kUnits = kTile / kNearUnit;
    int rank = 0;
    const int lane = threadIdx.x & 63;
    for (int c0 = 0; c0 < a.ntiles; c0 += 64) {
        const bool f = (c0 + lane < a.ntiles) && row[c0 + lane];
        uint64_t bal = __ballot(f);  // uniform
        while (bal) {
            const int t = c0 + __ffsll((long long)bal) - 1;
            bal &= bal - 1;
            targets_to_frame<T>(op, a, x0, b, t);
            for (int q = 0; q < kUnits; ++q) {
                if ((rank * kUnits + q) % a.nsplit != split) continue;
                const int64_t u0 = (int64_t)t * kTile + q * kNearUnit;
                const src_ptr<T> ru = rec + u0 * Op::R;
                bool far_unit = wave_full && u0 + kNearUnit <= a.n;
                if (far_unit) {
                    const src_ptr<double> ub = (src_ptr<double>)a.uboxes + (u0 / kNearUnit) * 6;
                    double d2 = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        const double gap = fmax(0.0, fmax(wb[2 * c] - ub[2 * c + 1], ub[2 * c] - wb[2 * c + 1]));
                        d2 += gap * gap;
                    }
                    far_unit = d2 >= a.rcu2;
                }
#pragma unroll 1
                for (int jb = 0; jb < kNearUnit; jb += B) {
                    if (far_unit) {
#pragma unroll 1
                        for (int jj = jb; jj < jb + B; jj += FU)
                            pair_group<Op, T, false, FU>(op, ru + jj * Op::R, id, id2, rc2);
                    } else {
#pragma unroll 1
                        for (int jj = jb; jj < jb + B; jj += NU)
                            pair_group<Op, T, true, NU>(op, ru + jj * Op::R, id, id2, rc2);
                    }
                    op.flush();
                }
            }
            ++rank;
        }
    }
    if (i < a.n) op.store(a, a.nsplit + split, i);
}

template <class Op, typename T>
__global__ __launch_bounds__(kTPB) void near_pairs(KArgs a) {
    near_body<Op, T>(a, blockIdx.x);
}

// Far and near blocks of one pass in a single launch: blocks [0, T S) run the
// far-field body, blocks [T S, 2 T S) the near-field one.  The far blocks are
// dispatched first and the near blocks fill the CUs as the far ones drain, so
// the pass does not wait for the far launch's last wave before the near work
// starts.  Both write disjoint partial slots.  The register count of a
// launch is that of its larger body: the same for the float passes; the
// double passes are held to 8 waves per SIMD (pass_pairs below).
template <class Op>
__global__ __launch_bounds__(kTPB) void pass_pairs_lds(KArgs a) {
    const int nfar = a.ntiles * a.nsplit;
    if ((int)blockIdx.x < nfar) far_lds_body<Op>(a, blockIdx.x);
    else near_body<Op, float>(a, (int)blockIdx.x - nfar);
}

// Scalar-cache records (the double passes).  The double near body alone
// would take 76 VGPRs (6 waves per SIMD); held to 8 waves per SIMD the
// compiler keeps 64 and spills a few words outside the pair loops, and the
// double passes run 3-4% faster.  The position-gradient passes hold far more
// state and keep their registers.
template <class Op, typename T>
__global__ __launch_bounds__(kTPB) __attribute__((amdgpu_waves_per_eu(8))) void pass_pairs(KArgs a) {
    const int nfar = a.ntiles * a.nsplit;
    if ((int)blockIdx.x < nfar) far_body<Op, T>(a, blockIdx.x);
    else near_body<Op, T>(a, (int)blockIdx.x - nfar);
}

// The same without the wave target (position-gradient passes).
template <class Op, typename T>
__global__ __launch_bounds__(kTPB) void pass_pairs_wide(KArgs a) {
    const int nfar = a.ntiles * a.nsplit;
    if ((int)blockIdx.x < nfar) far_body<Op, T>(a, blockIdx.x);
    else near_body<Op, T>(a, (int)blockIdx.x - nfar);
}

// Sum the 2 nsplit partial slots of each target in a fixed order, then
//   out = tw * sum + base_scale * base + comp_scale * comp[0] * (1 or n_i) + add
// out may alias base when perm is null (each lane reads its own elements before
// writing them).
// Epilogues run 32 targets per block with 8 threads each: thread group g adds
// the partial slots g, g + 8, g + 16, ... of its target, and the 8 group sums
// are added in group order (a fixed order: results are bitwise reproducible).
// One thread per target left one block per CU and the slot loads
// latency-bound.
constexpr int kEpiTargets = 32, kEpiGroups = 8, kEpiThreads = kEpiTargets * kEpiGroups;

// the group sums of v[0..C) for the block's targets, added in group order
// into the g == 0 threads' v (the other threads' v are left as they are)
template <int C>
__device__ __forceinline__ void epi_combine(double (&v)[C], int g, int jj) {
    __shared__ double red[kEpiGroups][C][kEpiTargets];
#pragma unroll
    for (int c = 0; c < C; ++c) red[g][c][jj] = v[c];
    __syncthreads();
    if (g != 0) return;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kEpiGroups; ++k) s += red[k][c][jj];
        v[c] = s;
    }
}

// the terms a pass adds to its pair sums v (target weight, base vector,
// completion, constant) and the store in the caller's node order
template <int C>
__device__ __forceinline__ void epi_finish(int64_t n, int64_t i, const double (&v)[C],
                                           const double* __restrict__ tw, const double* base, double base_scale,
                                           const double* __restrict__ comp, double comp_scale,
                                           const double* __restrict__ nrm, double add0, double add1, double add2,
                                           double* out, const int32_t* __restrict__ perm) {
    const double cs = comp ? comp_scale * comp[0] : 0.0;
    const int64_t o = perm ? (int64_t)perm[i] : i;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double s = v[c];
        if (tw) s *= tw[i];
        if (base) s += base_scale * base[c * n + i];
        if (comp) s += cs * (C == 3 ? nrm[c * n + i] : 1.0);
        s += (c == 0 ? add0 : (c == 1 ? add1 : add2));
        out[c * n + o] = s;
    }
}

template <int C>
__global__ __launch_bounds__(kEpiThreads) void epilogue(int64_t n, int nslots, const double* __restrict__ partial,
                                                        const double* __restrict__ tw, const double* base,
                                                        double base_scale, const double* __restrict__ comp,
                                                        double comp_scale, const double* __restrict__ nrm,
                                                        double add0, double add1, double add2, double* out,
                                                        const int32_t* __restrict__ perm) {
    const int g = threadIdx.x / kEpiTargets, jj = threadIdx.x % kEpiTargets;
    const int64_t i = (int64_t)blockIdx.x * kEpiTargets + jj;
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = 0.0;
    if (i < n)
        for (int sl = g; sl < nslots; sl += kEpiGroups)
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] += partial[((int64_t)sl * C + c) * n + i];
    epi_combine<C>(v, g, jj);
    if (g == 0 && i < n) epi_finish<C>(n, i, v, tw, base, base_scale, comp, comp_scale, nrm, add0, add1, add2, out, perm);
}

// --------------------------------------------------------------------------
// Target-source symmetric far field.  The pair kernels are even (single
// layers) or odd (double layers) in D = x_i - x_j, so the two ordered pairs of
// one unordered pair share the geometry (D, r, 1/r) and most of the kernel
// algebra; the paper's CPU code halves its pair work this way.  Here each far
// tile pair {a, b} (a < b, every pair beyond the cutoff) is evaluated once:
// every lane of a block holds one target of tile a and, in turn, one source
// of tile b.  Within a wave the sources rotate across the 16 lanes of each
// row: at step K lane l meets the source of lane (l - K) mod 16, its fields
// read from the tile staged in LDS at that index (SymSrc; fields can also be
// taken by DPP row rotations of the lane's own record), so at every step each lane
// evaluates one pair, adds the forward contribution to its own target and
// hands the reverse one back to the source's lane through the inverse
// rotation.  A wave meets its 64
// targets with a quarter of the 256 sources per phase (4 row rotations of 16
// steps); the quarters' reverse sums pass between the waves in LDS, as double
// sums to which each row rotation adds its 16 terms.
// Forward sums of the target tile go to one slot per block, reverse sums of
// the source tile to one slot per tile pair; the symmetric epilogue adds them
// (and the near-field slots) in a fixed order.
// --------------------------------------------------------------------------

// lane l of a 16-lane row reads lane (l - K) mod 16 of the same row (DPP
// row_ror:K; K = 0 reads itself).  rot<K> and rot<16 - K> are inverse
// permutations whichever way the hardware rotates, which is all the
// symmetric pass relies on.  A rotation reads a valid lane everywhere, so the
// bound control is set and no old value needs to be kept in the destination.
template <int K>
__device__ __forceinline__ float rot(float v) {
    if constexpr (K == 0) {
        return v;
    } else {
        return __builtin_bit_cast(
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + K, 0xf, 0xf, true));
    }
}
template <int K>
__device__ __forceinline__ double rot(double v) {
    if constexpr (K == 0) {
        return v;
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x120 + K, 0xf, 0xf, true);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x120 + K, 0xf, 0xf, true);
        return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}

// The source record a lane meets at step K of a row rotation: the record of
// lane (l - K) mod 16 of its 16-lane row.  Fields whose bit is set in DPP
// come from the lane's own record by a DPP rotation (a VALU operand, issued
// at half rate); the others are read from the tile staged in LDS at the
// rotated index (the LDS pipe, not the VALU).  lds: field f of source j at
// lds[f * kTile + j]; jb: first source of the lane's row; l16: lane in row.
template <typename T, int R, unsigned DPP>
struct SymSrc {
    const T* lds;
    int jb, l16;
    T own[R];
    template <int K, int F>
    __device__ __forceinline__ T get() const {
        if constexpr ((DPP >> F) & 1u) return rot<K>(own[F]);
        else return lds[F * kTile + jb + ((l16 - K) & 15)];
    }
};

// One step of the symmetric Laplace far field: the lane's target t against
// the source of the lane K places back in its row (its record read through
// rot<K>).  Forward (into acc, target t): c_dl w_s (q_s - SUB q_t)(D.n_s) / r^3
// + c_sl w_s g_s / r; reverse (returned, for source s): the same kernels with
// D -> -D and the roles swapped, (q_s - q_t)(D.n_t) / r^3 (SUB) or -q_t
// (D.n_t) / r^3, plus c_sl w_t g_t / r.  Records as LaplaceOp's.
template <typename T, bool DL, bool SL, bool SUB>
struct SymLaplace {
    using Op = LaplaceOp<T, DL, SL, SUB>;
    static constexpr int C = 1, R = Op::R;
    static constexpr int kFamilyBit = SDBIE_SYM_LAPLACE;
    static constexpr int Q = Op::Q, NX = Op::NX, NY = Op::NY, NZ = Op::NZ, G = Op::G;
    template <int K, class Src>
    __device__ __forceinline__ static void step(const T (&tr)[R], const Src& sr, T (&acc)[C], T (&racc)[C]) {
        const T dx = tr[0] - sr.template get<K, 0>();
        const T dy = tr[1] - sr.template get<K, 1>();
        const T dz = tr[2] - sr.template get<K, 2>();
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T ir = rsq_pos(r2);
        T f = T(0), rv = T(0);
        if constexpr (DL) {
            const T k2 = ir * ir * ir;
            const T dns =
                fma(dx, sr.template get<K, NX>(), fma(dy, sr.template get<K, NY>(), dz * sr.template get<K, NZ>()));
            const T dnt = fma(dx, tr[NX], fma(dy, tr[NY], dz * tr[NZ]));
            const T qs = sr.template get<K, Q>();
            if constexpr (SUB) {
                const T dq = (qs - tr[Q]) * k2;
                f = dq * dns;
                rv = dq * dnt;
            } else {
                f = qs * dns * k2;
                rv = -tr[Q] * dnt * k2;
            }
        }
        if constexpr (SL) {
            f = fma(sr.template get<K, G>(), ir, f);
            rv = fma(tr[G], ir, rv);
        }
        acc[0] += f;
        racc[0] += rot<(16 - K) & 15>(rv);
    }
};

// One step of the symmetric Stokes far field (records as StokesOp's: n and f
// carry c w of their node, u does not).  With D' = -D and ud' = (u_t - SUB
// u_s).D' the reverse terms are those of the forward ones with the target's
// fields: the stresslet ud' (D'.n_t) D' / r^5 = ud' (D.n_t) D / r^5 and the
// Stokeslet [f_t + D (D.f_t) / r^2] / r; with both, 1/r is factored out as in
// StokesOp.  ud' = ud with the subtraction, -(u_t.D) without it.
template <typename T, bool DL, bool SL, bool SUB, bool SLIP>
struct SymStokes {
    using Op = StokesOp<T, DL, SL, SUB, SLIP>;
    static constexpr int C = 3, R = Op::R;
    static constexpr int kFamilyBit = SDBIE_SYM_STOKES;
    static constexpr int NX = Op::NX, NY = Op::NY, NZ = Op::NZ, UX = Op::UX, UY = Op::UY, UZ = Op::UZ;
    static constexpr int FX = Op::FX, FY = Op::FY, FZ = Op::FZ;
    template <int K, class Src>
    __device__ __forceinline__ static void step(const T (&tr)[R], const Src& sr, T (&acc)[C], T (&racc)[C]) {
        const T dx = tr[0] - sr.template get<K, 0>();
        const T dy = tr[1] - sr.template get<K, 1>();
        const T dz = tr[2] - sr.template get<K, 2>();
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const T ir = rsq_pos(r2);
        const T ir2 = ir * ir;
        T ud = T(0), udr = T(0), dns = T(0), dnt = T(0);
        if constexpr (DL) {
            const T ux = sr.template get<K, UX>() - (SUB ? tr[UX] : T(0));
            const T uy = sr.template get<K, UY>() - (SUB ? tr[UY] : T(0));
            const T uz = sr.template get<K, UZ>() - (SUB ? tr[UZ] : T(0));
            ud = fma(ux, dx, fma(uy, dy, uz * dz));
            udr = SUB ? ud : -fma(tr[UX], dx, fma(tr[UY], dy, tr[UZ] * dz));
            dns = fma(dx, sr.template get<K, NX>(), fma(dy, sr.template get<K, NY>(), dz * sr.template get<K, NZ>()));
            dnt = fma(dx, tr[NX], fma(dy, tr[NY], dz * tr[NZ]));
        }
        T rc[3];
        if constexpr (SL) {
            // (1/r) [f + D (1/r^2) ((u.D)(D.n)/r^2 + D.f)] in each direction: 1/r
            // multiplies the sum, not each of its terms
            const T fsx = sr.template get<K, FX>(), fsy = sr.template get<K, FY>(), fsz = sr.template get<K, FZ>();
            const T dfs = fma(dx, fsx, fma(dy, fsy, dz * fsz));
            const T dft = fma(dx, tr[FX], fma(dy, tr[FY], dz * tr[FZ]));
            const T ef = (DL ? fma(ud * dns, ir2, dfs) : dfs) * ir2;
            const T er = (DL ? fma(udr * dnt, ir2, dft) : dft) * ir2;
            acc[0] = fma(fma(ef, dx, fsx), ir, acc[0]);
            acc[1] = fma(fma(ef, dy, fsy), ir, acc[1]);
            acc[2] = fma(fma(ef, dz, fsz), ir, acc[2]);
            rc[0] = fma(er, dx, tr[FX]) * ir;
            rc[1] = fma(er, dy, tr[FY]) * ir;
            rc[2] = fma(er, dz, tr[FZ]) * ir;
        } else {
            const T k4 = ir * ir2 * ir2;
            const T cf = ud * dns * k4, cr = udr * dnt * k4;
            acc[0] = fma(cf, dx, acc[0]);
            acc[1] = fma(cf, dy, acc[1]);
            acc[2] = fma(cf, dz, acc[2]);
            rc[0] = cr * dx;
            rc[1] = cr * dy;
            rc[2] = cr * dz;
        }
        racc[0] += rot<(16 - K) & 15>(rc[0]);
        racc[1] += rot<(16 - K) & 15>(rc[1]);
        racc[2] += rot<(16 - K) & 15>(rc[2]);
    }
};

template <class Op> struct SymOf { using type = void; };
template <typename T, bool DL, bool SL, bool SUB>
struct SymOf<LaplaceOp<T, DL, SL, SUB>> { using type = SymLaplace<T, DL, SL, SUB>; };
template <typename T, bool DL, bool SL, bool SUB, bool SLIP>
struct SymOf<StokesOp<T, DL, SL, SUB, SLIP>> { using type = SymStokes<T, DL, SL, SUB, SLIP>; };

// the 16 steps of one row rotation, K = 0 .. 15 (compile-time DPP controls)
template <class Sym, typename T, int K>
struct SymSteps {
    template <class Src>
    __device__ __forceinline__ static void run(const T (&tr)[Sym::R], const Src& sr, T (&acc)[Sym::C],
                                               T (&racc)[Sym::C]) {
        Sym::template step<K>(tr, sr, acc, racc);
        SymSteps<Sym, T, K + 1>::run(tr, sr, acc, racc);
    }
};
template <class Sym, typename T>
struct SymSteps<Sym, T, 16> {
    template <class Src>
    __device__ __forceinline__ static void run(const T (&)[Sym::R], const Src&, T (&)[Sym::C], T (&)[Sym::C]) {}
};

// Source fields a symmetric step takes by DPP rotation (bit f: field f; the
// rest by indexed LDS reads).  A DPP operand costs the VALU half an issue slot
// more per use; an LDS read costs LDS bandwidth (64 lanes x 4 bytes per field
// and step) and no VALU slot.  Measured at h = 1/64 (ms per launch, float
// Stokes single layer / double layer / Laplace double layer): every field by
// DPP 2.24 / 2.48 / 1.59, the coordinates by DPP 1.92 / 1.96 / 1.45, every
// field from LDS 1.80 / 1.92 / 1.39 (the mixed solve 116.5 ms against 119.4 ms
// with the coordinates by DPP); a double rotation is two DPP moves.  Every
// field comes from LDS by default; the reverse sums still rotate by DPP.
#ifndef SDBIE_SYM_DPP_F32
#define SDBIE_SYM_DPP_F32 0x0u
#endif
#ifndef SDBIE_SYM_DPP_F64
#define SDBIE_SYM_DPP_F64 0x0u
#endif
template <typename T>
constexpr unsigned sym_dpp_fields() { return sizeof(T) == 4 ? SDBIE_SYM_DPP_F32 : SDBIE_SYM_DPP_F64; }

struct SymArgs {
    int nblocks;
    const int32_t* items;   // [npairs][3]: target tile a, source tile b, pair index p
    const int32_t* blocks;  // [nblocks][2]: first item, item count
    double* fwd;            // [nblocks][C][kTile]
    void* rev;              // [npairs][C][kTile] of T
};

template <class Sym, typename T>
__device__ __forceinline__ void sym_far_body(const KArgs& a, const SymArgs& sa, int blk) {
    constexpr int R = Sym::R, C = Sym::C;
    static_assert(kTile == kTPB && kTile == 256, "one target and one staged source per thread, four waves");
    static_assert(block_terms<T>() >= 16, "a row rotation of 16 steps sums in T");
    __shared__ T srec[R * kTile];  // the source tile, field-major: field f of source j at srec[f * kTile + j]
    __shared__ double sracc[C * kTile];  // reverse sums of the tile pair, one 16-step rotation at a time
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int first = sa.blocks[2 * blk], cnt = sa.blocks[2 * blk + 1];
    const int ta = sa.items[3 * first];
    const T* rec = static_cast<const T*>(a.rec);
    T tr[R];
#pragma unroll
    for (int f = 0; f < R; ++f) tr[f] = rec[((int64_t)ta * kTile + tid) * R + f];
    const T x0[3] = {tr[0], tr[1], tr[2]};  // the targets in their own tile's frame
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    T* rev = static_cast<T*>(sa.rev);
    constexpr unsigned DPP = sym_dpp_fields<T>();
    SymSrc<T, R, DPP> src;
    src.lds = srec;
    src.l16 = lane & 15;
    for (int it = first; it < first + cnt; ++it) {
        const int tb = sa.items[3 * it + 1], p = sa.items[3 * it + 2];
        if constexpr (sizeof(T) == 4) {  // the targets in the source tile's frame
#pragma unroll
            for (int c = 0; c < 3; ++c) tr[c] = x0[c] + (float)(tile_centre(a, ta, c) - tile_centre(a, tb, c));
        }
        __syncthreads();  // the previous tile pair is done with the LDS
#pragma unroll
        for (int f = 0; f < R; ++f) srec[f * kTile + tid] = rec[((int64_t)tb * kTile + tid) * R + f];
#pragma unroll
        for (int c = 0; c < C; ++c) sracc[c * kTile + tid] = 0.0;
        __syncthreads();
#pragma unroll 1
        for (int ph = 0; ph < 4; ++ph) {
            const int q = (wave + ph) & 3;  // the four waves take the four quarters of the sources
#pragma unroll 1
            for (int rr = 0; rr < 4; ++rr) {
                // row r of the wave holds row (r + rr) mod 4 of the quarter
                src.jb = 64 * q + ((((lane >> 4) + rr) & 3) << 4);
                const int j = src.jb + src.l16;
#pragma unroll
                for (int f = 0; f < R; ++f)
                    if ((DPP >> f) & 1u) src.own[f] = srec[f * kTile + j];
                T facc[C], racc[C];
#pragma unroll
                for (int c = 0; c < C; ++c) facc[c] = racc[c] = T(0);
                SymSteps<Sym, T, 0>::run(tr, src, facc, racc);
                // 16 terms of each sum in T, then into the double sums
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += (double)facc[c];
                    sracc[c * kTile + j] += (double)racc[c];
                }
            }
            __syncthreads();  // each quarter's reverse sums go to the wave that takes it next
        }
#pragma unroll
        for (int c = 0; c < C; ++c) rev[((int64_t)p * C + c) * kTile + tid] = T(sracc[c * kTile + tid]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sa.fwd[((int64_t)blk * C + c) * kTile + tid] = acc[c];
}

// symmetric far blocks first, then the near-field blocks of the pass.  Left
// alone, the compiler hoists the LDS reads of a whole row rotation ahead of
// its 16 steps (up to 134 VGPRs, 3 waves per SIMD for the float Laplace double
// layer); the float passes are held to 8 waves per SIMD.
template <class Op, class Sym, typename T>
__global__ __launch_bounds__(kTPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1)))
void sym_pass_pairs(KArgs a, SymArgs sa) {
    if ((int)blockIdx.x < sa.nblocks) sym_far_body<Sym, T>(a, sa, blockIdx.x);
    else near_body<Op, T>(a, (int)blockIdx.x - sa.nblocks);
}

// Sum of the symmetric pass per target, in a fixed order, then the terms of
// epilogue(): the forward slots of its tile's blocks, the reverse slots of the
// far tile pairs with its tile as the source tile (about T/2 of them), the
// near-field split slots; each kind split over the 8 thread groups of the
// target as in epilogue().
template <int C, typename RT>
__global__ __launch_bounds__(kEpiThreads) void sym_epilogue(
    int64_t n, const int32_t* __restrict__ fwd_start, const double* __restrict__ fwd,
    const int32_t* __restrict__ rev_start, const RT* __restrict__ rev, int nsplit,
    const double* __restrict__ partial, const double* __restrict__ tw, const double* base, double base_scale,
    const double* __restrict__ comp, double comp_scale, const double* __restrict__ nrm, double add0, double add1,
    double add2, double* out, const int32_t* __restrict__ perm) {
    static_assert(kTile % kEpiTargets == 0, "a block's targets lie in one tile");
    const int g = threadIdx.x / kEpiTargets, jj = threadIdx.x % kEpiTargets;
    const int64_t i = (int64_t)blockIdx.x * kEpiTargets + jj;
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = 0.0;
    if (i < n) {
        const int64_t t = i / kTile, j = i % kTile;
        const int b1 = fwd_start[t + 1], p1 = rev_start[t + 1];
        for (int b = fwd_start[t] + g; b < b1; b += kEpiGroups)
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] += fwd[((int64_t)b * C + c) * kTile + j];
        for (int p = rev_start[t] + g; p < p1; p += kEpiGroups)
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] += (double)rev[((int64_t)p * C + c) * kTile + j];
        for (int sl = g; sl < nsplit; sl += kEpiGroups)
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] += partial[((int64_t)(nsplit + sl) * C + c) * n + i];
    }
    epi_combine<C>(v, g, jj);
    if (g == 0 && i < n) epi_finish<C>(n, i, v, tw, base, base_scale, comp, comp_scale, nrm, add0, add1, add2, out, perm);
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
    a.tboxes = P.boxes;
    a.mask = d.mixed ? P.mask32 : P.mask64;
    a.dl_dens = d.dl_dens;
    a.sl_dens = d.sl_dens;
    a.c_dl = d.c_dl;
    a.c_sl = d.c_sl;
    a.slip_beta = d.slip_beta;
    a.inv_delta = 1.0 / P.delta;
    a.rc2 = (cut * P.delta) * (cut * P.delta);
    a.rcu2 = (cut * P.delta * (1.0 + 1e-6)) * (cut * P.delta * (1.0 + 1e-6));
    a.uboxes = P.uboxes;
    a.partial = P.partial;
    a.rec = P.rec;
    a.unit_w = d.unit_src_weight ? 1 : 0;
    a.dl_tgt = d.dl_target;
    a.g_p = a.g_v = a.g_u = a.g_f = a.g_l1 = a.g_l2 = nullptr;
    a.g_mu = a.g_K = 1.0;
    return a;
}

template <class Op>
struct family_is_gradient { static constexpr bool value = false; };
template <bool SWAP>
struct family_is_gradient<GradOp<SWAP>> { static constexpr bool value = true; };

// pack and pair kernels of one pass, each timed on its own when kernel timing
// is on (pairs: all N^2 for a pass kernel; with separate far and near
// launches, the real-node pairs of the far / near tile pairs)
// Returns true when the far field ran target-source symmetric (the sums then
// need sym_epilogue).
template <class Op, typename T>
bool launch_pair_kernels(const Plan& P, const KArgs& a, hipStream_t st, int family, int code, bool mixed) {
    static_assert(Op::R * sizeof(T) <= kRecBytes, "record larger than its workspace slot");
    if (Op::C > P.max_comps) throw Error(SDBIE_ERR_ARG, "this workspace holds no partial slots for that pass");
    const double all = (double)P.n * (double)P.n;
    const double near = mixed ? P.near_pairs32 : P.near_pairs64;
    {
        ProfScope prof(prof_variant(family, mixed, code, 2), 0.0, st);
        hipLaunchKernelGGL((pack_sources<Op, T>), dim3((unsigned)(a.npad / 256)), dim3(256), 0, st, a);
        SDBIE_LAUNCHED();
    }
    using Sym = typename SymOf<Op>::type;
    if constexpr (!std::is_same<Sym, void>::value) {
        const int k = mixed ? 1 : 0;
        const int kind = mixed ? Sym::kFamilyBit : Sym::kFamilyBit << 2;  // SDBIE_SYM_* of this pass
        if ((P.symmetric & kind) && P.sym_items[k] && P.sym_nblocks[k] > 0 && !a.dl_tgt) {
            SymArgs sa;
            sa.nblocks = P.sym_nblocks[k];
            sa.items = P.sym_items[k];
            sa.blocks = P.sym_blocks[k];
            sa.fwd = P.sym_fwd;
            sa.rev = P.sym_rev;
            ProfScope prof(prof_variant(family, mixed, code, 4), all, st);
            hipLaunchKernelGGL((sym_pass_pairs<Op, Sym, T>), dim3((unsigned)(sa.nblocks + a.ntiles * a.nsplit)),
                               dim3(kTPB), 0, st, a, sa);
            SDBIE_LAUNCHED();
            return true;
        }
    }
    const dim3 grid((unsigned)((int64_t)a.ntiles * a.nsplit));
    if constexpr (SDBIE_ONE_LAUNCH) {
        // far and near blocks in one launch (timed as one kernel, all N^2 pairs)
        ProfScope prof(prof_variant(family, mixed, code, 3), all, st);
        if constexpr (sizeof(T) == 4 && SDBIE_FAR_LDS)
            hipLaunchKernelGGL((pass_pairs_lds<Op>), dim3(2 * grid.x), dim3(kTPB), 0, st, a);
        else if constexpr (family_is_gradient<Op>::value)
            hipLaunchKernelGGL((pass_pairs_wide<Op, T>), dim3(2 * grid.x), dim3(kTPB), 0, st, a);
        else
            hipLaunchKernelGGL((pass_pairs<Op, T>), dim3(2 * grid.x), dim3(kTPB), 0, st, a);
        SDBIE_LAUNCHED();
        return false;
    }
    {
        ProfScope prof(prof_variant(family, mixed, code, 0), all - near, st);
        if constexpr (sizeof(T) == 4 && SDBIE_FAR_LDS)
            hipLaunchKernelGGL((far_pairs_lds<Op>), grid, dim3(kTPB), 0, st, a);
        else
            hipLaunchKernelGGL((far_pairs<Op, T>), grid, dim3(kTPB), 0, st, a);
        SDBIE_LAUNCHED();
    }
    {
        ProfScope prof(prof_variant(family, mixed, code, 1), near, st);
        hipLaunchKernelGGL((near_pairs<Op, T>), grid, dim3(kTPB), 0, st, a);
        SDBIE_LAUNCHED();
    }
    return false;
}

// The epilogue of a pass: split (and, after a symmetric far field, block and
// tile-pair) partials summed per target, then the pass's extra terms.
template <int C>
void launch_epilogue(const Plan& P, const PassDesc& d, int S, bool sym, hipStream_t st) {
    const unsigned eb = (unsigned)((P.n + kEpiTargets - 1) / kEpiTargets);
    const dim3 et(kEpiThreads);
    const double* add = d.add_const;
    const double a0 = add ? add[0] : 0.0, a1 = add && C > 1 ? add[1] : 0.0, a2 = add && C > 2 ? add[2] : 0.0;
    const double* tw = d.target_weight ? (const double*)P.w : nullptr;
    const int32_t* perm = d.scatter ? (const int32_t*)P.perm : nullptr;
    if (sym) {
        const int k = d.mixed ? 1 : 0;
        if (d.mixed)
            hipLaunchKernelGGL((sym_epilogue<C, float>), dim3(eb), et, 0, st, P.n,
                               (const int32_t*)P.sym_fwd_start[k], (const double*)P.sym_fwd,
                               (const int32_t*)P.sym_rev_start[k], (const float*)P.sym_rev, S,
                               (const double*)P.partial, tw, d.base, d.base_scale, d.comp, d.comp_scale,
                               (const double*)P.nrm, a0, a1, a2, d.out, perm);
        else
            hipLaunchKernelGGL((sym_epilogue<C, double>), dim3(eb), et, 0, st, P.n,
                               (const int32_t*)P.sym_fwd_start[k], (const double*)P.sym_fwd,
                               (const int32_t*)P.sym_rev_start[k], (const double*)P.sym_rev, S,
                               (const double*)P.partial, tw, d.base, d.base_scale, d.comp, d.comp_scale,
                               (const double*)P.nrm, a0, a1, a2, d.out, perm);
    } else {
        hipLaunchKernelGGL((epilogue<C>), dim3(eb), et, 0, st, P.n, 2 * S, (const double*)P.partial, tw,
                           d.base, d.base_scale, d.comp, d.comp_scale, (const double*)P.nrm, a0, a1, a2, d.out,
                           perm);
    }
    SDBIE_LAUNCHED();
}

}  // namespace

namespace {
// SDBIE_DEBUG >= 3 prints every pair pass as it is enqueued (family, precision, terms)
bool trace_passes() {
    static const bool on = [] {
        const char* e = std::getenv("SDBIE_DEBUG");
        return e && std::atoi(e) >= 3;
    }();
    return on;
}
void trace(const char* family, const PassDesc& d) {
    if (trace_passes())
        std::fprintf(stderr, "[sdbie] pass %s %s%s%s%s%s%s\n", family, d.mixed ? "f32" : "f64", d.dl ? " dl" : "",
                     d.sub ? " sub" : "", d.sl ? " sl" : "", d.slip_beta != 0.0 && !d.sl_dens ? " slip" : "",
                     d.target_normal ? " transposed" : "");
}
}  // namespace

int choose_splits(int64_t n) {
    const int64_t tblocks = (n + kTPB - 1) / kTPB;
    int64_t s = 8 * ((SDBIE_SPLIT_TARGET + 8 * tblocks - 1) / (8 * tblocks));
    if (s > kMaxSplit) s = kMaxSplit;
    while (s > 1 && n / s < 64) s /= 2;
    return (int)(s < 1 ? 1 : s);
}

// The smoothing cutoff rho_cut of a pass is the Stokes one (the larger) for
// both families, matching the tile masks built at staging.
void launch_laplace_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    trace("laplace", d);
    const int S = P.nsplit;
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_STOKES_F32 : SDBIE_RHO_CUT_STOKES_F64;
    const KArgs a = make_args(P, d, S, cut);
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0);
    bool sym = false;
    if (d.target_normal) {
        if (!d.dl || d.sl || d.sub) throw Error(SDBIE_ERR_ARG, "transposed Laplace pass takes a double layer only");
        if (d.mixed) launch_pair_kernels<LaplaceTNOp<float>, float>(P, a, st, 0, 16 | 1, true);
        else launch_pair_kernels<LaplaceTNOp<double>, double>(P, a, st, 0, 16 | 1, false);
    } else {
        const int pc = d.sl && !d.dl ? 2 : code;
#define SDBIE_LAP(T, DL, SL, SUB) sym = launch_pair_kernels<LaplaceOp<T, DL, SL, SUB>, T>(P, a, st, 0, pc, d.mixed)
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
    launch_epilogue<1>(P, d, S, sym, st);
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

void launch_stokes_pass(const Plan& P, const PassDesc& d, hipStream_t st) {
    trace("stokes", d);
    const int S = P.nsplit;
    const double cut = d.mixed ? (double)SDBIE_RHO_CUT_STOKES_F32 : SDBIE_RHO_CUT_STOKES_F64;
    const KArgs a = make_args(P, d, S, cut);
    const bool slip = d.sl && d.slip_beta != 0.0 && d.sl_dens == nullptr;
    const int code = (d.dl ? 1 : 0) | (d.sl ? 2 : 0) | (d.sub ? 4 : 0) | (slip ? 8 : 0);
    if (d.target_normal && d.sl) {
        // transposed stresslet and Stokeslet of one density: six outputs
        // [out | out + 3n] (the partial buffer holds six components per slot)
        if (!d.dl || d.sub || d.sl_dens != d.dl_dens || !(d.c_dl != 0.0) || d.base || d.comp || d.add_const)
            throw Error(SDBIE_ERR_ARG, "transposed Stokes pass: double and single layer of one density");
        if (d.mixed) launch_pair_kernels<StokesTNSLOp<float>, float>(P, a, st, 1, 16 | 2 | 1, true);
        else launch_pair_kernels<StokesTNSLOp<double>, double>(P, a, st, 1, 16 | 2 | 1, false);
        hipLaunchKernelGGL((epilogue<6>), dim3((unsigned)((P.n + kEpiTargets - 1) / kEpiTargets)), dim3(kEpiThreads),
                           0, st, P.n, 2 * S,
                           (const double*)P.partial, d.target_weight ? (const double*)P.w : nullptr, nullptr, 0.0,
                           nullptr, 0.0, (const double*)P.nrm, 0.0, 0.0, 0.0, d.out,
                           d.scatter ? (const int32_t*)P.perm : nullptr);
        SDBIE_LAUNCHED();
        Plan& Pm = const_cast<Plan&>(P);
        (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
        Pm.pairs += (double)P.n * (double)P.n;
        return;
    }
    bool sym = false;
    if (d.target_normal) {
        if (!d.dl || d.sl || d.sub) throw Error(SDBIE_ERR_ARG, "transposed Stokes pass takes a double layer only");
        if (d.mixed) launch_pair_kernels<StokesTNOp<float>, float>(P, a, st, 1, 16 | 1, true);
        else launch_pair_kernels<StokesTNOp<double>, double>(P, a, st, 1, 16 | 1, false);
    } else {
#define SDBIE_STO(T, DL, SL, SUB, SLIP) \
    sym = launch_pair_kernels<StokesOp<T, DL, SL, SUB, SLIP>, T>(P, a, st, 1, code, d.mixed)
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
    launch_epilogue<3>(P, d, S, sym, st);
    Plan& Pm = const_cast<Plan&>(P);
    (d.mixed ? Pm.applies_mixed : Pm.applies_fp64) += 1;
    Pm.pairs += (double)P.n * (double)P.n;
}

void launch_grad_pass(const Plan& P, const GradDesc& g, hipStream_t st) {
    const int S = P.nsplit;
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
    const unsigned eb = (unsigned)((P.n + kEpiTargets - 1) / kEpiTargets);
    const dim3 et(kEpiThreads);
    {
        // node as target: A_m = sum_j g_mj
        launch_pair_kernels<GradOp<false>, double>(P, a, st, 2, 0, false);
        hipLaunchKernelGGL((epilogue<3>), dim3(eb), et, 0, st, P.n, 2 * S, (const double*)P.partial,
                           (const double*)nullptr, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0,
                           (const double*)P.nrm, 0.0, 0.0, 0.0, g.out, (const int32_t*)nullptr);
        SDBIE_LAUNCHED();
        // node as source: out = sum_i g_im - A_m
        launch_pair_kernels<GradOp<true>, double>(P, a, st, 2, 16, false);
    }
    hipLaunchKernelGGL((epilogue<3>), dim3(eb), et, 0, st, P.n, 2 * S, (const double*)P.partial,
                       (const double*)nullptr, (const double*)g.out, -1.0, (const double*)nullptr, 0.0,
                       (const double*)P.nrm, 0.0, 0.0, 0.0, g.out, (const int32_t*)nullptr);
    SDBIE_LAUNCHED();
    Plan& Pm = const_cast<Plan&>(P);
    Pm.applies_fp64 += 2;
    Pm.pairs += 2.0 * (double)P.n * (double)P.n;
}

}  // namespace sdbie
