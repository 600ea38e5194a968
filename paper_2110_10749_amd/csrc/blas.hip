// Vector kernels of the Krylov solver and the interface loop (double).
//
// Reductions are deterministic: a fixed grid of kRedBlocks blocks writes one
// partial per block (wave shuffles, then LDS in a fixed order) and a single
// block adds the partials in a fixed order.  Results are bitwise
// reproducible from run to run.
#include "internal.h"

namespace sdbie {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block of 256 lanes -> sum in lane 0 (fixed order)
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t len, double* __restrict__ part) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256)
        s += b ? a[i] * b[i] : a[i];
    const double r = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// part: [nb][k] -> out[j] = sum_b part[b][j], one block per j
__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ part, int nb, int k,
                                                     double* __restrict__ out) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(int64_t)b * k + j];
    const double r = block_sum(s, sh);
    if (threadIdx.x == 0) out[j] = r;
}

// part[b][j] = sum over block b's chunk of V_j . w; blockIdx.y takes kDotCols
// columns at a time, so w is read once per kDotCols columns (fixed order)
constexpr int kDotCols = 8;
__global__ __launch_bounds__(256) void k_multidot_partial(const double* __restrict__ V, int64_t ld, int k,
                                                          const double* __restrict__ w, int64_t len,
                                                          double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < len ? lo + chunk : len;
    const int j0 = blockIdx.y * kDotCols;
    const int nc = k - j0 < kDotCols ? k - j0 : kDotCols;
    double acc[kDotCols];
#pragma unroll
    for (int c = 0; c < kDotCols; ++c) acc[c] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double wi = w[i];
#pragma unroll
        for (int c = 0; c < kDotCols; ++c)
            if (c < nc) acc[c] += V[(int64_t)(j0 + c) * ld + i] * wi;
    }
    for (int c = 0; c < nc; ++c) {
        const double r = block_sum(acc[c], sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * k + j0 + c] = r;
    }
}

__global__ void k_multi_axpy(const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ h,
                             double sign, double* __restrict__ w, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * V[(int64_t)j * ld + i];
    w[i] += sign * s;
}

// out may alias x or y (elementwise: each lane reads its element before writing it)
__global__ void k_axpby(double a, const double* x, double b, const double* y, double* out, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void k_fill(double v, double* __restrict__ out, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] = v;
}

__global__ void k_add_scalar(double* __restrict__ x, const double* __restrict__ d, double scale, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] += scale * d[0];
}

__global__ void k_normal_comp(int64_t n, const double* __restrict__ nrm, const double* __restrict__ u,
                              double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = nrm[i] * u[i] + nrm[n + i] * u[n + i] + nrm[2 * n + i] * u[2 * n + i];
}

__global__ void k_traction(int64_t n, const double* __restrict__ nrm, const double* __restrict__ p,
                           const double* __restrict__ u, double beta, const double* __restrict__ fx,
                           double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nx = nrm[i], ny = nrm[n + i], nz = nrm[2 * n + i];
    const double pi = p ? p[i] : 0.0;
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (u && beta != 0.0) {
        const double ux = u[i], uy = u[n + i], uz = u[2 * n + i];
        const double un = ux * nx + uy * ny + uz * nz;
        tx = beta * (ux - un * nx);
        ty = beta * (uy - un * ny);
        tz = beta * (uz - un * nz);
    }
    f[i] = -pi * nx + tx + (fx ? fx[i] : 0.0);
    f[n + i] = -pi * ny + ty + (fx ? fx[n + i] : 0.0);
    f[2 * n + i] = -pi * nz + tz + (fx ? fx[2 * n + i] : 0.0);
}

__global__ void k_gather(int64_t n, int comps, const int32_t* __restrict__ perm, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * n + i] = src[c * n + o];
}

__global__ void k_scatter(int64_t n, int comps, const int32_t* __restrict__ perm, const double* __restrict__ src,
                          double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * n + o] = src[c * n + i];
}

// flag[0] = 1 if some entry is not finite, flag[1] = 1 if some finite entry exceeds bound in magnitude
__global__ void k_check_finite(const double* __restrict__ a, int64_t len, double bound, int* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    if (!isfinite(a[i])) flag[0] = 1;
    else if (fabs(a[i]) > bound) flag[1] = 1;
}

// ---- adjoint helpers ------------------------------------------------------
// out = tn + lam * dl1 + w * (*sum) / area      (transposed completed Darcy operator)
__global__ void k_adj_darcy(int64_t n, const double* __restrict__ tn, const double* __restrict__ lam,
                            const double* __restrict__ dl1, const double* __restrict__ w,
                            const double* __restrict__ sum, double inv_area, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = tn[i] + lam[i] * dl1[i] + w[i] * sum[0] * inv_area;
}

// out = lam + sum_c mneg_c lam_c + tns + w n (*flux)/area + beta P_tau sv, where sv
// already carries the target weight w
// (transposed completed Stokes operator with slip); mneg_c[a][i] = -(M_i)_{ac}
__global__ void k_adj_stokes(int64_t n, const double* __restrict__ lam, const double* __restrict__ m0,
                             const double* __restrict__ m1, const double* __restrict__ m2,
                             const double* __restrict__ tns, const double* __restrict__ sv,
                             const double* __restrict__ nrm, const double* __restrict__ w,
                             const double* __restrict__ flux, double inv_area, double beta, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l[3] = {lam[i], lam[n + i], lam[2 * n + i]};
    const double nv[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
    double svn = 0.0;
    if (sv) svn = sv[i] * nv[0] + sv[n + i] * nv[1] + sv[2 * n + i] * nv[2];
    const double fl = flux[0] * inv_area;
    for (int a = 0; a < 3; ++a) {
        const int64_t k = a * n + i;
        double v = l[a] + m0[k] * l[0] + m1[k] * l[1] + m2[k] * l[2] + tns[k] + w[i] * nv[a] * fl;
        if (sv) v += beta * (sv[k] - svn * nv[a]);  // sv carries the target weight
        out[k] = v;
    }
}

// out3 = scale * s n
__global__ void k_scalar_normal(int64_t n, const double* __restrict__ s, double scale, const double* __restrict__ nrm,
                                double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 3; ++c) out[c * n + i] = scale * s[i] * nrm[c * n + i];
}

// x += scale * (*d) * w
__global__ void k_axpy_w(int64_t n, double* __restrict__ x, const double* __restrict__ w, const double* __restrict__ d,
                         double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += scale * d[0] * w[i];
}

// gp = -w (e.n);  gu = beta w (e - (e.n) n)
__global__ void k_adj_rhs(int64_t n, const double* __restrict__ nrm, const double* __restrict__ w, double e0, double e1,
                          double e2, double beta, double* __restrict__ gp, double* __restrict__ gu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nx = nrm[i], ny = nrm[n + i], nz = nrm[2 * n + i];
    const double en = e0 * nx + e1 * ny + e2 * nz;
    gp[i] = -w[i] * en;
    gu[i] = beta * w[i] * (e0 - en * nx);
    gu[n + i] = beta * w[i] * (e1 - en * ny);
    gu[2 * n + i] = beta * w[i] * (e2 - en * nz);
}

inline unsigned nblk(int64_t len) { return (unsigned)((len + 255) / 256); }

}  // namespace

void dev_dot(const Plan& P, const double* a, const double* b, int64_t len, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, a, b, len, P.red);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, s, (const double*)P.red, kRedBlocks, 1, out);
    SDBIE_LAUNCHED();
}

void dev_multidot(const Plan& P, const double* V, int64_t ld, int k, const double* w, int64_t len,
                  double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot_partial, dim3(kRedBlocks, (unsigned)((k + kDotCols - 1) / kDotCols)), dim3(256), 0,
                       s, V, ld, k, w, len, P.red);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_cols, dim3(k), dim3(256), 0, s, (const double*)P.red, kRedBlocks, k, out);
    SDBIE_LAUNCHED();
}

void dev_multi_axpy_sub(const double* V, int64_t ld, int k, const double* h, double* w, int64_t len,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(len)), dim3(256), 0, s, V, ld, k, h, -1.0, w, len);
    SDBIE_LAUNCHED();
}

void dev_multi_axpy_add(const double* V, int64_t ld, int k, const double* y, double* x, int64_t len,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(len)), dim3(256), 0, s, V, ld, k, y, 1.0, x, len);
    SDBIE_LAUNCHED();
}

void dev_axpby(double a, const double* x, double b, const double* y, double* out, int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(nblk(len)), dim3(256), 0, s, a, x, b, y, out, len);
    SDBIE_LAUNCHED();
}

void dev_scale(double a, const double* x, double* out, int64_t len, hipStream_t s) {
    dev_axpby(a, x, 0.0, nullptr, out, len, s);
}

void dev_fill(double v, double* out, int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(nblk(len)), dim3(256), 0, s, v, out, len);
    SDBIE_LAUNCHED();
}

void dev_add_scaled_scalar(double* x, const double* d, double scale, int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(k_add_scalar, dim3(nblk(len)), dim3(256), 0, s, x, d, scale, len);
    SDBIE_LAUNCHED();
}

void dev_normal_component(const Plan& P, const double* u, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_normal_comp, dim3(nblk(P.n)), dim3(256), 0, s, P.n, (const double*)P.nrm, u, out);
    SDBIE_LAUNCHED();
}

void dev_traction(const Plan& P, const double* p, const double* u, double beta, const double* f_extra,
                  double* f, hipStream_t s) {
    hipLaunchKernelGGL(k_traction, dim3(nblk(P.n)), dim3(256), 0, s, P.n, (const double*)P.nrm, p, u, beta,
                       f_extra, f);
    SDBIE_LAUNCHED();
}

void dev_gather(const Plan& P, const double* src, double* dst, int comps, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(nblk(P.n)), dim3(256), 0, s, P.n, comps, (const int32_t*)P.perm, src, dst);
    SDBIE_LAUNCHED();
}

void dev_scatter(const Plan& P, const double* src, double* dst, int comps, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3(nblk(P.n)), dim3(256), 0, s, P.n, comps, (const int32_t*)P.perm, src, dst);
    SDBIE_LAUNCHED();
}

void dev_check_finite(const double* a, int64_t len, double bound, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(nblk(len)), dim3(256), 0, s, a, len, bound, flag);
    SDBIE_LAUNCHED();
}

void dev_adj_darcy(const Plan& P, const double* tn, const double* lam, const double* dl1, const double* sum,
                   double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_darcy, dim3(nblk(P.n)), dim3(256), 0, s, P.n, tn, lam, dl1, (const double*)P.w, sum,
                       1.0 / P.area, out);
    SDBIE_LAUNCHED();
}

void dev_adj_stokes(const Plan& P, const double* lam, const double* m0, const double* m1, const double* m2,
                    const double* tns, const double* sv, const double* flux, double beta, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_stokes, dim3(nblk(P.n)), dim3(256), 0, s, P.n, lam, m0, m1, m2, tns, sv,
                       (const double*)P.nrm, (const double*)P.w, flux, 1.0 / P.area, beta, out);
    SDBIE_LAUNCHED();
}

void dev_scalar_normal(const Plan& P, const double* sv, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_scalar_normal, dim3(nblk(P.n)), dim3(256), 0, s, P.n, sv, scale, (const double*)P.nrm, out);
    SDBIE_LAUNCHED();
}

void dev_axpy_w(const Plan& P, double* x, const double* d, double scale, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_w, dim3(nblk(P.n)), dim3(256), 0, s, P.n, x, (const double*)P.w, d, scale);
    SDBIE_LAUNCHED();
}

void dev_adj_rhs(const Plan& P, const double e[3], double beta, double* gp, double* gu, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_rhs, dim3(nblk(P.n)), dim3(256), 0, s, P.n, (const double*)P.nrm, (const double*)P.w, e[0],
                       e[1], e[2], beta, gp, gu);
    SDBIE_LAUNCHED();
}

double host_read_scalar(const double* d, hipStream_t s) {
    double v = 0.0;
    SDBIE_HIP(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, s));
    SDBIE_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace sdbie
