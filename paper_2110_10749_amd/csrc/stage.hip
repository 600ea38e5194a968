// Surface staging: spatial (Morton) order and the sorted node copies.
//
// The pair kernels give each wave 64 consecutive targets; sorting the nodes
// along a Morton (Z-order) curve makes those 64 targets spatial neighbours,
// so the near-field branch (rho < rho_cut) is taken by few waves per source
// and the rest run the plain far-field kernel.
//
// Steps (all on the device): bounding box (min/max reduction), 30-bit Morton
// key per node (10 bits per axis), key<<32 | index sorted by a bitonic network
// over the next power of two (padding keys = UINT64_MAX; keys are unique, so
// the order is deterministic), then gather of x, n, w into sorted double
// arrays and the weighted normals w n; copies padded to whole tiles of kTile
// nodes for the pair kernels; per-tile bounding boxes; a float copy of the
// coordinates in the frame of each node's tile; and the near-field masks of
// tile pairs (box distance below rho_cut delta, one mask for the double cutoff
// and one for the float cutoff).
#include <vector>

#include "smoothing_coeffs.h"
#include "solver.h"

namespace sdbie {
namespace {

__global__ __launch_bounds__(256) void k_bbox(int64_t n, const double* __restrict__ x, double* __restrict__ out) {
    // one block per axis: out[2c] = min, out[2c+1] = max
    __shared__ double smin[256], smax[256];
    const int c = blockIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = x[c * n + i];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * c] = smin[0];
        out[2 * c + 1] = smax[0];
    }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(int64_t n, int64_t npow2, const double* __restrict__ x, const double* __restrict__ bb,
                         uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow2) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    uint32_t code = 0;
    // a cube of the largest extent, so the curve is isotropic
    const double ext = fmax(fmax(bb[1] - bb[0], bb[3] - bb[2]), bb[5] - bb[4]);
    const double sc = ext > 0.0 ? 1023.0 / ext : 0.0;
    for (int c = 0; c < 3; ++c) {
        double t = (x[c * n + i] - bb[2 * c]) * sc;
        t = fmin(fmax(t, 0.0), 1023.0);
        code |= spread10((uint32_t)t) << (2 - c);
    }
    keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

__global__ void k_bitonic(uint64_t* __restrict__ keys, int64_t npow2, int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow2) return;
    const int64_t l = i ^ j;
    if (l > i) {
        const uint64_t a = keys[i], b = keys[l];
        const bool up = (i & k) == 0;
        if ((a > b) == up) {
            keys[i] = b;
            keys[l] = a;
        }
    }
}

__global__ void k_stage(int64_t n, const uint64_t* __restrict__ keys, const double* __restrict__ x,
                        const double* __restrict__ nrm, const double* __restrict__ w, int32_t* __restrict__ perm,
                        double* __restrict__ xs, double* __restrict__ ns, double* __restrict__ wsrt,
                        double* __restrict__ wn) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t o = (int64_t)(keys[k] & 0xffffffffull);
    perm[k] = (int32_t)o;
    const double wk = w[o];
    wsrt[k] = wk;
    for (int c = 0; c < 3; ++c) {
        const double xv = x[c * n + o], nv = nrm[c * n + o];
        xs[c * n + k] = xv;
        ns[c * n + k] = nv;
        wn[c * n + k] = wk * nv;
    }
}

// padded copies for the pair kernels: nodes k >= n sit at a point `far`
// outside the bounding box (10 extents away) with zero weight and normal.
__global__ void k_pad(int64_t n, int64_t npad, const double* __restrict__ xs, const double* __restrict__ ns,
                      const double* __restrict__ ws, const double* __restrict__ bb, double* __restrict__ px,
                      double* __restrict__ pn, double* __restrict__ pw) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npad) return;
    const double ext = fmax(fmax(bb[1] - bb[0], bb[3] - bb[2]), bb[5] - bb[4]);
    for (int c = 0; c < 3; ++c) {
        const double xv = k < n ? xs[c * n + k] : bb[2 * c + 1] + 10.0 * ext + 1.0;
        px[c * npad + k] = xv;
        pn[c * npad + k] = k < n ? ns[c * n + k] : 0.0;
    }
    pw[k] = k < n ? ws[k] : 0.0;
}

// float coordinates in the frame of their tile: minus the centre of the tile's
// box (every tile holds at least one real node, so the centre is finite).  The
// kernels see coordinates only through differences x_i - x_j, formed after
// moving the targets into the source tile's frame, so the rounding of a float
// coordinate is set by the tile's extent, not by the body's or by the
// distance from the origin.
__global__ void k_frame32(int64_t npad, const double* __restrict__ px, const double* __restrict__ boxes,
                          float* __restrict__ px32) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npad) return;
    const double* b = boxes + (k / kTile) * 6;
    for (int c = 0; c < 3; ++c) px32[c * npad + k] = (float)(px[c * npad + k] - 0.5 * (b[2 * c] + b[2 * c + 1]));
}

// bounding box of each group of W consecutive (sorted) real nodes (empty:
// +inf / -inf for a group of padding only); one block of W threads per group
template <int W>
__global__ __launch_bounds__(W) void k_boxes(int64_t n, const double* __restrict__ xs, double* __restrict__ boxes) {
    __shared__ double sh[6][W];
    const int64_t k = (int64_t)blockIdx.x * W + threadIdx.x;
    for (int c = 0; c < 3; ++c) {
        const double v = k < n ? xs[c * n + k] : NAN;
        sh[2 * c][threadIdx.x] = k < n ? v : INFINITY;
        sh[2 * c + 1][threadIdx.x] = k < n ? v : -INFINITY;
    }
    __syncthreads();
    for (int s = W / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; ++c) {
                sh[2 * c][threadIdx.x] = fmin(sh[2 * c][threadIdx.x], sh[2 * c][threadIdx.x + s]);
                sh[2 * c + 1][threadIdx.x] = fmax(sh[2 * c + 1][threadIdx.x], sh[2 * c + 1][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) boxes[(int64_t)blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// mask[b][t] = 1 when the boxes of tiles b and t are closer than the cutoff.
// cnt[0], cnt[1] += the (target, source) pairs of real nodes in the near tile
// pairs of each precision (integer sums: exact in any order).
__global__ void k_near_masks(int nt, int64_t n, const double* __restrict__ boxes, double rc64, double rc32,
                             uint8_t* __restrict__ m64, uint8_t* __restrict__ m32,
                             unsigned long long* __restrict__ cnt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c64 = 0, c32 = 0;
    if (idx < (int64_t)nt * nt) {
        const int64_t b = idx / nt, t = idx % nt;
        const double* A = boxes + b * 6;
        const double* B = boxes + t * 6;
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double gap = fmax(0.0, fmax(A[2 * c] - B[2 * c + 1], B[2 * c] - A[2 * c + 1]));
            d2 += gap * gap;
        }
        const bool n64 = d2 < rc64 * rc64, n32 = d2 < rc32 * rc32;
        m64[idx] = n64 ? 1 : 0;
        m32[idx] = n32 ? 1 : 0;
        const int64_t rb = n - b * kTile < kTile ? n - b * kTile : kTile;
        const int64_t rt = n - t * kTile < kTile ? n - t * kTile : kTile;
        const unsigned long long pr = (unsigned long long)(rb * rt);
        c64 = n64 ? pr : 0;
        c32 = n32 ? pr : 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        c64 += __shfl_down(c64, off);
        c32 += __shfl_down(c32, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c64) atomicAdd(cnt, c64);
        if (c32) atomicAdd(cnt + 1, c32);
    }
}

// Work lists of the symmetric far field, from the near masks (host side):
// the far tile pairs {a < b} numbered column by column (pair p of column b
// owns a reverse-partial slot of source tile b; rev_start[b] is the first),
// and the same pairs as work items (a, b, p) row by row, cut into blocks of at
// most kSymChunk items of one target tile a (fwd_start[a] is its first block).
void build_symmetric_lists(Plan& P, hipStream_t st) {
    const int T = P.ntiles;
    std::vector<uint8_t> m((size_t)T * T);
    std::vector<int32_t> pid((size_t)T * T, -1), rev_start(T + 1), fwd_start(T + 1), items, blocks;
    for (int k = 0; k < 2; ++k) {
        SDBIE_HIP(hipMemcpyAsync(m.data(), k ? P.mask32 : P.mask64, m.size(), hipMemcpyDeviceToHost, st));
        SDBIE_HIP(hipStreamSynchronize(st));
        int np = 0;
        for (int b = 0; b < T; ++b) {
            rev_start[b] = np;
            for (int a = 0; a < b; ++a)
                if (!m[(size_t)a * T + b]) pid[(size_t)a * T + b] = np++;
        }
        rev_start[T] = np;
        items.clear();
        blocks.clear();
        for (int a = 0; a < T; ++a) {
            fwd_start[a] = (int32_t)(blocks.size() / 2);
            int cnt = 0;
            for (int b = a + 1; b < T; ++b) {
                if (m[(size_t)a * T + b]) continue;
                if (cnt == 0) {
                    blocks.push_back((int32_t)(items.size() / 3));
                    blocks.push_back(0);
                }
                items.push_back(a);
                items.push_back(b);
                items.push_back(pid[(size_t)a * T + b]);
                ++blocks.back();
                if (++cnt == kSymChunk) cnt = 0;
            }
        }
        fwd_start[T] = (int32_t)(blocks.size() / 2);
        P.sym_npairs[k] = np;
        P.sym_nblocks[k] = (int)(blocks.size() / 2);
        if (np > 0) {
            SDBIE_HIP(hipMemcpyAsync(P.sym_items[k], items.data(), items.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice, st));
            SDBIE_HIP(hipMemcpyAsync(P.sym_blocks[k], blocks.data(), blocks.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice, st));
        }
        SDBIE_HIP(hipMemcpyAsync(P.sym_fwd_start[k], fwd_start.data(), (T + 1) * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        SDBIE_HIP(hipMemcpyAsync(P.sym_rev_start[k], rev_start.data(), (T + 1) * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        SDBIE_HIP(hipStreamSynchronize(st));  // the host vectors are reused
    }
}

}  // namespace

void stage_surface(Plan& P, const sdbie_surface* s, hipStream_t st) {
    const int64_t n = P.n;
    // finite check of the node data first (Morton keys of NaN are meaningless)
    // flags and counters are cleared by a fill kernel, not a memset node (the
    // staging of the allocation-free entry point may sit in a captured stream)
    int* flag = reinterpret_cast<int*>(P.scal + kScalStage);
    dev_fill(0.0, P.scal + kScalStage, 1, st);  // two ints
    dev_check_finite(s->x, 3 * n, kMaxCoord, flag, st);
    dev_check_finite(s->nrm, 3 * n, HUGE_VAL, flag, st);
    dev_check_finite(s->w, n, HUGE_VAL, flag, st);
    int hflag[2] = {0, 0};
    SDBIE_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, st));
    SDBIE_HIP(hipStreamSynchronize(st));
    if (hflag[0]) throw Error(SDBIE_ERR_NONFINITE, "non-finite node coordinates, normals or weights");
    if (hflag[1]) throw Error(SDBIE_ERR_ARG, "node coordinates must not exceed 1e15 in magnitude");

    double* bb = P.scal + kScalStage + 2;
    hipLaunchKernelGGL(k_bbox, dim3(3), dim3(256), 0, st, n, s->x, bb);
    SDBIE_LAUNCHED();
    const unsigned nb = (unsigned)((P.npow2 + 255) / 256);
    hipLaunchKernelGGL(k_morton, dim3(nb), dim3(256), 0, st, n, P.npow2, s->x, (const double*)bb, P.keys);
    SDBIE_LAUNCHED();
    for (int64_t k = 2; k <= P.npow2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            hipLaunchKernelGGL(k_bitonic, dim3(nb), dim3(256), 0, st, P.keys, P.npow2, j, k);
            SDBIE_LAUNCHED();
        }
    hipLaunchKernelGGL(k_stage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, (const uint64_t*)P.keys,
                       s->x, s->nrm, s->w, P.perm, P.x, P.nrm, P.w, P.wn);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL(k_pad, dim3((unsigned)((P.npad + 255) / 256)), dim3(256), 0, st, n, P.npad,
                       (const double*)P.x, (const double*)P.nrm, (const double*)P.w, (const double*)bb, P.px, P.pn,
                       P.pw);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL((k_boxes<kTile>), dim3((unsigned)P.ntiles), dim3(kTile), 0, st, n, (const double*)P.x,
                       P.boxes);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL(k_frame32, dim3((unsigned)((P.npad + 255) / 256)), dim3(256), 0, st, P.npad,
                       (const double*)P.px, (const double*)P.boxes, P.px32);
    SDBIE_LAUNCHED();
    hipLaunchKernelGGL((k_boxes<kNearUnit>), dim3((unsigned)(P.npad / kNearUnit)), dim3(kNearUnit), 0, st, n,
                       (const double*)P.x, P.uboxes);
    SDBIE_LAUNCHED();
    // cutoffs with a relative margin of 1e-6 (the far kernels assume rho >= rho_cut)
    const double rc64 = SDBIE_RHO_CUT_STOKES_F64 * P.delta * (1.0 + 1e-6);
    const double rc32 = SDBIE_RHO_CUT_STOKES_F32 * P.delta * (1.0 + 1e-6);
    const int64_t nt2 = (int64_t)P.ntiles * P.ntiles;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(P.scal + kScalStage + 10);
    dev_fill(0.0, P.scal + kScalStage + 10, 2, st);  // two 64-bit counters (all-zero bits)
    hipLaunchKernelGGL(k_near_masks, dim3((unsigned)((nt2 + 255) / 256)), dim3(256), 0, st, P.ntiles, n,
                       (const double*)P.boxes, rc64, rc32, P.mask64, P.mask32, cnt);
    SDBIE_LAUNCHED();
    unsigned long long hc[2] = {0, 0};
    SDBIE_HIP(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st));
    SDBIE_HIP(hipStreamSynchronize(st));
    P.near_pairs64 = (double)hc[0];
    P.near_pairs32 = (double)hc[1];
    if (P.sym_items[0]) build_symmetric_lists(P, st);
    dev_dot(P, P.w, nullptr, n, P.scal + kScalStage + 8, st);
    P.area = host_read_scalar(P.scal + kScalStage + 8, st);
    if (!(P.area > 0.0)) throw Error(SDBIE_ERR_ARG, "the quadrature weights sum to zero");
}

}  // namespace sdbie
