// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/sdbie.h"

namespace sdbie {

// Error carried inside the library; converted to a status code at the C ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SDBIE_HIP(call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::sdbie::Error(SDBIE_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define SDBIE_LAUNCHED() SDBIE_HIP(hipGetLastError())

constexpr int kTPB = 256;        // threads per block of the pair kernels (4 waves)
constexpr int kTile = 256;       // sources staged in LDS per tile
constexpr int kMaxSplit = 64;    // source splits of one pair pass
constexpr int64_t kMaxNodes = (int64_t)1 << 23;  // the tile-pair masks grow as (n/256)^2 bytes
constexpr int kNearUnit = 64;    // sources per work unit of the near-field kernel
constexpr int kRecBytes = 128;   // largest per-source record of a pair pass
// bytes of source records per unrolled step of the pair loops
#ifndef SDBIE_GROUP_BYTES_F32
#define SDBIE_GROUP_BYTES_F32 128
#endif
// far- and near-field blocks of a pass in one launch (1) or in two (0)
#ifndef SDBIE_ONE_LAUNCH
#define SDBIE_ONE_LAUNCH 1
#endif
// float far-field records through LDS (1) or the scalar cache (0)
#ifndef SDBIE_FAR_LDS
#define SDBIE_FAR_LDS 1
#endif
#ifndef SDBIE_GROUP_BYTES_F64
#define SDBIE_GROUP_BYTES_F64 128
#endif
constexpr int kMaxRestart = 1000; // largest GMRES restart length of a plan
constexpr int kSymChunk = 8;      // far tile pairs per block of the symmetric far field
#ifndef SDBIE_SPLIT_TARGET
#define SDBIE_SPLIT_TARGET 4096      // far-field blocks a pass kernel aims for (the near-field blocks double them)
#endif
// accepted input range: |coordinates| <= kMaxCoord, delta in [kMinDelta, kMaxCoord],
// so every pair distance squared is a normal number in float and double
constexpr double kMaxCoord = 1e15;
constexpr double kMinDelta = 1e-15;
constexpr int kRedBlocks = 512;  // blocks of the deterministic reductions

// Pair-sum passes --------------------------------------------------------------
// Laplace pass:  out_i = base_i + c_dl * sum_j w_j (q_j - sub*q_i)(D.n_j) k2
//                               + c_sl * sum_j w_j g_j k1 + comp * cw_i
// Stokes pass:   out_i = base_i + c_dl * sum_j w_j ((u_j - sub*u_i).D)(D.n_j) D k4
//                               + c_sl * sum_j w_j [f_j k1 + D (D.f_j) k3]
//                               + comp * n_i
// where the Stokes single-layer density is f = sl_dens, or beta * P_tau u
// when slip_beta != 0 (computed on the fly from the double-layer density).
struct PassDesc {
    bool dl = false, sl = false, sub = false;
    double c_dl = 0.0, c_sl = 0.0;
    const double* dl_dens = nullptr;  // sorted
    const double* sl_dens = nullptr;  // sorted
    double slip_beta = 0.0;           // Stokes only
    const double* base = nullptr;     // sorted, [n] or [3][n], added to the result (nullable)
    double base_scale = 1.0;
    const double* comp = nullptr;     // device scalar (nullable): completion coefficient
    double comp_scale = 0.0;
    const double* add_const = nullptr; // host double[3] added to every node (nullable)
    double* out = nullptr;            // sorted, or original order when scatter
    bool scatter = false;             // write out[perm[i]] instead of out[i]
    bool mixed = false;
    // transposed sums (adjoint)
    bool unit_src_weight = false;     // sources enter with weight 1 instead of w_j
    bool target_weight = false;       // the pair sum is multiplied by the target's w_i
    bool target_normal = false;       // double layer contracted with the target's normal (transposed DL)
    const double* dl_target = nullptr;  // target density of the subtracted double layer (default dl_dens)
};

// Position-gradient pass of the adjoint: for every pair (i, j),
//   g_ij = grad_D [lam1_i T1_ij + lam2_i . T2_ij],  D = x_i - x_j,
//   T1_ij = c_l w_j (p_j - p_i)(D.n_j) K2 + (mu/K) c_l w_j v_j K1,
//   T2_ij = c_s w_j ((u_j - u_i).D)(D.n_j) D K4 + c_v w_j [f_j K1 + D (D.f_j) K3],
// with c_l = 1/(4 pi), c_s = -3/(4 pi), c_v = 1/(8 pi mu); the pass writes
// out_m = -sum_j g_mj + sum_i g_im (derivative of -lam^T F w.r.t. x_m).
struct GradDesc {
    double mu, K;
    const double *p, *v, *u, *f, *lam1, *lam2;  // sorted, stride n
    double* out;                                // sorted [3][n]
};

struct Plan {
    int64_t n = 0;
    int max_restart = 0;
    double delta = 0.0;
    double area = 0.0;  // sum of weights
    // sorted node data (double)
    double* x = nullptr;    // [3][n]
    double* nrm = nullptr;  // [3][n]
    double* w = nullptr;    // [n]
    double* wn = nullptr;   // [3][n] w_j n_j
    // sorted node data padded to whole tiles of kTile nodes (pair-kernel sources;
    // padding nodes sit far outside the body with zero weight and normal)
    int64_t npad = 0;       // ntiles * kTile
    int ntiles = 0;
    double* px = nullptr;   // [3][npad]
    double* pn = nullptr;   // [3][npad]
    double* pw = nullptr;   // [npad]
    float* px32 = nullptr;  // [3][npad], each node minus the centre of its tile's box
    double* boxes = nullptr;   // [ntiles][6] min/max per axis
    double* uboxes = nullptr;  // [npad / kNearUnit][6]: the same per near-field unit of sources
    uint8_t* mask64 = nullptr; // [ntiles][ntiles]: 1 if the tile pair may hold a pair with rho < double cutoff
    uint8_t* mask32 = nullptr; // [ntiles][ntiles]: same with the float cutoff
    int32_t* perm = nullptr;  // sorted index -> caller index
    uint64_t* keys = nullptr; // sort scratch, [npow2]
    int64_t npow2 = 0;
    // scratch
    int nsplit = 0;             // source splits of a pair pass (choose_splits(n) or fewer)
    int max_comps = 6;          // components a pass may write per slot (the partial buffer's C)
    double* partial = nullptr;  // [2 * nsplit][C][n], C <= max_comps: far splits then near splits
    void* rec = nullptr;        // per-pass source records, [npad][kRecBytes]
    double* red = nullptr;      // reduction partials [kRedBlocks * 64]
    double* scal = nullptr;     // small device scalars / columns [256]
    double* vecs = nullptr;     // general work vectors, kNumVec x [3][n]
    double* basis_in = nullptr;   // inner GMRES basis [(max_restart+1)][3n]
    double* basis_out = nullptr;  // outer GMRES basis [(max_restart+1)][n]
    double* image_out = nullptr;  // local solutions (p, u) and right-hand sides (b_D, b_S) of each outer
                                  // basis vector [(max_restart+1)][8n]
    double* basis_rc = nullptr;   // recycled inner basis (deflation space) [(max_restart+1)][3n]
    double* host_pinned = nullptr;  // not used (host buffers are plain)
    // (target, source) pairs of real nodes in the near tile pairs (double, float masks)
    double near_pairs64 = 0.0, near_pairs32 = 0.0;
    // target-source symmetric far field (for the pass kinds whose
    // SDBIE_SYM_* bit is set in `symmetric`): per
    // precision (index 0 double, 1 float) the far tile pairs {a < b} numbered
    // in column order (pair p owns a reverse slot), the work items (a, b, p) in
    // row order cut into blocks of at most kSymChunk items, the first block of
    // each target tile and the first pair of each source tile
    int symmetric = SDBIE_SYM_DEFAULT;
    int32_t* sym_items[2] = {};      // [npairs][3]
    int32_t* sym_blocks[2] = {};     // [nblocks][2]: first item, item count
    int32_t* sym_fwd_start[2] = {};  // [ntiles + 1]
    int32_t* sym_rev_start[2] = {};  // [ntiles + 1]
    int sym_nblocks[2] = {0, 0}, sym_npairs[2] = {0, 0};
    double* sym_fwd = nullptr;       // [nblocks][C][kTile] forward partials of the target tile, C <= 3
    void* sym_rev = nullptr;         // [npairs][C][kTile] reverse partials of the source tile (pass precision)
    // bookkeeping for info
    int64_t applies_fp64 = 0, applies_mixed = 0;
    double pairs = 0.0;
    double* vec(int k) const { return vecs + (size_t)k * 3 * n; }
};

constexpr int kNumVec = 31;
constexpr int kImageStride = 8;  // doubles per node of one image-basis slot: p, u, b_D, b_S

size_t workspace_bytes(int64_t n, int max_restart);
void carve_workspace(Plan& P, void* ws);
// layer applies only (no solver vectors), at most nsplit_cap source splits and
// three components per partial slot: bytes, and the carve (which also sets
// *in, a [3][n] buffer for the gathered density)
size_t layer_workspace_bytes(int64_t n, int nsplit_cap);
void carve_layer_workspace(Plan& P, void* ws, int nsplit_cap, double** in);
// the layer sums of the C ABI on a staged plan; `in` receives the density in
// staged order ([n] or [3][n])
void apply_laplace_layer(Plan& P, sdbie_layer layer, const double* dens, double* out, sdbie_precision prec,
                         hipStream_t st, double* in);
void apply_stokes_layer(Plan& P, double mu, sdbie_layer layer, const double* dens, double* out,
                        sdbie_precision prec, hipStream_t st, double* in);

// allocation-free layer sum (noalloc.hip): stages s into the library's static
// device array and applies the Stokes layer
void stokes_layer_apply_static(const sdbie_surface* s, double mu, sdbie_layer layer, const double* dens,
                               double* out, sdbie_precision prec, hipStream_t st);

// kernels (pair_kernels.hip) ----------------------------------------------------
void launch_laplace_pass(const Plan& P, const PassDesc& d, hipStream_t s);
void launch_stokes_pass(const Plan& P, const PassDesc& d, hipStream_t s);
void launch_grad_pass(const Plan& P, const GradDesc& g, hipStream_t s);
int choose_splits(int64_t n);

// kernel timing (profile.hip)
int prof_variant(int family, bool mixed, int code, int part);
struct ProfScope {
    ProfScope(int variant, double pairs, hipStream_t s);
    ~ProfScope();
    hipStream_t s_;
    long idx_ = -1;
};

// staging (stage.hip) --------------------------------------------------------------
void stage_surface(Plan& P, const sdbie_surface* s, hipStream_t st);

// vector kernels (blas.hip) ----------------------------------------------------------
// deterministic dot product sum_i a_i b_i (len elements) -> device scalar *out
void dev_dot(const Plan& P, const double* a, const double* b, int64_t len, double* out, hipStream_t s);
// dots of w against k columns of V (column stride ld) -> out[0..k-1]
void dev_multidot(const Plan& P, const double* V, int64_t ld, int k, const double* w, int64_t len,
                  double* out, hipStream_t s);
// w -= sum_j h[j] V_j  (h on device)
void dev_multi_axpy_sub(const double* V, int64_t ld, int k, const double* h, double* w, int64_t len,
                        hipStream_t s);
// x += sum_j y[j] V_j  (y on device)
void dev_multi_axpy_add(const double* V, int64_t ld, int k, const double* y, double* x, int64_t len,
                        hipStream_t s);
void dev_axpby(double a, const double* x, double b, const double* y, double* out, int64_t len, hipStream_t s);
void dev_scale(double a, const double* x, double* out, int64_t len, hipStream_t s);
void dev_fill(double v, double* out, int64_t len, hipStream_t s);
void dev_add_scaled_scalar(double* x, const double* dscal, double scale, int64_t len, hipStream_t s);
// out = u.n (per node)
void dev_normal_component(const Plan& P, const double* u, double* out, hipStream_t s);
// f = -p n + beta (u - (u.n) n) + f_extra   (u, f_extra nullable)
void dev_traction(const Plan& P, const double* p, const double* u, double beta, const double* f_extra,
                  double* f, hipStream_t s);
// sorted <-> caller order
void dev_gather(const Plan& P, const double* src, double* dst, int comps, hipStream_t s);
void dev_scatter(const Plan& P, const double* src, double* dst, int comps, hipStream_t s);
// non-finite check: *flag (device int) set to 1 if any element is not finite
void dev_check_finite(const double* a, int64_t len, double bound, int* flag, hipStream_t s);

// adjoint helpers (see blas.hip)
void dev_adj_darcy(const Plan& P, const double* tn, const double* lam, const double* dl1, const double* sum,
                   double* out, hipStream_t s);
void dev_adj_stokes(const Plan& P, const double* lam, const double* m0, const double* m1, const double* m2,
                    const double* tns, const double* sv, const double* flux, double beta, double* out, hipStream_t s);
void dev_scalar_normal(const Plan& P, const double* sv, double scale, double* out, hipStream_t s);
void dev_axpy_w(const Plan& P, double* x, const double* d, double scale, hipStream_t s);
void dev_adj_rhs(const Plan& P, const double e[3], double beta, double* gp, double* gu, hipStream_t s);

// host-side helpers
double host_read_scalar(const double* d, hipStream_t s);
// eigenvalues of an upper Hessenberg matrix (n x n, row-major, overwritten); false if the QR iteration stalls
bool hessenberg_eigenvalues(int n, double* A, double* wr, double* wi);

}  // namespace sdbie
