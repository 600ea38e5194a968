// C ABI of the library: argument checks, workspace layout, plans, and the
// conversion between the caller's node order and the staged (Morton) order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "solver.h"

namespace sdbie {
namespace {

thread_local std::string g_last_error;

constexpr double kPi = 3.14159265358979323846;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

struct Layout {
    size_t x, nrm, w, wn, px, pn, pw, px32, boxes, uboxes, mask64, mask32, perm, keys, partial, rec, red, scal, vecs,
        basis_in, basis_out, image_out, basis_rc, sym_items[2], sym_blocks[2], sym_fwd_start[2], sym_rev_start[2],
        sym_fwd, sym_rev, total;
};

// bounds of the symmetric far-field lists: at most T (T - 1) / 2 far tile
// pairs, and at most pairs / kSymChunk + T blocks.  The lists and partial
// slots grow as T^2 (about 3469 bytes per tile pair), so plans of more than
// kSymMaxTiles tiles hold none and run every pass one direction at a time.
constexpr int64_t kSymMaxTiles = 2048;  // 524288 nodes: 14.6 GB of lists and slots
bool sym_fits(int64_t nt) { return nt <= kSymMaxTiles; }
int64_t sym_max_pairs(int64_t nt) { return nt * (nt - 1) / 2; }
int64_t sym_max_blocks(int64_t nt) { return sym_max_pairs(nt) / kSymChunk + nt; }

// the node data, staging and pair-pass scratch every plan holds: nsplit
// source splits with up to `comps` components per partial slot, m the
// longest GMRES restart the reduction buffer serves
template <class Take>
void layout_common(Layout& L, Take& take, int64_t n, int m, int nsplit, int comps) {
    const size_t d = sizeof(double), f = sizeof(float);
    L.x = take(3 * n * d);
    L.nrm = take(3 * n * d);
    L.w = take(n * d);
    L.wn = take(3 * n * d);
    const int64_t nt = (n + kTile - 1) / kTile, npad = nt * kTile;
    L.px = take(3 * npad * d);
    L.pn = take(3 * npad * d);
    L.pw = take(npad * d);
    L.px32 = take(3 * npad * f);
    L.boxes = take(nt * 6 * d);
    L.uboxes = take(npad / kNearUnit * 6 * d);
    L.mask64 = take(nt * nt);
    L.mask32 = take(nt * nt);
    L.perm = take(n * sizeof(int32_t));
    L.keys = take(next_pow2(n) * sizeof(uint64_t));
    L.partial = take((size_t)2 * nsplit * comps * n * d);
    L.rec = take((size_t)npad * kRecBytes);
    L.red = take((size_t)kRedBlocks * (m + 2) * d);
    L.scal = take((size_t)(kScalGmres + 6 * (m + 2) + 64 > 1024 ? kScalGmres + 6 * (m + 2) + 64 : 1024) * d);
}

Layout layout(int64_t n, int m) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t d = sizeof(double);
    layout_common(L, take, n, m, choose_splits(n), 6);  // up to six components per pass (adjoint)
    L.vecs = take((size_t)kNumVec * 3 * n * d);
    L.basis_in = take((size_t)(m + 1) * 3 * n * d);
    L.basis_out = take((size_t)(m + 1) * n * d);
    L.image_out = take((size_t)(m + 1) * kImageStride * n * d);
    L.basis_rc = take((size_t)(m + 1) * 3 * n * d);
    const int64_t nt = (n + kTile - 1) / kTile;
    if (sym_fits(nt)) {
        for (int k = 0; k < 2; ++k) {
            L.sym_items[k] = take((size_t)sym_max_pairs(nt) * 3 * sizeof(int32_t));
            L.sym_blocks[k] = take((size_t)sym_max_blocks(nt) * 2 * sizeof(int32_t));
            L.sym_fwd_start[k] = take((size_t)(nt + 1) * sizeof(int32_t));
            L.sym_rev_start[k] = take((size_t)(nt + 1) * sizeof(int32_t));
        }
        L.sym_fwd = take((size_t)sym_max_blocks(nt) * 3 * kTile * d);
        L.sym_rev = take((size_t)sym_max_pairs(nt) * 3 * kTile * d);  // double partials for the FP64 passes
    }
    L.total = off;
    return L;
}

void fail(int code, const std::string& msg) { throw Error(code, msg); }

void check_finite_pos(double v, const char* name) {
    if (!(std::isfinite(v) && v > 0.0)) fail(SDBIE_ERR_ARG, std::string(name) + " must be finite and > 0");
}

Plan& plan_of(sdbie_plan p) {
    if (!p) fail(SDBIE_ERR_ARG, "null plan");
    return *reinterpret_cast<Plan*>(p);
}

void check_params(const sdbie_params* prm) {
    if (!prm) fail(SDBIE_ERR_ARG, "null params");
    check_finite_pos(prm->mu, "mu");
    check_finite_pos(prm->K, "K");
    if (!(std::isfinite(prm->alpha) && prm->alpha >= 0.0)) fail(SDBIE_ERR_ARG, "alpha must be finite and >= 0");
}

sdbie_opts checked_opts(const sdbie_opts* op, const Plan& P) {
    sdbie_opts o;
    sdbie_default_opts(&o);
    if (op) o = *op;
    check_finite_pos(o.tol_gmres, "tol_gmres");
    check_finite_pos(o.tol_ddm, "tol_ddm");
    if (!(o.theta > 0.0 && o.theta < 1.0)) fail(SDBIE_ERR_ARG, "theta must lie in (0, 1)");
    if (o.restart < 1 || o.restart > P.max_restart)
        fail(SDBIE_ERR_ARG, "restart must lie in [1, max_restart of the plan]");
    if (o.maxit_gmres < 1 || o.maxit_ddm < 1) fail(SDBIE_ERR_ARG, "iteration limits must be >= 1");
    if (o.outer != 0 && o.outer != 1) fail(SDBIE_ERR_ARG, "outer must be 0 or 1");
    if (o.slip != 0 && o.slip != 1) fail(SDBIE_ERR_ARG, "slip must be 0 or 1");
    if (o.prec != SDBIE_FP64 && o.prec != SDBIE_MIXED) fail(SDBIE_ERR_ARG, "prec must be SDBIE_FP64 or SDBIE_MIXED");
    if (!(o.tol_mixed > 0.0 && o.tol_mixed < 1.0)) fail(SDBIE_ERR_ARG, "tol_mixed must lie in (0, 1)");
    if (o.refine_max < 1) fail(SDBIE_ERR_ARG, "refine_max must be >= 1");
    if (o.mixed_mode < 0 || o.mixed_mode > 2) fail(SDBIE_ERR_ARG, "mixed_mode must be 0, 1 or 2");
    if (o.relax_outer != 0 && o.relax_outer != 1) fail(SDBIE_ERR_ARG, "relax_outer must be 0 or 1");
    if (o.local_solver != 0 && o.local_solver != 1) fail(SDBIE_ERR_ARG, "local_solver must be 0 or 1");
    if (o.recycle != 0 && o.recycle != 1) fail(SDBIE_ERR_ARG, "recycle must be 0 or 1");
    return o;
}

template <class F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SDBIE_ERR_DEVICE;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SDBIE_ERR_DEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return SDBIE_ERR_DEVICE;
    }
}

hipStream_t stream_of(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool is_zero(Ctx& c, const double* a, int64_t len) { return c.norm(a, len) == 0.0; }

int layer_splits(int64_t n, int nsplit_cap) {
    const int S = choose_splits(n);
    return S < nsplit_cap ? S : nsplit_cap;
}

// layer applies only: the common part with at most nsplit_cap splits and three
// components per slot, then one [3][n] vector for the gathered density
Layout layer_layout(int64_t n, int nsplit_cap) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    layout_common(L, take, n, 1, layer_splits(n, nsplit_cap), 3);
    L.vecs = take((size_t)3 * n * sizeof(double));
    L.total = off;
    return L;
}

void carve_common(Plan& P, const Layout& L, char* b) {
    P.x = reinterpret_cast<double*>(b + L.x);
    P.nrm = reinterpret_cast<double*>(b + L.nrm);
    P.w = reinterpret_cast<double*>(b + L.w);
    P.wn = reinterpret_cast<double*>(b + L.wn);
    P.ntiles = (int)((P.n + kTile - 1) / kTile);
    P.npad = (int64_t)P.ntiles * kTile;
    P.px = reinterpret_cast<double*>(b + L.px);
    P.pn = reinterpret_cast<double*>(b + L.pn);
    P.pw = reinterpret_cast<double*>(b + L.pw);
    P.px32 = reinterpret_cast<float*>(b + L.px32);
    P.boxes = reinterpret_cast<double*>(b + L.boxes);
    P.uboxes = reinterpret_cast<double*>(b + L.uboxes);
    P.mask64 = reinterpret_cast<uint8_t*>(b + L.mask64);
    P.mask32 = reinterpret_cast<uint8_t*>(b + L.mask32);
    P.perm = reinterpret_cast<int32_t*>(b + L.perm);
    P.keys = reinterpret_cast<uint64_t*>(b + L.keys);
    P.npow2 = next_pow2(P.n);
    P.partial = reinterpret_cast<double*>(b + L.partial);
    P.rec = b + L.rec;
    P.red = reinterpret_cast<double*>(b + L.red);
    P.scal = reinterpret_cast<double*>(b + L.scal);
}

}  // namespace

size_t workspace_bytes(int64_t n, int max_restart) { return layout(n, max_restart).total; }

void carve_workspace(Plan& P, void* ws) {
    const Layout L = layout(P.n, P.max_restart);
    char* b = static_cast<char*>(ws);
    carve_common(P, L, b);
    P.nsplit = choose_splits(P.n);
    P.max_comps = 6;
    P.vecs = reinterpret_cast<double*>(b + L.vecs);
    P.basis_in = reinterpret_cast<double*>(b + L.basis_in);
    P.basis_out = reinterpret_cast<double*>(b + L.basis_out);
    P.image_out = reinterpret_cast<double*>(b + L.image_out);
    P.basis_rc = reinterpret_cast<double*>(b + L.basis_rc);
    if (!sym_fits((P.n + kTile - 1) / kTile)) return;  // no symmetric lists: every pass one direction
    for (int k = 0; k < 2; ++k) {
        P.sym_items[k] = reinterpret_cast<int32_t*>(b + L.sym_items[k]);
        P.sym_blocks[k] = reinterpret_cast<int32_t*>(b + L.sym_blocks[k]);
        P.sym_fwd_start[k] = reinterpret_cast<int32_t*>(b + L.sym_fwd_start[k]);
        P.sym_rev_start[k] = reinterpret_cast<int32_t*>(b + L.sym_rev_start[k]);
    }
    P.sym_fwd = reinterpret_cast<double*>(b + L.sym_fwd);
    P.sym_rev = b + L.sym_rev;
}

size_t layer_workspace_bytes(int64_t n, int nsplit_cap) { return layer_layout(n, nsplit_cap).total; }

void carve_layer_workspace(Plan& P, void* ws, int nsplit_cap, double** in) {
    const Layout L = layer_layout(P.n, nsplit_cap);
    char* b = static_cast<char*>(ws);
    carve_common(P, L, b);
    P.nsplit = layer_splits(P.n, nsplit_cap);
    P.max_comps = 3;
    *in = reinterpret_cast<double*>(b + L.vecs);
}

void apply_laplace_layer(Plan& P, sdbie_layer layer, const double* dens, double* out, sdbie_precision prec,
                         hipStream_t st, double* in) {
    if (!dens || !out) fail(SDBIE_ERR_ARG, "null density or output");
    if (dens == out) fail(SDBIE_ERR_ARG, "output aliases the density");
    if (prec != SDBIE_FP64 && prec != SDBIE_MIXED) fail(SDBIE_ERR_ARG, "bad precision");
    PassDesc d;
    switch (layer) {
        case SDBIE_SL: d.sl = true; d.c_sl = -1.0 / (4.0 * kPi); d.sl_dens = in; break;
        case SDBIE_DL_RAW: d.dl = true; d.c_dl = -1.0 / (4.0 * kPi); d.dl_dens = in; break;
        case SDBIE_DL_SUB: d.dl = true; d.sub = true; d.c_dl = 1.0 / (4.0 * kPi); d.dl_dens = in; break;
        default: fail(SDBIE_ERR_ARG, "bad layer");
    }
    dev_gather(P, dens, in, 1, st);
    d.mixed = prec == SDBIE_MIXED;
    d.out = out;
    d.scatter = true;
    launch_laplace_pass(P, d, st);
}

void apply_stokes_layer(Plan& P, double mu, sdbie_layer layer, const double* dens, double* out,
                        sdbie_precision prec, hipStream_t st, double* in) {
    if (!dens || !out) fail(SDBIE_ERR_ARG, "null density or output");
    if (dens == out) fail(SDBIE_ERR_ARG, "output aliases the density");
    if (prec != SDBIE_FP64 && prec != SDBIE_MIXED) fail(SDBIE_ERR_ARG, "bad precision");
    PassDesc d;
    switch (layer) {
        case SDBIE_SL:
            check_finite_pos(mu, "mu");
            d.sl = true; d.c_sl = 1.0 / (8.0 * kPi * mu); d.sl_dens = in;
            break;
        case SDBIE_DL_RAW: d.dl = true; d.c_dl = -3.0 / (4.0 * kPi); d.dl_dens = in; break;
        case SDBIE_DL_SUB:
            d.dl = true; d.sub = true; d.c_dl = -3.0 / (4.0 * kPi); d.dl_dens = in; d.base = in;
            break;
        default: fail(SDBIE_ERR_ARG, "bad layer");
    }
    dev_gather(P, dens, in, 3, st);
    d.mixed = prec == SDBIE_MIXED;
    d.out = out;
    d.scatter = true;
    launch_stokes_pass(P, d, st);
}

}  // namespace sdbie

using namespace sdbie;

extern "C" {

void sdbie_default_opts(sdbie_opts* o) {
    if (!o) return;
    o->tol_gmres = 1e-10;
    o->tol_ddm = 1e-8;
    o->theta = 0.5;
    o->maxit_gmres = 500;
    o->restart = 50;
    o->maxit_ddm = 200;
    o->outer = 1;
    o->slip = 0;
    o->prec = SDBIE_FP64;
    o->tol_mixed = 1e-4;
    o->refine_max = 8;
    o->mixed_mode = 2;
    o->relax_outer = 1;
    o->local_solver = 0;
    o->recycle = 1;
}

size_t sdbie_workspace_bytes(int64_t n, int max_restart) {
    if (n < 1 || n > kMaxNodes || max_restart < 1 || max_restart > kMaxRestart) return 0;
    return workspace_bytes(n, max_restart);
}

int sdbie_abi_version(void) { return 4; }

const char* sdbie_last_error(void) { return g_last_error.c_str(); }

int sdbie_plan_create(sdbie_plan* out, const sdbie_surface* s, int max_restart, void* ws, size_t ws_bytes,
                      void* stream) {
    return guarded([&]() -> int {
        if (!out) fail(SDBIE_ERR_ARG, "null plan pointer");
        *out = nullptr;
        if (!s || !s->x || !s->nrm || !s->w) fail(SDBIE_ERR_ARG, "null surface array");
        if (s->n < 1 || s->n > kMaxNodes) fail(SDBIE_ERR_ARG, "n must lie in [1, 2^23]");
        check_finite_pos(s->delta, "delta");
        if (s->delta < kMinDelta || s->delta > kMaxCoord) fail(SDBIE_ERR_ARG, "delta must lie in [1e-15, 1e15]");
        if (max_restart < 1 || max_restart > kMaxRestart) fail(SDBIE_ERR_ARG, "max_restart must lie in [1, 1000]");
        if (!ws) fail(SDBIE_ERR_WORKSPACE, "null workspace");
        if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) fail(SDBIE_ERR_WORKSPACE, "workspace not 256-byte aligned");
        const size_t need = workspace_bytes(s->n, max_restart);
        if (ws_bytes < need)
            fail(SDBIE_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
        Plan* P = new Plan();
        P->n = s->n;
        P->max_restart = max_restart;
        P->delta = s->delta;
        carve_workspace(*P, ws);
        try {
            stage_surface(*P, s, stream_of(stream));
        } catch (...) {
            delete P;
            throw;
        }
        *out = reinterpret_cast<sdbie_plan>(P);
        return SDBIE_OK;
    });
}

int sdbie_plan_destroy(sdbie_plan plan) {
    delete reinterpret_cast<Plan*>(plan);
    return SDBIE_OK;
}

int64_t sdbie_plan_n(sdbie_plan plan) { return plan ? reinterpret_cast<Plan*>(plan)->n : -1; }

int sdbie_plan_set_symmetric(sdbie_plan plan, int families) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        if (families & ~SDBIE_SYM_ALL) fail(SDBIE_ERR_ARG, "unknown pass kind bits");
        P.symmetric = families;
        return SDBIE_OK;
    });
}

int laplace_layer_apply(sdbie_plan plan, sdbie_layer layer, const double* dens, double* out, sdbie_precision prec,
                        void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        apply_laplace_layer(P, layer, dens, out, prec, stream_of(stream), P.vec(kVecIn));
        return SDBIE_OK;
    });
}

int stokes_layer_apply(sdbie_plan plan, double mu, sdbie_layer layer, const double* dens, double* out,
                       sdbie_precision prec, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        apply_stokes_layer(P, mu, layer, dens, out, prec, stream_of(stream), P.vec(kVecIn));
        return SDBIE_OK;
    });
}

int stokes_layer_apply_noalloc(const sdbie_surface* s, double mu, sdbie_layer layer, const double* dens,
                               double* out, sdbie_precision prec, void* stream) {
    return guarded([&]() -> int {
        stokes_layer_apply_static(s, mu, layer, dens, out, prec, stream_of(stream));
        return SDBIE_OK;
    });
}

int darcy_solve(sdbie_plan plan, const sdbie_params* prm, const double* vn, double* p, const sdbie_opts* opts,
                sdbie_info* info, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        check_params(prm);
        if (!vn || !p) fail(SDBIE_ERR_ARG, "null vn or p");
        const sdbie_opts o = checked_opts(opts, P);
        Ctx c(P, stream_of(stream), o);
        double* v = P.vec(kVecIn);
        double* ps = P.vec(kVecP);
        dev_gather(P, vn, v, 1, c.s);
        dev_gather(P, p, ps, 1, c.s);
        c.darcy(*prm, v, ps, !is_zero(c, ps, P.n), nullptr);
        dev_scatter(P, ps, p, 1, c.s);
        SDBIE_HIP(hipStreamSynchronize(c.s));
        c.finish();
        if (info) *info = c.info;
        return c.converged ? SDBIE_OK : SDBIE_NOT_CONVERGED;
    });
}

int stokes_solve(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* p, const double* f_extra,
                 double* u, const sdbie_opts* opts, sdbie_info* info, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        check_params(prm);
        if (!U || !p || !u) fail(SDBIE_ERR_ARG, "null U, p or u");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(U[k])) fail(SDBIE_ERR_ARG, "non-finite U");
        const sdbie_opts o = checked_opts(opts, P);
        Ctx c(P, stream_of(stream), o);
        double* ps = P.vec(kVecP);
        double* us = P.vec(kVecU);
        double* fx = f_extra ? P.vec(kVecFx) : nullptr;
        dev_gather(P, p, ps, 1, c.s);
        dev_gather(P, u, us, 3, c.s);
        if (fx) dev_gather(P, f_extra, fx, 3, c.s);
        c.stokes(*prm, U, ps, fx, us, !is_zero(c, us, 3 * P.n), nullptr);
        dev_scatter(P, us, u, 3, c.s);
        SDBIE_HIP(hipStreamSynchronize(c.s));
        c.finish();
        if (info) *info = c.info;
        return c.converged ? SDBIE_OK : SDBIE_NOT_CONVERGED;
    });
}

int ddm_solve(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* f_extra, double* p,
              double* u, double drag[3], const sdbie_opts* opts, sdbie_info* info, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        check_params(prm);
        if (!U || !p || !u || !drag) fail(SDBIE_ERR_ARG, "null U, p, u or drag");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(U[k])) fail(SDBIE_ERR_ARG, "non-finite U");
        const sdbie_opts o = checked_opts(opts, P);
        if (o.outer == 1 && o.slip == 1 && prm->alpha != 0.0)
            fail(SDBIE_ERR_ARG, "outer GMRES needs the implicit slip form (slip = 0)");
        Ctx c(P, stream_of(stream), o);
        double* ps = P.vec(kVecP);
        double* us = P.vec(kVecU);
        double* fx = f_extra ? P.vec(kVecFx) : nullptr;
        if (fx) dev_gather(P, f_extra, fx, 3, c.s);
        c.ddm(*prm, U, fx, ps, us, drag);
        dev_scatter(P, ps, p, 1, c.s);
        dev_scatter(P, us, u, 3, c.s);
        SDBIE_HIP(hipStreamSynchronize(c.s));
        c.finish();
        if (info) *info = c.info;
        return c.converged ? SDBIE_OK : SDBIE_NOT_CONVERGED;
    });
}

int ddm_adjoint(sdbie_plan plan, const sdbie_params* prm, const double U[3], const double* f_extra, const double* p,
                const double* u, const double dJ_ddrag[3], double* dJ_dx, double* dJ_dlogK, double* dJ_dalpha,
                const sdbie_opts* opts, sdbie_info* info, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        check_params(prm);
        if (!U || !p || !u || !dJ_ddrag || !dJ_dx || !dJ_dlogK || !dJ_dalpha)
            fail(SDBIE_ERR_ARG, "null argument");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(U[k]) || !std::isfinite(dJ_ddrag[k])) fail(SDBIE_ERR_ARG, "non-finite U or dJ_ddrag");
        const sdbie_opts o = checked_opts(opts, P);
        Ctx c(P, stream_of(stream), o);
        double* ps = P.vec(kVecP);
        double* us = P.vec(kVecU);
        double* fx = f_extra ? P.vec(kVecFx) : nullptr;
        double* gs = P.vec(kVecSpare);
        dev_gather(P, p, ps, 1, c.s);
        dev_gather(P, u, us, 3, c.s);
        if (fx) dev_gather(P, f_extra, fx, 3, c.s);
        c.adjoint(*prm, U, fx, ps, us, dJ_ddrag, gs, dJ_dlogK, dJ_dalpha);
        dev_scatter(P, gs, dJ_dx, 3, c.s);
        SDBIE_HIP(hipStreamSynchronize(c.s));
        c.finish();
        if (info) *info = c.info;
        return c.converged ? SDBIE_OK : SDBIE_NOT_CONVERGED;
    });
}

int ddm_dn_spectrum(sdbie_plan plan, const sdbie_params* prm, const double* v0, int m, int k, double* eig_re,
                    double* eig_im, const sdbie_opts* opts, sdbie_info* info, void* stream) {
    return guarded([&]() -> int {
        Plan& P = plan_of(plan);
        check_params(prm);
        if (!v0 || !eig_re || !eig_im) fail(SDBIE_ERR_ARG, "null start vector or eigenvalue array");
        if (m < 1 || m > P.max_restart) fail(SDBIE_ERR_ARG, "m must lie in [1, max_restart of the plan]");
        if (k < 1 || k > m) fail(SDBIE_ERR_ARG, "k must lie in [1, m]");
        const sdbie_opts o = checked_opts(opts, P);
        if (o.slip != 0 && prm->alpha != 0.0) fail(SDBIE_ERR_ARG, "the D-N map is linear with implicit slip only");
        Ctx c(P, stream_of(stream), o);
        double* v = P.vec(kVecIn);
        dev_gather(P, v0, v, 1, c.s);
        std::vector<double> H;
        const int used = c.dn_arnoldi(*prm, v, m, H);
        std::vector<double> A((size_t)used * used), wr(used), wi(used);
        for (int i = 0; i < used; ++i)
            for (int j = 0; j < used; ++j) A[(size_t)i * used + j] = H[(size_t)i * m + j];
        const bool qr_ok = hessenberg_eigenvalues(used, A.data(), wr.data(), wi.data());
        if (!qr_ok) g_last_error = "the Hessenberg QR iteration did not converge";
        // decreasing modulus; eigenvalues the QR iteration did not reach (NaN) last
        auto mod = [&](int i) { return std::isnan(wr[i]) ? -1.0 : std::hypot(wr[i], wi[i]); };
        std::vector<int> order(used);
        for (int i = 0; i < used; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mod(a) > mod(b); });
        for (int i = 0; i < k; ++i) {
            eig_re[i] = i < used ? wr[order[i]] : NAN;
            eig_im[i] = i < used ? wi[order[i]] : NAN;
        }
        c.info.ddm_iters = used;
        c.finish();
        if (info) *info = c.info;
        return c.converged && qr_ok ? SDBIE_OK : SDBIE_NOT_CONVERGED;
    });
}

int sdbie_hessenberg_eigenvalues(int n, const double* H, double* eig_re, double* eig_im) {
    return guarded([&]() -> int {
        if (n < 1 || !H || !eig_re || !eig_im) fail(SDBIE_ERR_ARG, "bad Hessenberg eigenvalue arguments");
        std::vector<double> A(H, H + (size_t)n * n);
        for (int i = 2; i < n; ++i)
            for (int j = 0; j < i - 1; ++j) A[(size_t)i * n + j] = 0.0;  // only the Hessenberg part is read
        if (!hessenberg_eigenvalues(n, A.data(), eig_re, eig_im)) {
            g_last_error = "the Hessenberg QR iteration did not converge";
            return SDBIE_NOT_CONVERGED;
        }
        return SDBIE_OK;
    });
}

}  // extern "C"
