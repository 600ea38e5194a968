// Optional kernel timing: a HIP event pair around every pair-sum kernel.
//
// When enabled (sdbie_profile_enable(1)), each launch of a pair-sum kernel
// records an event before and after it on the stream it is launched on.
// sdbie_profile_read() waits for the recorded events and reports, per kernel
// variant, the launch count, the summed kernel time, the pair evaluations and
// the algorithmic flop count per pair (far field: FMA = 2, add/mul = 1,
// each rsqrt = 1; the near-field smoothing is not counted).
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace sdbie {
namespace {

struct Rec {
    int variant;
    double pairs;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;

}  // namespace

// variant = ((family * 8 + part) * 2 + mixed) * 32 + code
// family: 0 Laplace, 1 Stokes, 2 position gradient; part: 0 far kernel,
// 1 near kernel, 2 source-record packing, 3 far and near blocks in one
// launch, 4 the same with a target-source symmetric far field; code: DL 1,
// SL 2, SUB 4, SLIP 8, transposed (target normal) 16.
int prof_variant(int family, bool mixed, int code, int part) {
    return ((family * 8 + part) * 2 + (mixed ? 1 : 0)) * 32 + code;
}

namespace {
void decode(int v, int& family, int& part, int& mixed, int& code) {
    code = v & 31;
    mixed = (v >> 5) & 1;
    part = (v >> 6) & 7;
    family = v >> 9;
}

// Flops of one unordered far pair in the symmetric form (both directions,
// the shared geometry once), halved: per ordered pair.
double symmetric_flops_per_pair(int family, bool dl, bool sl, bool sub) {
    const double common = 9.0;  // D (3), r^2 (5), rsqrt (1)
    double f = common;
    if (family == 0) {
        if (dl) f += 2 + 5 + 5 + 4;  // k2, D.n_s, D.n_t, the two products with (q_s - q_t) or q
        if (sl) f += 4;              // g_s k1, g_t k1
        f += 2;                      // the two accumulations
        return 0.5 * f;
    }
    f += 1;  // 1/r^2
    if (dl) f += (sub ? 3 : 0) + 5 + (sub ? 0 : 6) + 5 + 5;  // u_s - u_t, ud, ud' (no subtraction), D.n_s, D.n_t
    if (sl) {
        f += 1 + 5 + 5 + (dl ? 6 : 2);  // 1/r^3, D.f_s, D.f_t, the two coefficients
        f += 12 + 9;                    // forward 1/r f_s + e D, reverse 1/r f_t + e D
    } else {
        f += 2 + 4 + 6 + 3;  // 1/r^5, the two coefficients, e D forward and reverse
    }
    f += 3;  // the reverse additions
    return 0.5 * f;
}
}  // namespace

std::string prof_name(int v) {
    int family, part, mixed, code;
    decode(v, family, part, mixed, code);
    static const char* parts[] = {"far", "near", "pack", "pass", "sympass", "?", "?", "?"};
    std::string s = family == 0 ? "laplace" : family == 1 ? "stokes" : "position_gradient";
    if (code & 16) s += "_T";
    s += std::string("_") + parts[part] + "<" + (mixed ? "f32" : "f64");
    if (family < 2) {
        if (code & 1) s += ",DL";
        if (code & 2) s += ",SL";
        if (code & 4) s += ",SUB";
        if (code & 8) s += ",SLIP";
    }
    return s + ">";
}

// Algorithmic flops of one pair in the far-field form the kernels evaluate
// (an FMA counts two; the near kernel's smoothing branch is not counted); 0
// for the packing kernel.
double flops_per_pair(int v) {
    int family, part, mixed, code;
    decode(v, family, part, mixed, code);
    const bool dl = code & 1, sl = code & 2, sub = code & 4;
    if (family == 2 || part == 2) return 0.0;  // gradient: not counted
    if (part == 4) return symmetric_flops_per_pair(family, dl, sl, sub);
    // common: D (3), r^2 (1 mul + 2 fma = 5), rsqrt (1)
    const double common = 9.0;
    if (code & 16) {
        if (family == 0) return common + 2 + 5 + 3;  // k2 (2), D.n_i (5), acc += (q dn) k2 (3)
        // transposed stresslet: ir2, k3, k4 (3), q.D (5), D.n_i (5), c (2), acc += c D (6);
        // with the Stokeslet of the same density: cs = (q.D) k3 (1), acc2 += q k1 + cs D (12)
        return common + 3 + 5 + 5 + 2 + 6 + (sl ? 1 + 12 : 0);
    }
    if (family == 0) {
        double f = common;
        if (dl) f += 2 + 5 + (sub ? 4 : 3);  // k2 = inv_r^3 (2), D.n (5), (q_j - q_i) dn k2 + acc
        if (sl) f += 2;                      // acc += g k1
        return f;
    }
    if (sl) {
        // acc += (1/r) [f + D ir2 ((u.D)(D.n) ir2 + D.f)]: ir2 (1), D.f (5), c *= ir2 (1),
        // per component fma(c, d, f) and fma(., 1/r, acc) (12); the double layer adds
        // u_j - u_i (3), u.D (5), D.n (5), (u.D)(D.n) (1) and its fma into c (2)
        return common + 1 + 5 + 1 + 12 + (dl ? (sub ? 3 : 0) + 5 + 5 + 1 + 2 : 0);
    }
    // double layer alone: ir2, k3, k4 (3), u_j - u_i, u.D, D.n, c = (u.D)(D.n) k4 (2), acc += c D
    return common + 3 + (sub ? 3 : 0) + 5 + 5 + 2 + 6;
}

ProfScope::ProfScope(int variant, double pairs, hipStream_t s) : s_(s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    Rec r{variant, pairs, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    g_recs.push_back(r);
    idx_ = (long)g_recs.size() - 1;
}

ProfScope::~ProfScope() {
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (idx_ < (long)g_recs.size()) (void)hipEventRecord(g_recs[idx_].b, s_);
}

}  // namespace sdbie

extern "C" {

int sdbie_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(sdbie::g_mu);
    for (auto& r : sdbie::g_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    sdbie::g_recs.clear();
    sdbie::g_on = on != 0;
    return SDBIE_OK;
}

int sdbie_profile_read(sdbie_kernel_stat* out, int max, int* count) {
    std::lock_guard<std::mutex> lk(sdbie::g_mu);
    if (!count || (max > 0 && !out)) return SDBIE_ERR_ARG;
    std::vector<sdbie_kernel_stat> acc;
    std::vector<int> ids;
    for (auto& r : sdbie::g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return SDBIE_ERR_DEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SDBIE_ERR_DEVICE;
        size_t k = 0;
        while (k < ids.size() && ids[k] != r.variant) ++k;
        if (k == ids.size()) {
            ids.push_back(r.variant);
            sdbie_kernel_stat st;
            std::memset(&st, 0, sizeof(st));
            std::strncpy(st.name, sdbie::prof_name(r.variant).c_str(), sizeof(st.name) - 1);
            st.flops_per_pair = sdbie::flops_per_pair(r.variant);
            acc.push_back(st);
        }
        acc[k].launches += 1;
        acc[k].ms += ms;
        acc[k].pairs += r.pairs;
    }
    *count = (int)acc.size();
    for (int i = 0; i < (int)acc.size() && i < max; ++i) out[i] = acc[i];
    return SDBIE_OK;
}

}  // extern "C"
