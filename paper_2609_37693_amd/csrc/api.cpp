// C-ABI of libozemu: argument validation, workspace layout and the call
// pipeline of Sec. V-A (Scale, Reduce, GEMMs with fused epilogue,
// Reconstruct) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ozemu.h"
#include "ozemu_internal.hpp"
#include "plan.hpp"
#include "slabs.hpp"

struct ozemu_plan_s {
    ozemu::Plan p;
};

// A grouped product: per-problem descriptors, plan constants and work
// prefixes, laid out as they are copied to the start of the workspace.
struct ozemu_group_s {
    int count = 0, nplans = 0, dmax = 2;
    bool big = false;  // some problem keeps more than kSmallBits bits
    size_t table_bytes = 0, ws_bytes = 0;
    size_t off_probs = 0, off_mods = 0, off_crts = 0, off_prefix = 0, off_order = 0,
           off_counter = 0;
    int32_t total[ozemu::kGKinds] = {};
    std::vector<char> tables;  // table_bytes, built at creation
    char* pinned = nullptr;    // pinned copy for the uploads, made by the first run
};

namespace {

thread_local std::string g_last_error;

ozemu_status fail(ozemu_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

ozemu_status ok() { return OZEMU_OK; }

ozemu_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return OZEMU_OK;
    return fail(OZEMU_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t round_up(int64_t v, int64_t t) { return (v + t - 1) / t * t; }

struct Dims {
    int64_t m_pad, n_pad, k_pad;
};

Dims dims_of(int64_t m, int64_t n, int64_t k) {
    return {round_up(m, ozemu::kTileM), round_up(n, ozemu::kTileN), round_up(k, ozemu::kTileK)};
}

// Float-channel plans: K padded to whole 64-byte plane blocks (128 values
// for FP4, two per byte).
Dims dims_of(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    if (p.format == OZEMU_E2M1)
        return {round_up(m, ozemu::kTileM), round_up(n, ozemu::kTileN), round_up(k, 128)};
    return dims_of(m, n, k);
}

bool is_fp(const ozemu::Plan& p) { return p.format != OZEMU_INT8; }

// bytes of a float plane row of k_pad values (FP6 packed: 48 bytes per 64)
int64_t fp_row_bytes(const ozemu::Plan& p, int64_t k_pad) {
    if (p.format == OZEMU_E2M1) return k_pad / 2;
    if (p.format == OZEMU_E2M3) return k_pad / 4 * 3;
    return k_pad;
}

struct Layout {
    size_t key_a, key_b, shift_a, shift_b, planes_a, planes_b, residues, bar_a, bar_b, gmax_a,
        gmax_b, tables, total;
};

Layout layout_of(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    Dims d = dims_of(p, m, n, k);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t N = (size_t)p.n;
    if (is_fp(p)) {
        const size_t planes = (size_t)p.fp.planes, kb = (size_t)fp_row_bytes(p, d.k_pad);
        L.shift_a = take(sizeof(int32_t) * (size_t)d.m_pad);
        L.shift_b = take(sizeof(int32_t) * (size_t)d.n_pad);
        L.tables = take(p.tables.size());
        L.planes_a = take(planes * (size_t)d.m_pad * kb);
        L.planes_b = take(planes * (size_t)d.n_pad * kb);
        L.residues = take(sizeof(uint16_t) * N * (size_t)d.m_pad * (size_t)d.n_pad);
        L.total = off;
        return L;
    }
    L.key_a = take(sizeof(int32_t) * (size_t)d.m_pad);
    L.key_b = take(sizeof(int32_t) * (size_t)d.n_pad);
    L.shift_a = take(sizeof(int32_t) * (size_t)d.m_pad);
    L.shift_b = take(sizeof(int32_t) * (size_t)d.n_pad);
    L.planes_a = take(N * (size_t)d.m_pad * (size_t)d.k_pad);
    L.planes_b = take(N * (size_t)d.n_pad * (size_t)d.k_pad);
    L.residues = take(N * (size_t)d.m_pad * (size_t)d.n_pad);
    if (p.scaling == OZEMU_SCALE_BOUND) {
        L.bar_a = take((size_t)d.m_pad * (size_t)d.k_pad);
        L.bar_b = take((size_t)d.n_pad * (size_t)d.k_pad);
        L.gmax_a = take(sizeof(int32_t) * (size_t)d.m_pad);
        L.gmax_b = take(sizeof(int32_t) * (size_t)d.n_pad);
    }
    L.total = off;
    return L;
}

// Scale-phase workspace needs: only the bound-adaptive mode uses it.
size_t scale_ws_need(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    return p.scaling == OZEMU_SCALE_BOUND ? layout_of(p, m, n, k).total : 0;
}

ozemu_status check_plan(ozemu_plan plan) {
    if (!plan) return fail(OZEMU_ERR_INVALID_ARG, "plan is NULL");
    return ok();
}

// The reconstruction caps of the whole inner dimension (modes F53 and W);
// the accumulation cap is checked separately.
ozemu_status check_window(const ozemu::Plan& p, int64_t k) {
    if (p.scaling == OZEMU_SCALE_F53 && k > 0 && !ozemu::window_holds(p, k, 53, 53))
        return fail(OZEMU_ERR_K_TOO_LARGE,
                    "k = " + std::to_string(k) +
                        " exceeds the reconstruction cap of this modulus set at 53 bits");
    if (p.scaling == OZEMU_SCALE_WINDOW && k > 0 && ozemu::window_bits(p, k) < 2)
        return fail(OZEMU_ERR_K_TOO_LARGE, "modulus product too small for this k");
    return ok();
}

ozemu_status check_shape(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    if (m > (1ll << 31) || n > (1ll << 31)) return fail(OZEMU_ERR_INVALID_ARG, "dimension too large");
    if (k > p.kappa_acc)
        return fail(OZEMU_ERR_K_TOO_LARGE,
                    "k = " + std::to_string(k) + " exceeds the INT32 accumulation cap " +
                        std::to_string(p.kappa_acc) + " of this modulus set");
    if (ozemu_status s = check_window(p, k)) return s;
    if (is_fp(p) && k > 0) {
        int ba = 53, bb = 53;
        if (p.scaling == OZEMU_SCALE_WINDOW) {
            const int w = ozemu::window_bits(p, k);
            ba = (w + 1) / 2, bb = w / 2;
        }
        if (ba > 63 || bb > 63)
            return fail(OZEMU_ERR_UNSUPPORTED, "float-channel plans keep at most 63 bits per entry");
    }
    if (p.scaling == OZEMU_SCALE_BOUND && k > 524287)
        return fail(OZEMU_ERR_K_TOO_LARGE, "bound product would overflow INT32");
    return ok();
}

ozemu_status check_operands(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                            const void* B, int64_t ldb) {
    if (m > 0 && k > 0) {
        if (!A) return fail(OZEMU_ERR_INVALID_ARG, "A is NULL");
        if (lda < k) return fail(OZEMU_ERR_INVALID_ARG, "lda < k");
    }
    if (k > 0 && n > 0) {
        if (!B) return fail(OZEMU_ERR_INVALID_ARG, "B is NULL");
        if (ldb < n) return fail(OZEMU_ERR_INVALID_ARG, "ldb < n");
    }
    return ok();
}

void kept_bits_of(const ozemu::Plan& p, int64_t k, int& ba, int& bb) {
    if (p.scaling == OZEMU_SCALE_F53) {
        ba = bb = 53;
        return;
    }
    int w = ozemu::window_bits(p, k);
    ba = (w + 1) / 2;
    bb = w / 2;
    if (ba > ozemu::kBetaCap) ba = ozemu::kBetaCap;
    if (bb > ozemu::kBetaCap) bb = ozemu::kBetaCap;
}

// True when some row or column may keep more than kSmallBits bits, so the
// encoder takes its exact form for any shift (with its shift table) (the bound mode's bits are decided on the device,
// up to kBetaCap).
bool big_encode(const ozemu::Plan& p, int64_t k) {
    if (p.scaling == OZEMU_SCALE_BOUND) return true;
    int ba, bb;
    kept_bits_of(p, k, ba, bb);
    return ba > ozemu::kSmallBits || bb > ozemu::kSmallBits;
}

// Scale with all arguments validated; ws may be NULL unless BOUND.
ozemu_status run_scale(const ozemu::Plan& p, hipStream_t st, int64_t m, int64_t n, int64_t k,
                       const double* A, int64_t lda, const double* B, int64_t ldb, int32_t* sa,
                       int32_t* sb, char* ws) {
    using namespace ozemu;
    if (p.scaling != OZEMU_SCALE_BOUND) {
        int ba, bb;
        kept_bits_of(p, k, ba, bb);
        if (k == 0) {
            ozemu_status s = hip_check(launch_fill_i32(st, m, 0, sa), "fill");
            if (s) return s;
            return hip_check(launch_fill_i32(st, n, 0, sb), "fill");
        }
        ozemu_status s = hip_check(launch_scale_rows(st, m, k, A, lda, sa), "scale_rows");
        if (s) return s;
        s = hip_check(launch_scale_cols(st, k, n, B, ldb, sb), "scale_cols");
        if (s) return s;
        s = hip_check(launch_keys_to_shifts(st, m, sa, ba, nullptr), "shifts_a");
        if (s) return s;
        return hip_check(launch_keys_to_shifts(st, n, sb, bb, nullptr), "shifts_b");
    }
    Layout L = layout_of(p, m, n, k);
    Dims d = dims_of(m, n, k);
    int32_t* key_a = reinterpret_cast<int32_t*>(ws + L.key_a);
    int32_t* key_b = reinterpret_cast<int32_t*>(ws + L.key_b);
    int8_t* bar_a = reinterpret_cast<int8_t*>(ws + L.bar_a);
    int8_t* bar_b = reinterpret_cast<int8_t*>(ws + L.bar_b);
    int32_t* gmax_a = reinterpret_cast<int32_t*>(ws + L.gmax_a);
    int32_t* gmax_b = reinterpret_cast<int32_t*>(ws + L.gmax_b);
    if (k == 0) {
        ozemu_status s = hip_check(launch_fill_i32(st, m, 0, sa), "fill");
        if (s) return s;
        return hip_check(launch_fill_i32(st, n, 0, sb), "fill");
    }
    ozemu_status s = hip_check(launch_scale_rows(st, m, k, A, lda, key_a), "scale_rows");
    if (!s) s = hip_check(launch_scale_cols(st, k, n, B, ldb, key_b), "scale_cols");
    if (!s)
        s = hip_check(launch_bound_planes_a(st, m, k, A, lda, key_a, d.m_pad, d.k_pad, bar_a),
                      "bound_planes_a");
    if (!s)
        s = hip_check(launch_bound_planes_b(st, k, n, B, ldb, key_b, d.n_pad, d.k_pad, bar_b),
                      "bound_planes_b");
    if (!s)
        s = hip_check(launch_bound_gemm(st, d.m_pad, d.n_pad, d.k_pad, bar_a, bar_b, gmax_a, gmax_b),
                      "bound_gemm");
    const int L2 = half_window_bits(p);
    if (!s) s = hip_check(launch_bound_shifts(st, m, key_a, gmax_a, L2, sa), "bound_shifts_a");
    if (!s) s = hip_check(launch_bound_shifts(st, n, key_b, gmax_b, L2, sb), "bound_shifts_b");
    return s;
}

// Kept bits of a cached forward: split at the largest inner dimension of
// the forward and both backward products, K* = max(m, n, k).
int64_t cache_k(int64_t m, int64_t n, int64_t k) { return std::max(std::max(m, n), k); }

// Kept bits of dY in a backward product of inner dimension `inner` against
// cached operand bits `cached`: all the window leaves (53 in F53).
int backward_bits(const ozemu::Plan& p, int64_t inner, int cached) {
    if (p.scaling == OZEMU_SCALE_F53) return 53;
    int b = ozemu::window_bits(p, inner) - cached;
    return b > ozemu::kBetaCap ? ozemu::kBetaCap : b;
}

ozemu_status check_cache_plan(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    if (is_fp(p)) return fail(OZEMU_ERR_UNSUPPORTED, "cached forward and backward take INT8 plans");
    if (p.scaling == OZEMU_SCALE_BOUND)
        return fail(OZEMU_ERR_UNSUPPORTED, "cached forward and backward support F53 and WINDOW");
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    if (k > (1ll << 31)) return fail(OZEMU_ERR_INVALID_ARG, "dimension too large");
    // every product's inner dimension (k, n, m) must pass the caps at K*
    return check_shape(p, m, n, cache_k(m, n, k));
}

// Backward workspace: the fold shifts, a zero shift vector and, shared by
// the two products in turn, the fresh operand's planes, the transposed
// cached planes and the residues.
struct BwdLayout {
    size_t shift_dx, shift_dw, zeros, planes_fresh, planes_t, residues, total;
};

BwdLayout bwd_layout_of(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k) {
    const size_t N = (size_t)p.n;
    const size_t mp = (size_t)round_up(m, ozemu::kTileM), np = (size_t)round_up(n, ozemu::kTileN);
    const size_t kp = (size_t)round_up(k, ozemu::kTileM);
    BwdLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.shift_dx = take(sizeof(int32_t) * mp);
    L.shift_dw = take(sizeof(int32_t) * np);
    L.zeros = take(sizeof(int32_t) * std::max(kp, (size_t)1));
    // dX: fresh mp x np, transposed W kp x np, residues mp x kp
    // dW: fresh np x mp, transposed X kp x mp, residues kp x np
    L.planes_fresh = take(N * mp * np);
    L.planes_t = take(N * kp * std::max(mp, np));
    L.residues = take(N * kp * std::max(mp, np));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

const char* ozemu_version(void) { return "ozemu 0.1 (gfx950)"; }

const char* ozemu_last_error(void) { return g_last_error.c_str(); }

const char* ozemu_status_string(int status) {
    switch (status) {
        case OZEMU_OK: return "OZEMU_OK";
        case OZEMU_ERR_INVALID_ARG: return "OZEMU_ERR_INVALID_ARG";
        case OZEMU_ERR_K_TOO_LARGE: return "OZEMU_ERR_K_TOO_LARGE";
        case OZEMU_ERR_UNSUPPORTED: return "OZEMU_ERR_UNSUPPORTED";
        case OZEMU_ERR_WORKSPACE: return "OZEMU_ERR_WORKSPACE";
        case OZEMU_ERR_HIP: return "OZEMU_ERR_HIP";
        default: return "unknown status";
    }
}

ozemu_status ozemu_plan_create_moduli(ozemu_plan* out, int format, int count,
                                      const int32_t* moduli, int scaling) {
    if (!out) return fail(OZEMU_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (format != OZEMU_INT8)
        return fail(OZEMU_ERR_UNSUPPORTED, "modulus plans are INT8; float formats: ozemu_plan_create_fp");
    if (count < 2 || count > ozemu::kMaxModuli || !moduli)
        return fail(OZEMU_ERR_INVALID_ARG, "number of moduli must be in [2, 32]");
    std::vector<int> ms(moduli, moduli + count);
    ozemu_plan p = new (std::nothrow) ozemu_plan_s;
    if (!p) return fail(OZEMU_ERR_INVALID_ARG, "out of host memory");
    std::string err = ozemu::build_plan(p->p, format, ms, scaling);
    if (!err.empty()) {
        delete p;
        return fail(OZEMU_ERR_INVALID_ARG, err);
    }
    *out = p;
    return ok();
}

ozemu_status ozemu_plan_create(ozemu_plan* out, int format, int num_moduli, int scaling) {
    if (!out) return fail(OZEMU_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (format != OZEMU_INT8)
        return fail(OZEMU_ERR_UNSUPPORTED, "modulus plans are INT8; float formats: ozemu_plan_create_fp");
    if (num_moduli < 2 || num_moduli > ozemu::kMaxModuli)
        return fail(OZEMU_ERR_INVALID_ARG, "number of moduli must be in [2, 32]");
    std::vector<int> ms = ozemu::best_coprime_set(num_moduli, 256);
    if ((int)ms.size() != num_moduli) return fail(OZEMU_ERR_INVALID_ARG, "no modulus set");
    std::vector<int32_t> m32(ms.begin(), ms.end());
    return ozemu_plan_create_moduli(out, format, num_moduli, m32.data(), scaling);
}

ozemu_status ozemu_plan_create_fp(ozemu_plan* out, int format, int gemms, int64_t k_slab,
                                  int scaling) {
    if (!out) return fail(OZEMU_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (format != OZEMU_E4M3 && format != OZEMU_E2M3 && format != OZEMU_E2M1)
        return fail(OZEMU_ERR_UNSUPPORTED,
                    "float plans are built for OZEMU_E4M3, OZEMU_E2M3 and OZEMU_E2M1");
    ozemu_plan p = new (std::nothrow) ozemu_plan_s;
    if (!p) return fail(OZEMU_ERR_INVALID_ARG, "out of host memory");
    std::string err = ozemu::build_plan_fp(p->p, format, gemms, k_slab, scaling);
    if (!err.empty()) {
        delete p;
        return fail(OZEMU_ERR_INVALID_ARG, err);
    }
    *out = p;
    return ok();
}

ozemu_status ozemu_plan_channels(ozemu_plan plan, int32_t* moduli, int32_t* ranks,
                                 int32_t* bases, int cap, int* count) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!count) return fail(OZEMU_ERR_INVALID_ARG, "count is NULL");
    const ozemu::Plan& p = plan->p;
    *count = p.n;
    if (moduli || ranks || bases) {
        if (cap < p.n) return fail(OZEMU_ERR_INVALID_ARG, "capacity too small");
        for (int i = 0; i < p.n; ++i) {
            const bool fp = is_fp(p);
            if (moduli) moduli[i] = fp ? p.chans[i].m : p.moduli[i];
            if (ranks) ranks[i] = fp ? p.chans[i].rank : 1;
            if (bases) bases[i] = fp ? p.chans[i].base : 0;
        }
    }
    return ok();
}

ozemu_status ozemu_plan_destroy(ozemu_plan plan) {
    if (plan && plan->p.pinned_tables) (void)hipHostFree(plan->p.pinned_tables);
    delete plan;
    return ok();
}

ozemu_status ozemu_plan_moduli(ozemu_plan plan, int32_t* out, int cap, int* count) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!count) return fail(OZEMU_ERR_INVALID_ARG, "count is NULL");
    *count = plan->p.n;
    if (out) {
        if (cap < plan->p.n) return fail(OZEMU_ERR_INVALID_ARG, "capacity too small");
        for (int i = 0; i < plan->p.n; ++i) out[i] = plan->p.moduli[i];
    }
    return ok();
}

ozemu_status ozemu_plan_kept_bits(ozemu_plan plan, int64_t k, int* beta_a, int* beta_b) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!beta_a || !beta_b) return fail(OZEMU_ERR_INVALID_ARG, "NULL output");
    if (plan->p.scaling == OZEMU_SCALE_BOUND)
        return fail(OZEMU_ERR_UNSUPPORTED, "bound mode decides bits per row and column");
    if (is_fp(plan->p)) {
        if (ozemu_status s = check_shape(plan->p, 1, 1, k)) return s;
    } else {
        // INT8: the window alone (k beyond the accumulation cap runs in the blocked call)
        if (k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
        if (ozemu_status s = check_window(plan->p, k)) return s;
    }
    kept_bits_of(plan->p, k, *beta_a, *beta_b);
    return ok();
}

ozemu_status ozemu_plan_k_max(ozemu_plan plan, int64_t* k_max) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!k_max) return fail(OZEMU_ERR_INVALID_ARG, "NULL output");
    int64_t km = plan->p.kappa_acc;
    if (plan->p.scaling == OZEMU_SCALE_F53) {
        // largest k with the window at 53 bits, by bisection on the exact test
        int64_t lo = 0, hi = km;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo + 1) / 2;
            if (ozemu::window_holds(plan->p, mid, 53, 53))
                lo = mid;
            else
                hi = mid - 1;
        }
        km = lo;
    } else if (plan->p.scaling == OZEMU_SCALE_BOUND && km > 524287) {
        km = 524287;
    }
    *k_max = km;
    return ok();
}

ozemu_status ozemu_plane_dims(ozemu_plan plan, int64_t m, int64_t n, int64_t k, int64_t* m_pad,
                              int64_t* n_pad, int64_t* k_pad) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    Dims d = dims_of(plan->p, m, n, k);
    if (m_pad) *m_pad = d.m_pad;
    if (n_pad) *n_pad = d.n_pad;
    if (k_pad) *k_pad = d.k_pad;
    return ok();
}

ozemu_status ozemu_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                  size_t* bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!bytes) return fail(OZEMU_ERR_INVALID_ARG, "bytes is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    *bytes = layout_of(plan->p, m, n, k).total;
    return ok();
}

ozemu_status ozemu_scale(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                         const double* A, int64_t lda, const double* B, int64_t ldb,
                         int32_t* shift_a, int32_t* shift_b, void* workspace, size_t ws_bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (ozemu_status s = check_shape(p, m, n, k)) return s;
    if (ozemu_status s = check_operands(m, n, k, A, lda, B, ldb)) return s;
    if ((m > 0 && !shift_a) || (n > 0 && !shift_b))
        return fail(OZEMU_ERR_INVALID_ARG, "shift output is NULL");
    const size_t need = scale_ws_need(p, m, n, k);
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_workspace_size");
    if (m == 0 && n == 0) return ok();
    return run_scale(p, (hipStream_t)stream, m, n, k, A, lda, B, ldb, shift_a, shift_b,
                     (char*)workspace);
}

ozemu_status ozemu_reduce(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                          const double* A, int64_t lda, const double* B, int64_t ldb,
                          const int32_t* shift_a, const int32_t* shift_b, int8_t* planes_a,
                          int8_t* planes_b) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (is_fp(p)) return fail(OZEMU_ERR_UNSUPPORTED, "phase calls take INT8 plans");
    if (ozemu_status s = check_shape(p, m, n, k)) return s;
    if (ozemu_status s = check_operands(m, n, k, A, lda, B, ldb)) return s;
    Dims d = dims_of(m, n, k);
    hipStream_t st = (hipStream_t)stream;
    if (d.m_pad > 0 && d.k_pad > 0) {
        if (!planes_a || !shift_a) return fail(OZEMU_ERR_INVALID_ARG, "planes_a or shift_a is NULL");
        if (ozemu_status s = hip_check(ozemu::launch_encode_a(st, p.mod, m, k, A, lda, shift_a,
                                                              d.m_pad, d.k_pad, planes_a,
                                                              big_encode(p, k)),
                                       "encode_a"))
            return s;
    }
    if (d.n_pad > 0 && d.k_pad > 0) {
        if (!planes_b || !shift_b) return fail(OZEMU_ERR_INVALID_ARG, "planes_b or shift_b is NULL");
        if (ozemu_status s = hip_check(ozemu::launch_encode_b(st, p.mod, k, n, B, ldb, shift_b,
                                                              d.n_pad, d.k_pad, planes_b,
                                                              big_encode(p, k)),
                                       "encode_b"))
            return s;
    }
    return ok();
}

ozemu_status ozemu_residue_gemm(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                const int8_t* planes_a, const int8_t* planes_b,
                                uint8_t* residues) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (is_fp(p)) return fail(OZEMU_ERR_UNSUPPORTED, "phase calls take INT8 plans");
    if (ozemu_status s = check_shape(p, m, n, k)) return s;
    Dims d = dims_of(m, n, k);
    if (d.m_pad == 0 || d.n_pad == 0) return ok();
    if (!residues) return fail(OZEMU_ERR_INVALID_ARG, "residues is NULL");
    if (d.k_pad > 0 && (!planes_a || !planes_b))
        return fail(OZEMU_ERR_INVALID_ARG, "planes are NULL");
    if (d.k_pad == 0) {
        return hip_check(ozemu::launch_fill_i32((hipStream_t)stream,
                                                (int64_t)p.n * d.m_pad * d.n_pad / 4, 0,
                                                reinterpret_cast<int32_t*>(residues)),
                         "zero residues");
    }
    return hip_check(ozemu::launch_residue_gemm((hipStream_t)stream, p.mod, d.m_pad, d.n_pad,
                                                d.k_pad, planes_a, planes_b, residues),
                     "residue_gemm");
}

ozemu_status ozemu_reconstruct(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                               const uint8_t* residues, const int32_t* shift_a,
                               const int32_t* shift_b, double* C, int64_t ldc) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (is_fp(p)) return fail(OZEMU_ERR_UNSUPPORTED, "phase calls take INT8 plans");
    if (ozemu_status s = check_shape(p, m, n, k)) return s;
    if (m == 0 || n == 0) return ok();
    if (!C || ldc < n) return fail(OZEMU_ERR_INVALID_ARG, "C is NULL or ldc < n");
    if (!residues || !shift_a || !shift_b)
        return fail(OZEMU_ERR_INVALID_ARG, "residues or shifts are NULL");
    Dims d = dims_of(m, n, k);
    return hip_check(ozemu::launch_reconstruct((hipStream_t)stream, p.crt, m, n, d.m_pad, d.n_pad,
                                               residues, shift_a, shift_b, C, ldc),
                     "reconstruct");
}

namespace {

// C = A B through the float channels of plan p (arguments validated).
ozemu_status dgemm_fp(const ozemu::Plan& p, hipStream_t st, int64_t m, int64_t n, int64_t k,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                      int64_t ldc, char* ws, const Layout& L) {
    using namespace ozemu;
    Dims d = dims_of(p, m, n, k);
    int32_t* sa = reinterpret_cast<int32_t*>(ws + L.shift_a);
    int32_t* sb = reinterpret_cast<int32_t*>(ws + L.shift_b);
    int8_t* pa = reinterpret_cast<int8_t*>(ws + L.planes_a);
    int8_t* pb = reinterpret_cast<int8_t*>(ws + L.planes_b);
    uint16_t* z = reinterpret_cast<uint16_t*>(ws + L.residues);
    uint8_t* tables = reinterpret_cast<uint8_t*>(ws + L.tables);
    if (ozemu_status s = run_scale(p, st, m, n, k, A, lda, B, ldb, sa, sb, ws)) return s;
    ozemu::Plan& mp = const_cast<ozemu::Plan&>(p);
    if (!mp.pinned_tables) {
        uint8_t* h = nullptr;
        if (ozemu_status s = hip_check(hipHostMalloc((void**)&h, p.tables.size(),
                                                     hipHostMallocDefault),
                                       "pinned channel tables"))
            return s;
        std::memcpy(h, p.tables.data(), p.tables.size());
        mp.pinned_tables = h;
    }
    if (ozemu_status s = hip_check(hipMemcpyAsync(tables, p.pinned_tables, p.tables.size(),
                                                  hipMemcpyHostToDevice, st),
                                   "channel tables"))
        return s;
    if (ozemu_status s = hip_check(
            launch_encode_fp(st, p.fp, tables, (int)p.tables.size(), m, n, k, A, lda, B, ldb, sa,
                             sb, d.m_pad, d.n_pad, d.k_pad, pa, pb),
            "encode_fp"))
        return s;
    const int64_t kb_pad = fp_row_bytes(p, d.k_pad);
    const int64_t slab_b = fp_row_bytes(p, p.k_slab);
    const int64_t tiles = (d.m_pad / kTileM) * (d.n_pad / kTileN);
    for (int64_t kb0 = 0; kb0 < kb_pad; kb0 += slab_b) {
        for (int r = 0; r < 3; ++r) {
            FpGemmArgs g{};
            g.first = (kb0 == 0 && r == 0) ? 1 : 0;
            g.scale = (float)(1 << (2 * p.fp.es));
            g.m_pad = d.m_pad;
            g.n_pad = d.n_pad;
            g.kb_pad = kb_pad;
            g.kb_begin = kb0;
            g.kb_len = std::min(slab_b, kb_pad - kb0);
            g.pa = pa;
            g.pb = pb;
            g.z = z;
            int cnt = 0;
            int64_t start = 0;
            for (int c = 0; c < p.fp.n; ++c) {
                if (p.fp.rank[c] <= r) continue;
                g.start[cnt] = start;
                g.plane[cnt] = p.fp.plane0[c] + r;
                g.chan[cnt] = c;
                g.m[cnt] = p.fp.m[c];
                g.mu[cnt] = p.fp.mu[c];
                g.lbar[cnt] = p.fp.lbar[c][r];
                start += tiles;
                ++cnt;
            }
            g.start[cnt] = start;
            g.count = cnt;
            if (cnt == 0) continue;
            if (ozemu_status s = hip_check(launch_fp_gemm(st, g, p.fp.fmt), "fp_gemm")) return s;
        }
    }
    return hip_check(launch_reconstruct16(st, p.crt, m, n, d.m_pad, d.n_pad, z, sa, sb, C, ldc),
                     "reconstruct");
}

}  // namespace

ozemu_status ozemu_dgemm(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                         const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                         int64_t ldc, void* workspace, size_t ws_bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (ozemu_status s = check_shape(p, m, n, k)) return s;
    if (m == 0 || n == 0) return ok();
    if (ozemu_status s = check_operands(m, n, k, A, lda, B, ldb)) return s;
    if (!C || ldc < n) return fail(OZEMU_ERR_INVALID_ARG, "C is NULL or ldc < n");
    hipStream_t st = (hipStream_t)stream;
    if (k == 0) return hip_check(ozemu::launch_zero_c(st, m, n, C, ldc), "zero C");
    Layout L = layout_of(p, m, n, k);
    if (!workspace || ws_bytes < L.total)
        return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_workspace_size");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(OZEMU_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    char* ws = static_cast<char*>(workspace);
    if (is_fp(p)) return dgemm_fp(p, st, m, n, k, A, lda, B, ldb, C, ldc, ws, L);
    int32_t* sa = reinterpret_cast<int32_t*>(ws + L.shift_a);
    int32_t* sb = reinterpret_cast<int32_t*>(ws + L.shift_b);
    int8_t* pa = reinterpret_cast<int8_t*>(ws + L.planes_a);
    int8_t* pb = reinterpret_cast<int8_t*>(ws + L.planes_b);
    uint8_t* z = reinterpret_cast<uint8_t*>(ws + L.residues);
    Dims d = dims_of(m, n, k);
    if (ozemu_status s = run_scale(p, st, m, n, k, A, lda, B, ldb, sa, sb, ws)) return s;
    if (ozemu_status s = hip_check(
            ozemu::launch_encode_a(st, p.mod, m, k, A, lda, sa, d.m_pad, d.k_pad, pa,
                                   big_encode(p, k)),
            "encode_a"))
        return s;
    if (ozemu_status s = hip_check(
            ozemu::launch_encode_b(st, p.mod, k, n, B, ldb, sb, d.n_pad, d.k_pad, pb,
                                   big_encode(p, k)),
            "encode_b"))
        return s;
    if (ozemu_status s = hip_check(
            ozemu::launch_residue_gemm(st, p.mod, d.m_pad, d.n_pad, d.k_pad, pa, pb, z),
            "residue_gemm"))
        return s;
    return hip_check(ozemu::launch_reconstruct(st, p.crt, m, n, d.m_pad, d.n_pad, z, sa, sb, C, ldc),
                     "reconstruct");
}

namespace {

// Workspace of the blocked call: shifts, the planes of one slab, the running
// residues and (with more than one slab) one slab's residues.
struct BlockedLayout {
    size_t shift_a, shift_b, planes_a, planes_b, z_run, z_slab, total;
};

BlockedLayout blocked_layout(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k,
                             int64_t k_slab) {
    const Dims d = dims_of(m, n, std::min(k, k_slab));
    BlockedLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t N = (size_t)p.n;
    L.shift_a = take(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
    L.shift_b = take(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    L.planes_a = take(N * (size_t)d.m_pad * (size_t)d.k_pad);
    L.planes_b = take(N * (size_t)d.n_pad * (size_t)d.k_pad);
    L.z_run = take(N * (size_t)d.m_pad * (size_t)d.n_pad);
    L.z_slab = k > k_slab ? take(N * (size_t)d.m_pad * (size_t)d.n_pad) : L.z_run;
    L.total = off;
    return L;
}

// The accumulation cap applies to a slab, the reconstruction cap to the
// whole inner dimension.
ozemu_status check_blocked(const ozemu::Plan& p, int64_t m, int64_t n, int64_t k,
                           int64_t k_slab) {
    if (is_fp(p))
        return fail(OZEMU_ERR_UNSUPPORTED,
                    "blocked call: INT8 plans only (float-channel plans take their slab "
                    "length at creation)");
    if (p.scaling == OZEMU_SCALE_BOUND)
        return fail(OZEMU_ERR_UNSUPPORTED, "blocked call: scaling modes F53 and W only");
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    if (m > (1ll << 31) || n > (1ll << 31)) return fail(OZEMU_ERR_INVALID_ARG, "dimension too large");
    if (k_slab < 1) return fail(OZEMU_ERR_INVALID_ARG, "k_slab must be positive");
    if (k_slab > p.kappa_acc)
        return fail(OZEMU_ERR_K_TOO_LARGE,
                    "k_slab = " + std::to_string(k_slab) + " exceeds the INT32 accumulation cap " +
                        std::to_string(p.kappa_acc) + " of this modulus set");
    return check_window(p, k);
}

}  // namespace

ozemu_status ozemu_blocked_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                          int64_t k_slab, size_t* bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!bytes) return fail(OZEMU_ERR_INVALID_ARG, "NULL output");
    if (ozemu_status s = check_blocked(plan->p, m, n, k, k_slab)) return s;
    *bytes = blocked_layout(plan->p, m, n, k, k_slab).total;
    return ok();
}

ozemu_status ozemu_dgemm_blocked(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                 int64_t k_slab, const double* A, int64_t lda, const double* B,
                                 int64_t ldb, double* C, int64_t ldc, void* workspace,
                                 size_t ws_bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (ozemu_status s = check_blocked(p, m, n, k, k_slab)) return s;
    if (m == 0 || n == 0) return ok();
    if (ozemu_status s = check_operands(m, n, k, A, lda, B, ldb)) return s;
    if (!C || ldc < n) return fail(OZEMU_ERR_INVALID_ARG, "C is NULL or ldc < n");
    hipStream_t st = (hipStream_t)stream;
    if (k == 0) return hip_check(ozemu::launch_zero_c(st, m, n, C, ldc), "zero C");
    const BlockedLayout L = blocked_layout(p, m, n, k, k_slab);
    if (!workspace || ws_bytes < L.total)
        return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_blocked_workspace_size");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(OZEMU_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    char* ws = static_cast<char*>(workspace);
    int32_t* sa = reinterpret_cast<int32_t*>(ws + L.shift_a);
    int32_t* sb = reinterpret_cast<int32_t*>(ws + L.shift_b);
    int8_t* pa = reinterpret_cast<int8_t*>(ws + L.planes_a);
    int8_t* pb = reinterpret_cast<int8_t*>(ws + L.planes_b);
    uint8_t* z_run = reinterpret_cast<uint8_t*>(ws + L.z_run);
    uint8_t* z_slab = reinterpret_cast<uint8_t*>(ws + L.z_slab);
    // shifts and kept bits from the whole inner dimension
    if (ozemu_status s = run_scale(p, st, m, n, k, A, lda, B, ldb, sa, sb, nullptr)) return s;
    const bool big = big_encode(p, k);
    Dims d{};
    for (int64_t h0 = 0; h0 < k; h0 += k_slab) {
        const int64_t kt = std::min(k_slab, k - h0);
        d = dims_of(m, n, kt);
        uint8_t* out = h0 == 0 ? z_run : z_slab;
        if (ozemu_status s = hip_check(
                ozemu::launch_encode_a(st, p.mod, m, kt, A + h0, lda, sa, d.m_pad, d.k_pad, pa, big),
                "encode_a"))
            return s;
        if (ozemu_status s = hip_check(
                ozemu::launch_encode_b(st, p.mod, kt, n, B + h0 * ldb, ldb, sb, d.n_pad, d.k_pad,
                                       pb, big),
                "encode_b"))
            return s;
        if (ozemu_status s = hip_check(
                ozemu::launch_residue_gemm(st, p.mod, d.m_pad, d.n_pad, d.k_pad, pa, pb, out),
                "residue_gemm"))
            return s;
        if (h0 > 0)
            if (ozemu_status s = hip_check(ozemu::launch_add_residues(st, p.mod, p.n,
                                                                      d.m_pad * d.n_pad, z_run,
                                                                      z_slab),
                                           "add_residues"))
                return s;
    }
    return hip_check(
        ozemu::launch_reconstruct(st, p.crt, m, n, d.m_pad, d.n_pad, z_run, sa, sb, C, ldc),
        "reconstruct");
}

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

int32_t cdiv32(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

}  // namespace

ozemu_status ozemu_group_create(ozemu_group* out, int count, const ozemu_plan* plans,
                                const int64_t* m, const int64_t* n, const int64_t* k,
                                const double* const* A, const int64_t* lda,
                                const double* const* B, const int64_t* ldb, double* const* C,
                                const int64_t* ldc) {
    using namespace ozemu;
    if (!out) return fail(OZEMU_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 0 || count > kMaxGroup)
        return fail(OZEMU_ERR_INVALID_ARG, "count must be in [0, 4096]");
    if (count > 0 && (!plans || !m || !n || !k || !A || !lda || !B || !ldb || !C || !ldc))
        return fail(OZEMU_ERR_INVALID_ARG, "NULL host array");
    // distinct plans, in first-use order
    std::vector<const ozemu::Plan*> uniq;
    std::vector<int32_t> pidx(count);
    for (int p = 0; p < count; ++p) {
        if (!plans[p]) return fail(OZEMU_ERR_INVALID_ARG, "plan of problem " + std::to_string(p) + " is NULL");
        const Plan* pl = &plans[p]->p;
        if (pl->format != OZEMU_INT8)
            return fail(OZEMU_ERR_UNSUPPORTED, "grouped products take INT8 plans");
        if (pl->scaling == OZEMU_SCALE_BOUND)
            return fail(OZEMU_ERR_UNSUPPORTED, "grouped products support F53 and WINDOW");
        int at = -1;
        for (size_t u = 0; u < uniq.size(); ++u)
            if (uniq[u] == pl) at = (int)u;
        if (at < 0) {
            at = (int)uniq.size();
            uniq.push_back(pl);
        }
        pidx[p] = at;
    }
    std::vector<GProblem> probs(count);
    for (int p = 0; p < count; ++p) {
        const Plan& pl = *uniq[pidx[p]];
        const std::string where = " (problem " + std::to_string(p) + ")";
        if (ozemu_status st = check_shape(pl, m[p], n[p], k[p])) {
            g_last_error += where;
            return st;
        }
        GProblem& P = probs[p];
        P.m = m[p];
        P.n = n[p];
        P.k = k[p];
        const bool active = m[p] > 0 && n[p] > 0;
        if (active) {
            if (ozemu_status st = check_operands(m[p], n[p], k[p], A[p], lda[p], B[p], ldb[p])) {
                g_last_error += where;
                return st;
            }
            if (!C[p] || ldc[p] < n[p])
                return fail(OZEMU_ERR_INVALID_ARG, "C is NULL or ldc < n" + where);
        }
        Dims d = dims_of(m[p], n[p], k[p]);
        P.m_pad = d.m_pad;
        P.n_pad = d.n_pad;
        P.k_pad = d.k_pad;
        P.A = A[p];
        P.B = B[p];
        P.C = C[p];
        P.lda = lda[p];
        P.ldb = ldb[p];
        P.ldc = ldc[p];
        P.plan = pidx[p];
        int ba = 0, bb = 0;
        if (k[p] > 0) kept_bits_of(pl, k[p], ba, bb);
        P.beta_a = ba;
        P.beta_b = bb;
        P.big = (ba > kSmallBits || bb > kSmallBits) ? 1 : 0;
    }
    ozemu_group g = new (std::nothrow) ozemu_group_s;
    if (!g) return fail(OZEMU_ERR_INVALID_ARG, "out of host memory");
    g->count = count;
    g->nplans = (int)uniq.size();
    // table layout
    size_t off = 0;
    g->off_probs = off;
    off = align256(off + sizeof(GProblem) * (size_t)count);
    g->off_mods = off;
    off = align256(off + sizeof(ModConsts) * uniq.size());
    g->off_crts = off;
    off = align256(off + sizeof(CrtConsts) * uniq.size());
    g->off_prefix = off;
    off = align256(off + sizeof(int32_t) * (size_t)kGKinds * (count + 1));
    g->off_order = off;
    off = align256(off + sizeof(int32_t) * (size_t)count);
    g->off_counter = off;
    off = align256(off + sizeof(int32_t) * kXcds);
    g->table_bytes = off;
    // per-problem workspace regions and work prefixes
    std::vector<int32_t> prefix((size_t)kGKinds * (count + 1), 0);
    std::vector<int32_t> order(count);
    for (int p = 0; p < count; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return probs[a].k_pad > probs[b].k_pad; });
    int64_t tot[kGKinds] = {};
    for (int p = 0; p < count; ++p) {
        GProblem& P = probs[p];
        const size_t N = (size_t)uniq[P.plan]->n;
        const bool active = P.m > 0 && P.n > 0;
        const bool work = active && P.k > 0;
        P.off_sa = (int64_t)off;
        off = align256(off + sizeof(int32_t) * (size_t)P.m_pad);
        P.off_sb = (int64_t)off;
        off = align256(off + sizeof(int32_t) * (size_t)P.n_pad);
        P.off_pa = (int64_t)off;
        if (work) off = align256(off + N * (size_t)P.m_pad * (size_t)P.k_pad);
        P.off_pb = (int64_t)off;
        if (work) off = align256(off + N * (size_t)P.n_pad * (size_t)P.k_pad);
        P.off_z = (int64_t)off;
        if (work) off = align256(off + N * (size_t)P.m_pad * (size_t)P.n_pad);
        int64_t blocks[kGKinds] = {};
        if (work) {
            blocks[kGColInit] = cdiv32(P.n, 256);
            blocks[kGRows] = P.m;
            blocks[kGCols] = (int64_t)cdiv32(P.n, 256) * cdiv32(P.k, 64);
            blocks[kGShifts] = cdiv32(P.m + P.n, 256);
            blocks[kGEncA] = cdiv32(P.m_pad * (P.k_pad / 16), 256);
            blocks[kGEncB] = (P.n_pad / 64) * (P.k_pad / 64);
        }
        if (active) blocks[kGCrt] = cdiv32(P.m * ((P.n + 3) / 4), 256);
        for (int kind = 0; kind < kGTiles; ++kind) {
            prefix[(size_t)kind * (count + 1) + p] = (int32_t)tot[kind];
            tot[kind] += blocks[kind];
        }
        if (work && P.big) g->big = true;
    }
    // per-XCD GEMM work lists over the problems in descending-K order
    for (int q = 0; q < count; ++q) {
        const GProblem& P = probs[order[q]];
        const bool work = P.m > 0 && P.n > 0 && P.k > 0;
        const int64_t T = (P.m_pad / kTileM) * (P.n_pad / kTileN);
        for (int x = 0; x < kXcds; ++x) {
            prefix[(size_t)(kGTiles + x) * (count + 1) + q] = (int32_t)tot[kGTiles + x];
            int first, cnt;
            xcd_moduli(uniq[P.plan]->n, x, q, first, cnt);
            if (work) tot[kGTiles + x] += (int64_t)cnt * T;
        }
    }
    for (int kind = 0; kind < kGKinds; ++kind) {
        if (tot[kind] > INT32_MAX) {
            delete g;
            return fail(OZEMU_ERR_INVALID_ARG, "group too large for one launch");
        }
        prefix[(size_t)kind * (count + 1) + count] = (int32_t)tot[kind];
        g->total[kind] = (int32_t)tot[kind];
    }
    g->ws_bytes = off;
    g->dmax = 2;
    for (const Plan* pl : uniq) g->dmax = std::max(g->dmax, pl->crt.d);
    g->tables.assign(g->table_bytes, 0);
    char* t = g->tables.data();
    if (count > 0) std::memcpy(t + g->off_probs, probs.data(), sizeof(GProblem) * count);
    for (size_t u = 0; u < uniq.size(); ++u) {
        std::memcpy(t + g->off_mods + u * sizeof(ModConsts), &uniq[u]->mod, sizeof(ModConsts));
        std::memcpy(t + g->off_crts + u * sizeof(CrtConsts), &uniq[u]->crt, sizeof(CrtConsts));
    }
    std::memcpy(t + g->off_prefix, prefix.data(), sizeof(int32_t) * prefix.size());
    if (count > 0) std::memcpy(t + g->off_order, order.data(), sizeof(int32_t) * count);
    *out = g;
    return ok();
}

ozemu_status ozemu_group_workspace_size(ozemu_group group, size_t* bytes) {
    if (!group) return fail(OZEMU_ERR_INVALID_ARG, "group is NULL");
    if (!bytes) return fail(OZEMU_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = group->ws_bytes;
    return ok();
}

ozemu_status ozemu_group_run(ozemu_group group, void* stream, void* workspace, size_t ws_bytes) {
    using namespace ozemu;
    if (!group) return fail(OZEMU_ERR_INVALID_ARG, "group is NULL");
    if (group->count == 0 || (group->total[kGCrt] == 0)) return ok();
    if (!workspace || ws_bytes < group->ws_bytes)
        return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_group_workspace_size");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(OZEMU_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    if (!group->pinned) {
        // pinned and never rewritten, so every run (and a captured graph's
        // replays) can copy from it asynchronously
        char* h = nullptr;
        if (ozemu_status s = hip_check(hipHostMalloc((void**)&h, group->table_bytes,
                                                     hipHostMallocDefault),
                                       "pinned group tables"))
            return s;
        std::memcpy(h, group->tables.data(), group->table_bytes);
        group->pinned = h;
    }
    if (ozemu_status s = hip_check(hipMemcpyAsync(ws, group->pinned, group->table_bytes,
                                                  hipMemcpyHostToDevice, st),
                                   "group tables"))
        return s;
    GroupArgs a;
    a.probs = reinterpret_cast<const GProblem*>(ws + group->off_probs);
    a.mods = reinterpret_cast<const ModConsts*>(ws + group->off_mods);
    a.crts = reinterpret_cast<const CrtConsts*>(ws + group->off_crts);
    a.prefix = reinterpret_cast<const int32_t*>(ws + group->off_prefix);
    a.order = reinterpret_cast<const int32_t*>(ws + group->off_order);
    a.ws = ws;
    a.counter = reinterpret_cast<int32_t*>(ws + group->off_counter);
    a.count = group->count;
    const int32_t* T = group->total;
    // one persistent GEMM workgroup per compute unit (its LDS allows one)
    int dev = 0, workers = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&workers, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        workers <= 0)
        workers = 256;
    ozemu_status s = hip_check(launch_group_init(st, a, T[kGColInit]), "group init");
    if (!s) s = hip_check(launch_group_scale(st, a, T[kGRows], T[kGCols], T[kGShifts]), "group scale");
    if (!s)
        s = hip_check(launch_group_encode(st, a, T[kGEncA], T[kGEncB], group->big), "group encode");
    if (!s) s = hip_check(launch_group_gemm(st, a, T + kGTiles, workers), "group gemm");
    if (!s) s = hip_check(launch_group_reconstruct(st, a, T[kGCrt], group->dmax), "group reconstruct");
    return s;
}

ozemu_status ozemu_group_destroy(ozemu_group group) {
    if (group) {
        if (group->pinned) (void)hipHostFree(group->pinned);
        delete group;
    }
    return ok();
}

ozemu_status ozemu_dgemm_fwd_cache(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                   const double* X, int64_t ldx, const double* W, int64_t ldw,
                                   double* Y, int64_t ldy, int32_t* shift_x, int32_t* shift_w,
                                   int8_t* planes_x, int8_t* planes_w, void* workspace,
                                   size_t ws_bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (ozemu_status s = check_cache_plan(p, m, n, k)) return s;
    if (m == 0 || n == 0) return ok();
    if (ozemu_status s = check_operands(m, n, k, X, ldx, W, ldw)) return s;
    if (!Y || ldy < n) return fail(OZEMU_ERR_INVALID_ARG, "Y is NULL or ldy < n");
    hipStream_t st = (hipStream_t)stream;
    if (k == 0) return hip_check(ozemu::launch_zero_c(st, m, n, Y, ldy), "zero Y");
    if (!shift_x || !shift_w || !planes_x || !planes_w)
        return fail(OZEMU_ERR_INVALID_ARG, "cache buffers are NULL");
    Layout L = layout_of(p, m, n, k);
    if (!workspace || ws_bytes < L.total)
        return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_workspace_size");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(OZEMU_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    uint8_t* z = reinterpret_cast<uint8_t*>(static_cast<char*>(workspace) + L.residues);
    Dims d = dims_of(m, n, k);
    const int64_t ks = cache_k(m, n, k);
    int bx, bw;
    kept_bits_of(p, ks, bx, bw);
    const bool big = bx > ozemu::kSmallBits || bw > ozemu::kSmallBits;
    using namespace ozemu;
    ozemu_status s = hip_check(launch_scale_rows(st, m, k, X, ldx, shift_x), "scale_rows");
    if (!s) s = hip_check(launch_scale_cols(st, k, n, W, ldw, shift_w), "scale_cols");
    if (!s) s = hip_check(launch_keys_to_shifts(st, m, shift_x, bx, nullptr), "shifts_x");
    if (!s) s = hip_check(launch_keys_to_shifts(st, n, shift_w, bw, nullptr), "shifts_w");
    if (!s)
        s = hip_check(launch_encode_a(st, p.mod, m, k, X, ldx, shift_x, d.m_pad, d.k_pad, planes_x,
                                      big),
                      "encode_x");
    if (!s)
        s = hip_check(launch_encode_b(st, p.mod, k, n, W, ldw, shift_w, d.n_pad, d.k_pad, planes_w,
                                      big),
                      "encode_w");
    if (!s)
        s = hip_check(launch_residue_gemm(st, p.mod, d.m_pad, d.n_pad, d.k_pad, planes_x, planes_w, z),
                      "residue_gemm");
    if (!s)
        s = hip_check(launch_reconstruct(st, p.crt, m, n, d.m_pad, d.n_pad, z, shift_x, shift_w, Y,
                                         ldy),
                      "reconstruct");
    return s;
}

ozemu_status ozemu_bwd_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                      size_t* bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    if (!bytes) return fail(OZEMU_ERR_INVALID_ARG, "bytes is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(OZEMU_ERR_INVALID_ARG, "negative dimension");
    *bytes = bwd_layout_of(plan->p, m, n, k).total;
    return ok();
}

ozemu_status ozemu_dgemm_bwd(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                             const double* dY, int64_t lddy, const int32_t* shift_x,
                             const int32_t* shift_w, const int8_t* planes_x,
                             const int8_t* planes_w, double* dX, int64_t lddx, double* dW,
                             int64_t lddw, void* workspace, size_t ws_bytes) {
    if (ozemu_status s = check_plan(plan)) return s;
    const ozemu::Plan& p = plan->p;
    if (ozemu_status s = check_cache_plan(p, m, n, k)) return s;
    const bool want_dx = dX && m > 0 && k > 0;
    const bool want_dw = dW && k > 0 && n > 0;
    if (want_dx && lddx < k) return fail(OZEMU_ERR_INVALID_ARG, "lddx < k");
    if (want_dw && lddw < n) return fail(OZEMU_ERR_INVALID_ARG, "lddw < n");
    hipStream_t st = (hipStream_t)stream;
    using namespace ozemu;
    // an empty inner dimension gives a zero gradient
    const bool dx_zero = want_dx && n == 0, dw_zero = want_dw && m == 0;
    const bool dx_run = want_dx && !dx_zero, dw_run = want_dw && !dw_zero;
    if (dx_run || dw_run) {
        if (!dY || lddy < n) return fail(OZEMU_ERR_INVALID_ARG, "dY is NULL or lddy < n");
        if ((dx_run && (!shift_w || !planes_w)) || (dw_run && (!shift_x || !planes_x)))
            return fail(OZEMU_ERR_INVALID_ARG, "cache buffers are NULL");
    }
    int bx, bw;
    kept_bits_of(p, cache_k(m, n, k), bx, bw);
    const int beta_dx = dx_run ? backward_bits(p, n, bw) : 1;
    const int beta_dw = dw_run ? backward_bits(p, m, bx) : 1;
    if (beta_dx < 1 || beta_dw < 1)
        return fail(OZEMU_ERR_K_TOO_LARGE, "no bits left for dY at this inner dimension");
    BwdLayout L = bwd_layout_of(p, m, n, k);
    if (dx_run || dw_run) {
        if (!workspace || ws_bytes < L.total)
            return fail(OZEMU_ERR_WORKSPACE, "workspace smaller than ozemu_bwd_workspace_size");
        if (reinterpret_cast<uintptr_t>(workspace) & 255)
            return fail(OZEMU_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    }
    if (dx_zero)
        if (ozemu_status s = hip_check(launch_zero_c(st, m, k, dX, lddx), "zero dX")) return s;
    if (dw_zero)
        if (ozemu_status s = hip_check(launch_zero_c(st, k, n, dW, lddw), "zero dW")) return s;
    if (!dx_run && !dw_run) return ok();
    char* ws = static_cast<char*>(workspace);
    int32_t* s2 = reinterpret_cast<int32_t*>(ws + L.shift_dx);
    int32_t* t3 = reinterpret_cast<int32_t*>(ws + L.shift_dw);
    int32_t* zeros = reinterpret_cast<int32_t*>(ws + L.zeros);
    int8_t* fresh = reinterpret_cast<int8_t*>(ws + L.planes_fresh);
    int8_t* tr = reinterpret_cast<int8_t*>(ws + L.planes_t);
    uint8_t* z = reinterpret_cast<uint8_t*>(ws + L.residues);
    const int64_t mp = round_up(m, kTileM), np = round_up(n, kTileN), kp = round_up(k, kTileM);
    const int64_t kp64 = round_up(k, kTileK);
    ozemu_status s = hip_check(launch_fill_i32(st, kp, 0, zeros), "zeros");
    if (!s && dx_run) {
        // dX = dY W^T: rows of dY folded by 2^-t, cached W planes transposed
        const bool big = beta_dx > kSmallBits;
        s = hip_check(launch_scale_rows(st, m, n, dY, lddy, s2, shift_w), "scale_rows dY");
        if (!s) s = hip_check(launch_keys_to_shifts(st, m, s2, beta_dx, nullptr), "shifts dY");
        if (!s)
            s = hip_check(launch_encode_a(st, p.mod, m, n, dY, lddy, s2, mp, np, fresh, big, shift_w),
                          "encode dY");
        if (!s)
            s = hip_check(launch_transpose_planes(st, p.n, np, kp64, kp, planes_w, tr),
                          "transpose W planes");
        if (!s) s = hip_check(launch_residue_gemm(st, p.mod, mp, kp, np, fresh, tr, z), "gemm dX");
        if (!s)
            s = hip_check(launch_reconstruct(st, p.crt, m, k, mp, kp, z, s2, zeros, dX, lddx),
                          "reconstruct dX");
    }
    if (!s && dw_run) {
        // dW = X^T dY: columns of dY folded by 2^-s, cached X planes transposed
        const bool big = beta_dw > kSmallBits;
        s = hip_check(launch_scale_cols(st, m, n, dY, lddy, t3, shift_x), "scale_cols dY");
        if (!s) s = hip_check(launch_keys_to_shifts(st, n, t3, beta_dw, nullptr), "shifts dY");
        if (!s)
            s = hip_check(launch_encode_b(st, p.mod, m, n, dY, lddy, t3, np, mp, fresh, big, shift_x),
                          "encode dY");
        if (!s)
            s = hip_check(launch_transpose_planes(st, p.n, mp, kp64, kp, planes_x, tr),
                          "transpose X planes");
        if (!s) s = hip_check(launch_residue_gemm(st, p.mod, kp, np, mp, tr, fresh, z), "gemm dW");
        if (!s)
            s = hip_check(launch_reconstruct(st, p.crt, k, n, kp, np, z, zeros, t3, dW, lddw),
                          "reconstruct dW");
    }
    return s;
}

}  // extern "C"
