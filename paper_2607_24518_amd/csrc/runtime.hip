// C ABI of the SymNMF library: contexts, S storage, solver state, the step
// sequence and the stop-rule driven solve loop (paper section "Convergence
// Criterion"; appendix "Detailed Algorithm Descriptions", family 3).
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace symnmf;

namespace {
// kernel ids of the profiling hook
enum { PK_STREAM = 0, PK_UPDATE = 1, PK_FINALIZE = 2, PK_PLAN = 3, PK_IMAGE = 4, PK_COUNT = 5 };

struct ProfScope {
    symnmf_ctx* ctx;
    int id;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(symnmf_ctx* c, int kid) : ctx(c), id(kid) {
        if (!ctx->profiling) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, ctx->stream);
    }
    ~ProfScope() {
        if (!a) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->events.push_back({id, {a, b}});
    }
};
}  // namespace

void* CallScratch::get(int64_t bytes, bool zero) {
    const int64_t b = ws_round(bytes);
    need += b;
    if (err != hipSuccess) return nullptr;
    symnmf_ctx* c = ctx_;
    char* p = nullptr;
    for (;;) {
        if (c->ws_top_block < c->ws.size()) {
            WsBlock& blk = c->ws[c->ws_top_block];
            if (c->ws_top_off + b <= blk.bytes) {
                p = blk.p + c->ws_top_off;
                c->ws_top_off += b;
                break;
            }
            ++c->ws_top_block;
            c->ws_top_off = 0;
            continue;
        }
        if (c->ws_attached) {
            err = hipErrorOutOfMemory;
            return nullptr;
        }
        const int64_t last = c->ws.empty() ? 0 : c->ws.back().bytes;
        const int64_t nb = std::max<int64_t>({b, last, (int64_t)64 << 20});
        void* q = nullptr;
        err = hipMalloc(&q, (size_t)nb);
        if (err != hipSuccess) return nullptr;
        c->ws.push_back({(char*)q, nb, true});
        ++c->ws_allocs;
    }
    if (zero) err = launch_zero(p, (size_t)b, c->stream);
    return err == hipSuccess ? p : nullptr;
}

symnmf_status scratch_fail(symnmf_ctx* ctx, const CallScratch& sc, const char* what) {
    if (ctx->ws_attached && sc.err == hipErrorOutOfMemory)
        return fail(ctx, SYMNMF_ENOMEM, "%s: the attached workspace is too small (the call needs %lld bytes)", what,
                    (long long)sc.need);
    return fail(ctx, sc.err == hipErrorOutOfMemory ? SYMNMF_ENOMEM : SYMNMF_EDEVICE, "%s: scratch: %s", what,
                hipGetErrorString(sc.err));
}

namespace {

constexpr int HCAP = 128;   // ring of per-step device statistics

int64_t elem_bytes(int32_t dtype) {
    switch (dtype) {
        case SYMNMF_S_FP32: return 4;
        case SYMNMF_S_BF16: return 2;
        case SYMNMF_S_FP8: return 1;
        case SYMNMF_S_FP64: return 8;
    }
    return 0;
}

struct Layout {
    int64_t ld, rows_pad, data_bytes, scale_off, diag_off, total;
};

Layout s_layout(int64_t rows, int64_t n, int32_t dtype, int64_t panel_rows) {
    Layout L;
    L.ld = round_up(n, PAD);
    L.rows_pad = round_up(rows, PAD);
    L.data_bytes = round_up(L.rows_pad * L.ld * elem_bytes(dtype), 256);
    L.scale_off = L.data_bytes;
    L.diag_off = L.data_bytes;
    L.total = L.data_bytes;
    if (dtype == SYMNMF_S_FP8) {
        const int64_t panels = (rows + panel_rows - 1) / panel_rows;
        L.diag_off = L.scale_off + round_up(panels * 4, 256);
        L.total = L.diag_off + round_up(L.rows_pad * 4, 256);
    }
    return L;
}

}  // namespace

struct symnmf_state {
    symnmf_ctx* ctx = nullptr;
    symnmf_S S{};
    symnmf_params p{};
    int64_t k = 0, n = 0, n_pad = 0, rows = 0, rows_pad = 0, row0 = 0, tiles = 0, chunks = 0;
    int h_f64 = 0;
    int64_t hsz = 4;
    int32_t P = 0;
    std::vector<void*> allocs;
    void* H[2] = {nullptr, nullptr};
    int cur = 0;
    void *G = nullptr, *M = nullptr, *Theta = nullptr, *Mu = nullptr, *Gout = nullptr, *part = nullptr;
    void* minv = nullptr;            // ADMM: (2 W^T W + rho I)^-1 (M holds the dual U)
    void *D = nullptr, *Gp = nullptr;   // Adan: average of gradient differences, previous gradient
    double *tile_gram = nullptr, *tile_tr = nullptr, *tile_kkt = nullptr;
    int32_t* tile_bad = nullptr;
    double* gram64[2] = {nullptr, nullptr};
    void* gram_eff = nullptr;
    double* gram_fixed = nullptr;
    double* ring = nullptr;
    int32_t *plan = nullptr, *tiles_I = nullptr, *tiles_J = nullptr, *counts = nullptr;
    void* sel = nullptr;
    void* img[2] = {nullptr, nullptr};   // chunk images of H and 2H (MFMA stream)
    int64_t img_bytes = 0, part_bytes = 0;   // capacities of img[*] and part
    bool mfma = false;
    bool tall = false;               // full steps run the 8-wave stream kernel
    int32_t P_tall = 0;
    double* scal = nullptr;          // device scalars (median, sums)
    int64_t t = 0;
    int ring_full[HCAP] = {};
    double ring_phi[HCAP] = {};
    // control state of the stop rule and the check-time rules
    double phi = 1.0;
    bool have_E0 = false, have_prev = false;
    double E0 = 0.0, E_prev = 0.0;
    int64_t stag_run = 0;
    bool pw_enabled = true, pw_cool = false;
    double pw_cool_target = 0.0, pw_E_reset = 0.0;
    int64_t pw_resets = 0;
    std::vector<symnmf_stats> checks;   // statistics of every check iteration evaluated so far
    std::chrono::steady_clock::time_point t0;
    symnmf_stats last{};
};

extern "C" {

int32_t symnmf_abi_version(void) { return 4; }

void symnmf_params_default(symnmf_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->method = SYMNMF_ADAGRAD;
    p->softplus = 0;
    p->eta = 0.02;
    p->eps = 1e-10;
    p->alpha = 0.99;
    p->mu = 0.5;
    p->c = 10.0;
    p->c_r = 10.0;
    p->eps_med = 1e-30;
    p->row_frac = 0.5;
    p->phi0 = 0.75;
    p->c_grow = 10.0;
    p->grow_checks = 3;
    p->snapshot_s = 10;
    p->block_rows = 1024;
    p->independent_blocks = 1;
    p->delta = 10;
    p->warmup = 50;
    p->max_iter = 1000;
    p->tau_E = 0.1;
    p->tau_g_inf = 1e-4;
    p->n_ref = 1e4;
    p->tau_stag = 1e-5;
    p->seed = 0;
    p->rho = 500.0;
    p->beta1 = 0.9;
    p->beta2 = 0.999;
    p->beta3 = 0.99;
}

symnmf_status symnmf_create(symnmf_ctx** out, int32_t device, void* hip_stream) {
    if (!out) return SYMNMF_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SYMNMF_EDEVICE;
    auto* ctx = new symnmf_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return SYMNMF_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->cus = prop.multiProcessorCount;
    // device address of the allocation-free entry points' scratch array (looked
    // up once per device; a failure is reported by those entry points)
    (void)noalloc_scratch_init(device);
    if (const char* e = std::getenv("SYMNMF_WGS_PER_CU")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 16) ctx->wgs_per_cu = v;
    }
    *out = ctx;
    return SYMNMF_OK;
}

void symnmf_destroy(symnmf_ctx* ctx) {
    if (!ctx) return;
    if (!ctx->ws.empty()) (void)hipStreamSynchronize(ctx->stream);
    for (auto& b : ctx->ws)
        if (b.owned) (void)hipFree(b.p);
    delete ctx;
}

symnmf_status symnmf_set_workspace(symnmf_ctx* ctx, void* dev, int64_t bytes) {
    if (!ctx) return SYMNMF_EINVAL;
    if ((dev == nullptr) != (bytes == 0) || bytes < 0)
        return fail(ctx, SYMNMF_EINVAL, "set_workspace: give a device buffer and its size, or NULL and 0");
    if (ctx->ws_top_block != 0 || ctx->ws_top_off != 0)
        return fail(ctx, SYMNMF_EINVAL, "set_workspace: a call is using the pool");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if (!ctx->ws.empty()) HIP_OK(ctx, hipStreamSynchronize(ctx->stream));   // kernels may still read the old pool
    for (auto& b : ctx->ws)
        if (b.owned) (void)hipFree(b.p);
    ctx->ws.clear();
    ctx->ws_attached = dev != nullptr;
    if (dev) ctx->ws.push_back({(char*)dev, bytes, false});
    return SYMNMF_OK;
}

symnmf_status symnmf_workspace_info(symnmf_ctx* ctx, int64_t* held, int64_t* allocs) {
    if (!ctx) return SYMNMF_EINVAL;
    int64_t h = 0;
    for (auto& b : ctx->ws) h += b.bytes;
    if (held) *held = h;
    if (allocs) *allocs = ctx->ws_allocs;
    return SYMNMF_OK;
}

const char* symnmf_last_error(const symnmf_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int64_t symnmf_S_offset(int64_t r, int64_t c, int64_t rows_pad, int64_t ld, int32_t dtype) {
    if (r < 0 || c < 0 || r >= rows_pad || c >= ld || elem_bytes(dtype) == 0 || rows_pad % 256 || ld % 256) return -1;
    if (dtype == SYMNMF_S_FP64) return r * ld + c;
    return tiled_offset(r, c, ld / KC, elems_per_16B(dtype));
}

int64_t symnmf_S_bytes(int64_t rows, int64_t n, int32_t dtype, int64_t fp8_panel_rows) {
    if (rows < 1 || n < 1 || elem_bytes(dtype) == 0) return -1;
    if (dtype == SYMNMF_S_FP8 && fp8_panel_rows < 1) return -1;
    return s_layout(rows, n, dtype, fp8_panel_rows).total;
}

static symnmf_status fill_descriptor(symnmf_ctx* ctx, void* buf, int64_t n, int64_t row0, int64_t rows, int32_t dtype,
                                     int32_t kind, int64_t panel_rows, const Layout& L, const double* sums,
                                     symnmf_S* out) {
    (void)ctx;
    std::memset(out, 0, sizeof(*out));
    out->data = buf;
    out->panel_scale = dtype == SYMNMF_S_FP8 ? (float*)((char*)buf + L.scale_off) : nullptr;
    out->diag = dtype == SYMNMF_S_FP8 ? (float*)((char*)buf + L.diag_off) : nullptr;
    out->n = n;
    out->row0 = row0;
    out->rows = rows;
    out->ld = L.ld;
    out->rows_pad = L.rows_pad;
    out->fp8_panel_rows = dtype == SYMNMF_S_FP8 ? panel_rows : 0;
    out->dtype = dtype;
    out->kind = kind;
    out->sum = sums[0];
    out->fro2 = sums[1];
    out->fro2_stored = sums[2];
    out->mean = sums[0] / ((double)rows * (double)n);
    return SYMNMF_OK;
}

static BuildOut build_out(void* buf, const Layout& L, int64_t n, int64_t row0, int64_t rows, int32_t dtype,
                          int64_t panel_rows) {
    BuildOut o;
    o.data = buf;
    o.scale = dtype == SYMNMF_S_FP8 ? (float*)((char*)buf + L.scale_off) : nullptr;
    o.diag = dtype == SYMNMF_S_FP8 ? (float*)((char*)buf + L.diag_off) : nullptr;
    o.rows = rows;
    o.rows_pad = L.rows_pad;
    o.ld = L.ld;
    o.n = n;
    o.row0 = row0;
    o.dtype = dtype;
    o.panel_rows = dtype == SYMNMF_S_FP8 ? panel_rows : 1;
    return o;
}

// Scratch of symnmf_build_S: Z (K x ldz), the FP64 sums, the FP8 panel maxima,
// the input-check flags, the TPDM rank workspace and the bf16 operand planes.
struct BuildWs {
    int64_t K, Kpad, ldz, z, sums, pmax, bad, work, planes;
};
static bool build_ws(const symnmf_sbuild_params* p, BuildWs& w) {
    if (!p || p->n < 1 || p->T < 2 || p->rows < 1 || elem_bytes(p->dtype) == 0) return false;
    if (p->dtype == SYMNMF_S_FP8 && p->fp8_panel_rows < 1) return false;
    w.K = p->T;
    if (p->kind == SYMNMF_TPDM) w.K = (int64_t)std::floor(p->q * (double)p->T);
    if (w.K < 1) return false;
    const Layout L = s_layout(p->rows, p->n, p->dtype, p->fp8_panel_rows);
    const int64_t zsz = p->dtype == SYMNMF_S_FP64 ? 8 : 4;
    w.ldz = round_up(std::max(p->n, p->row0 + L.rows_pad), 256);
    w.Kpad = round_up(w.K, 16);
    w.z = w.Kpad * w.ldz * zsz;
    BuildOut o;
    o.rows = p->rows;
    o.rows_pad = L.rows_pad;
    o.ld = L.ld;
    o.n = p->n;
    o.row0 = p->row0;
    o.dtype = p->dtype;
    o.panel_rows = p->dtype == SYMNMF_S_FP8 ? p->fp8_panel_rows : 1;
    w.sums = syrk_sum_words(o) * 8;
    w.pmax = (p->dtype == SYMNMF_S_FP8 ? (p->rows + p->fp8_panel_rows - 1) / p->fp8_panel_rows : 1) * 4;
    w.bad = 4;
    w.work = p->kind == SYMNMF_TPDM ? tpdm_work_bytes(p->T, p->n, p->raw_marginals) : 0;
    w.planes = (p->dtype == SYMNMF_S_BF16 || p->dtype == SYMNMF_S_FP8) ? syrk_split_ws_bytes(w.K, w.ldz) : 0;
    return true;
}

int64_t symnmf_build_S_workspace(const symnmf_sbuild_params* p) {
    BuildWs w;
    if (!build_ws(p, w)) return -1;
    return ws_sum({w.z, w.sums, w.pmax, w.bad}) + (w.work ? ws_round(w.work) : 0) +
           (w.planes ? ws_round(w.planes) : 0);
}

symnmf_status symnmf_build_S(symnmf_ctx* ctx, const float* X, const symnmf_sbuild_params* p, void* buf,
                             int64_t buf_bytes, symnmf_S* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!X || !p || !buf || !out) return fail(ctx, SYMNMF_EINVAL, "build_S: null argument");
    if (p->n < 1 || p->T < 2) return fail(ctx, SYMNMF_EINVAL, "build_S: need n >= 1 and T >= 2 (n=%lld T=%lld)",
                                          (long long)p->n, (long long)p->T);
    if (p->row0 < 0 || p->rows < 1 || p->row0 + p->rows > p->n)
        return fail(ctx, SYMNMF_EINVAL, "build_S: bad row range [%lld, %lld) of n=%lld", (long long)p->row0,
                    (long long)(p->row0 + p->rows), (long long)p->n);
    if (p->kind != SYMNMF_ABS_CORR && p->kind != SYMNMF_TPDM) return fail(ctx, SYMNMF_EINVAL, "build_S: bad kind");
    if (elem_bytes(p->dtype) == 0) return fail(ctx, SYMNMF_EINVAL, "build_S: bad dtype");
    if (p->dtype == SYMNMF_S_FP8 && p->fp8_panel_rows < 1)
        return fail(ctx, SYMNMF_EINVAL, "build_S: fp8_panel_rows must be >= 1");
    const int64_t n = p->n, T = p->T;
    int64_t K = T;
    if (p->kind == SYMNMF_TPDM) {
        if (!(p->q > 0.0 && p->q <= 1.0)) return fail(ctx, SYMNMF_EINVAL, "build_S: q must be in (0, 1]");
        K = (int64_t)std::floor(p->q * (double)T);
        if (K < 1) return fail(ctx, SYMNMF_EINVAL, "build_S: floor(q T) = 0 exceedances");
        if (p->raw_marginals != 0 && p->raw_marginals != 1)
            return fail(ctx, SYMNMF_EINVAL, "build_S: raw_marginals must be 0 or 1");
        if (!p->raw_marginals && T > 32768)
            return fail(ctx, SYMNMF_EUNSUPPORTED, "build_S: the rank transform supports T <= 32768");
    }
    const Layout L = s_layout(p->rows, n, p->dtype, p->fp8_panel_rows);
    if (buf_bytes < L.total)
        return fail(ctx, SYMNMF_ENOMEM, "build_S: buffer has %lld bytes, needs %lld", (long long)buf_bytes,
                    (long long)L.total);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int z_f64 = p->dtype == SYMNMF_S_FP64;
    BuildWs w;
    if (!build_ws(p, w)) return fail(ctx, SYMNMF_EINVAL, "build_S: bad parameters");
    const int64_t ldz = w.ldz, Kpad = w.Kpad;
    const BuildOut o = build_out(buf, L, n, p->row0, p->rows, p->dtype, p->fp8_panel_rows);
    CallScratch sc(ctx);
    void* Z = sc.get(w.z);
    void* sums = sc.get(w.sums);
    void* pmax = sc.get(w.pmax);
    void* bad = sc.get(w.bad);
    void* work = w.work ? sc.get(w.work) : nullptr;
    void* planes = w.planes ? sc.get(w.planes) : nullptr;
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "build_S");
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(launch_zero(buf, L.total, st));
    if (p->kind == SYMNMF_ABS_CORR) chk(launch_standardise(X, T, n, Z, z_f64, ldz, (int32_t*)bad, st));
    else {
        const float sign = p->raw_marginals ? (p->lower_tail ? -1.0f : 1.0f) : 0.0f;
        chk(launch_check_input(X, T * n, sign, (int32_t*)bad, st));
        chk(launch_tpdm_omega(X, T, n, p->lower_tail, p->raw_marginals, Z, z_f64, ldz, K, work, st));
    }
    int32_t hbad = 0;
    chk(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e == hipSuccess && (hbad & BAD_NONFINITE)) {
        return fail(ctx, SYMNMF_ENUMERIC, "build_S: X holds a non-finite value");
    }
    if (e == hipSuccess && (hbad & BAD_NEGATIVE)) {
        return fail(ctx, SYMNMF_EINVAL, "build_S: raw TPDM marginals need X >= 0 in the chosen tail orientation");
    }
    if (e == hipSuccess && hbad) {
        return fail(ctx, SYMNMF_EINVAL, "build_S: %d zero-variance column(s)", hbad);
    }
    // S-building GEMM: split-precision bf16 MFMA for BF16 / FP8 storage, FP32
    // MFMA for FP32, FP64 FMAs for FP64
    const bool split = p->dtype == SYMNMF_S_BF16 || p->dtype == SYMNMF_S_FP8;
    if (split && e == hipSuccess) {
        chk(launch_syrk_split_store((const float*)Z, K, ldz, o, (double*)sums, (uint32_t*)pmax, planes, st));
    } else {
        chk(launch_syrk_store(Z, z_f64, Kpad, ldz, o, (double*)sums, (uint32_t*)pmax, st));
    }
    double hs[3] = {0, 0, 0};
    chk(hipMemcpyAsync(hs, sums, 24, hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "build_S: %s", hipGetErrorString(e));
    if (!std::isfinite(hs[0]) || !std::isfinite(hs[1])) return fail(ctx, SYMNMF_ENUMERIC, "build_S: non-finite S");
    return fill_descriptor(ctx, buf, n, p->row0, p->rows, p->dtype, p->kind, p->fp8_panel_rows, L, hs, out);
}

symnmf_status symnmf_S_load(symnmf_ctx* ctx, const void* src, int32_t src_is_f64, int64_t n, int64_t row0,
                            int64_t rows, int32_t dtype, int64_t fp8_panel_rows, void* buf, int64_t buf_bytes,
                            symnmf_S* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!src || !buf || !out) return fail(ctx, SYMNMF_EINVAL, "S_load: null argument");
    if (n < 1 || row0 < 0 || rows < 1 || row0 + rows > n) return fail(ctx, SYMNMF_EINVAL, "S_load: bad shape");
    if (elem_bytes(dtype) == 0) return fail(ctx, SYMNMF_EINVAL, "S_load: bad dtype");
    if (dtype == SYMNMF_S_FP8 && fp8_panel_rows < 1) return fail(ctx, SYMNMF_EINVAL, "S_load: fp8_panel_rows >= 1");
    const Layout L = s_layout(rows, n, dtype, fp8_panel_rows);
    if (buf_bytes < L.total) return fail(ctx, SYMNMF_ENOMEM, "S_load: buffer too small");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const BuildOut o = build_out(buf, L, n, row0, rows, dtype, fp8_panel_rows);
    const int64_t panels = dtype == SYMNMF_S_FP8 ? (rows + fp8_panel_rows - 1) / fp8_panel_rows : 1;
    CallScratch sc(ctx);
    void* sums = sc.get((4 + 3 * L.rows_pad) * 8);
    void* pmax = sc.get(panels * 4);
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "S_load");
    hipError_t e = launch_zero(buf, L.total, st);
    if (e == hipSuccess) e = launch_store_dense(src, src_is_f64, o, (double*)sums, (uint32_t*)pmax, st);
    double hs[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hs, sums, 24, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "S_load: %s", hipGetErrorString(e));
    if (!std::isfinite(hs[0]) || !std::isfinite(hs[1])) return fail(ctx, SYMNMF_ENUMERIC, "S_load: non-finite S");
    return fill_descriptor(ctx, buf, n, row0, rows, dtype, SYMNMF_ABS_CORR, fp8_panel_rows, L, hs, out);
}

symnmf_status symnmf_init_H(symnmf_ctx* ctx, const symnmf_S* S, int64_t k, uint64_t seed, float* H) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !H || k < 1 || k > KMAX) return fail(ctx, SYMNMF_EINVAL, "init_H: bad argument (k=%lld)", (long long)k);
    if (!(S->mean >= 0.0) || !std::isfinite(S->mean)) return fail(ctx, SYMNMF_EINVAL, "init_H: S has no valid mean");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    const float scale = (float)std::sqrt(S->mean / (double)k);
    HIP_OK(ctx, launch_init_H(H, S->n, k, seed, scale, ctx->stream));
    return SYMNMF_OK;
}

void symnmf_state_destroy(symnmf_state* st) {
    if (!st) return;
    for (void* p : st->allocs)
        if (p) (void)hipFree(p);
    delete st;
}

static symnmf_status state_alloc(symnmf_state* st, void** out, int64_t bytes) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 8);
    if (e != hipSuccess)
        return fail(st->ctx, SYMNMF_ENOMEM, "state: hipMalloc(%lld) failed: %s", (long long)bytes, hipGetErrorString(e));
    st->allocs.push_back(p);
    e = launch_zero(p, bytes > 0 ? bytes : 8, st->ctx->stream);
    if (e != hipSuccess) return fail(st->ctx, SYMNMF_EDEVICE, "state: memset failed: %s", hipGetErrorString(e));
    *out = p;
    return SYMNMF_OK;
}

static double tau_g_of(const symnmf_state* st) {
    const double n = (double)st->n;
    return st->p.tau_g_inf * std::max(1.0, st->p.n_ref / n);
}

symnmf_status symnmf_state_create(symnmf_ctx* ctx, const symnmf_S* S, int64_t k, const symnmf_params* p,
                                  const void* H0, int32_t h0_is_f64, symnmf_state** out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !p || !H0 || !out) return fail(ctx, SYMNMF_EINVAL, "state_create: null argument");
    *out = nullptr;
    if (k < 1 || k > KMAX) return fail(ctx, SYMNMF_EINVAL, "state_create: k=%lld outside [1, %d]", (long long)k, KMAX);
    if (k > S->n) return fail(ctx, SYMNMF_EINVAL, "state_create: k > n");
    const int h_f64 = S->dtype == SYMNMF_S_FP64;
    if (h_f64 && !h0_is_f64) return fail(ctx, SYMNMF_EINVAL, "state_create: FP64 S needs an FP64 H0");
    if (h_f64 && k > 32) return fail(ctx, SYMNMF_EUNSUPPORTED, "state_create: FP64 state supports k <= 32");
    if (p->method < SYMNMF_ADAGRAD || p->method > SYMNMF_MU)
        return fail(ctx, SYMNMF_EINVAL, "state_create: bad method");
    if (p->method == SYMNMF_MU && p->softplus)
        return fail(ctx, SYMNMF_EINVAL, "state_create: MU keeps H >= 0 by construction and has no softplus form");
    if ((p->method == SYMNMF_ADAM || p->method == SYMNMF_NADAM || p->method == SYMNMF_ADAN) &&
        !(p->beta1 >= 0.0 && p->beta1 < 1.0 && p->beta2 >= 0.0 && p->beta2 < 1.0 && p->beta3 >= 0.0 &&
          p->beta3 < 1.0))
        return fail(ctx, SYMNMF_EINVAL, "state_create: beta1, beta2, beta3 must lie in [0, 1)");
    if (p->method == SYMNMF_ADMM && (!(p->rho > 0.0) || p->softplus))
        return fail(ctx, SYMNMF_EINVAL, "state_create: ADMM needs rho > 0 and the projected form");
    if (!(p->eta > 0.0) || !(p->eps >= 0.0) || p->delta < 1 || p->max_iter < 0)
        return fail(ctx, SYMNMF_EINVAL, "state_create: bad eta/eps/delta/max_iter");
    const bool svrg = p->method == SYMNMF_ROW_SVRG || p->method == SYMNMF_BLOCK_SVRG;
    if (svrg) {
        if (S->rows != S->n || S->row0 != 0)
            return fail(ctx, SYMNMF_EUNSUPPORTED, "state_create: SVRG methods need the full matrix, not a panel");
        if (p->block_rows < 256 || p->block_rows % 256)
            return fail(ctx, SYMNMF_EINVAL, "state_create: block_rows must be a positive multiple of 256");
        if (p->snapshot_s < 1 || p->delta % p->snapshot_s)
            return fail(ctx, SYMNMF_EINVAL, "state_create: delta must be a multiple of snapshot_s");
        if ((S->n + p->block_rows - 1) / p->block_rows > 4096)
            return fail(ctx, SYMNMF_EUNSUPPORTED, "state_create: more than 4096 row blocks");
        if (p->method == SYMNMF_ROW_SVRG && !(p->row_frac > 0.0 && p->row_frac <= 1.0))
            return fail(ctx, SYMNMF_EINVAL, "state_create: row_frac in (0, 1]");
        if (p->method == SYMNMF_BLOCK_SVRG && !(p->phi0 > 0.0 && p->phi0 <= 1.0))
            return fail(ctx, SYMNMF_EINVAL, "state_create: phi0 in (0, 1]");
    }
    HIP_OK(ctx, hipSetDevice(ctx->device));
    auto* st = new symnmf_state();
    st->ctx = ctx;
    st->S = *S;
    st->p = *p;
    st->k = k;
    st->n = S->n;
    st->n_pad = round_up(S->n, PAD);
    st->rows = S->rows;
    st->rows_pad = S->rows_pad;
    st->row0 = S->row0;
    st->tiles = S->rows_pad / TR;
    st->chunks = S->ld / KC;
    st->h_f64 = h_f64;
    st->hsz = h_f64 ? 8 : 4;
    st->P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : stream_wgs_per_cu(S->dtype, k));
    st->phi = p->method == SYMNMF_BLOCK_SVRG ? p->phi0 : 1.0;
    const int64_t hbytes = std::max(st->n_pad, st->row0 + st->rows_pad) * k * st->hsz;
    const int64_t pbytes = st->rows_pad * k * st->hsz;
    symnmf_status s;
#define ALLOC(ptr, bytes)                                              \
    do {                                                               \
        void* tmp_ = nullptr;                                          \
        if ((s = state_alloc(st, &tmp_, (bytes))) != SYMNMF_OK) {      \
            symnmf_state_destroy(st);                                  \
            return s;                                                  \
        }                                                              \
        ptr = (decltype(ptr))tmp_;                                     \
    } while (0)
    ALLOC(st->H[0], hbytes);
    ALLOC(st->H[1], hbytes);
    ALLOC(st->G, pbytes);
    if (p->method == SYMNMF_RMSPROP || p->method == SYMNMF_ADMM || p->method == SYMNMF_ADAM ||
        p->method == SYMNMF_NADAM || p->method == SYMNMF_ADAN)
        ALLOC(st->M, pbytes);
    if (p->method == SYMNMF_ADAN) {
        ALLOC(st->D, pbytes);
        ALLOC(st->Gp, pbytes);
    }
    if (p->method == SYMNMF_ADMM) ALLOC(st->minv, k * k * st->hsz);
    if (p->softplus) ALLOC(st->Theta, pbytes);
    if (svrg) ALLOC(st->Mu, pbytes);
    ALLOC(st->Gout, pbytes);
    st->mfma = stream_uses_mfma(S->dtype, h_f64, h_f64, k) != 0;
    if (st->mfma) {
        const int64_t iw = h_image_words(S->dtype, k, st->chunks);
        ALLOC(st->img[0], iw * 4);
        if (p->method == SYMNMF_BLOCK_SVRG) ALLOC(st->img[1], iw * 4);
        st->img_bytes = iw * 4;
    }
    st->tall = stream_tall_supported(S->dtype, h_f64, k) != 0 && std::getenv("SYMNMF_NO_TALL") == nullptr;
    st->P_tall = st->tall ? tall_wgs(ctx->cus, st->tiles) : ctx->cus;
    const int64_t part_tiles = std::max<int64_t>((int64_t)st->P + st->tiles,
                                                 st->tall ? 2 * ((int64_t)st->P_tall + tall_pairs(st->tiles)) : 0);
    ALLOC(st->part, part_tiles * TR * k * st->hsz);
    st->part_bytes = part_tiles * TR * k * st->hsz;
    ALLOC(st->tile_gram, st->tiles * SUBT * k * k * 8);
    ALLOC(st->tile_tr, st->tiles * SUBT * 8);
    ALLOC(st->tile_kkt, st->tiles * SUBT * 8);
    ALLOC(st->tile_bad, st->tiles * SUBT * 4);
    ALLOC(st->gram64[0], k * k * 8);
    ALLOC(st->gram64[1], k * k * 8);
    ALLOC(st->gram_eff, 3 * k * k * st->hsz);
    ALLOC(st->ring, HCAP * 4 * 8);
    ALLOC(st->scal, 16 * 8);
    ALLOC(st->sel, select_tmp_bytes());
    if (svrg) {
        ALLOC(st->plan, plan_words(st->tiles, st->chunks) * 4);
        ALLOC(st->tiles_I, st->tiles * 4);
        ALLOC(st->tiles_J, st->tiles * 4);
        ALLOC(st->counts, 16);
    }
    const bool panel = st->rows < st->n;
    if (panel) ALLOC(st->gram_fixed, k * k * 8);
#undef ALLOC
    hipStream_t sm = ctx->stream;
    hipError_t e = launch_copy_h(H0, h0_is_f64, st->H[0], h_f64, st->n * k, sm);
    // a step writes the panel rows of the other buffer only: the fixed rows
    // outside the panel must be present in both iterate buffers
    if (e == hipSuccess && panel) e = launch_copy_h(H0, h0_is_f64, st->H[1], h_f64, st->n * k, sm);
    if (e == hipSuccess && p->softplus) {
        // Theta and softplus(Theta) for the panel rows
        void* Hp = (char*)st->H[0] + st->row0 * k * st->hsz;
        e = launch_softplus_init(Hp, st->Theta, h_f64, st->rows * k, sm);
    }
    if (e == hipSuccess && panel)
        e = launch_gram_rows(st->H[0], h_f64, st->n, st->row0, st->row0 + st->rows, k, st->gram_fixed, sm);
    if (e == hipSuccess) e = launch_tile_gram(st->H[0], h_f64, st->row0, st->rows, st->tiles, k, st->tile_gram, sm);
    if (e == hipSuccess)
        e = launch_finalize(st->tiles * SUBT, k, st->tile_gram, st->tile_tr, st->tile_kkt, st->tile_bad, st->gram_fixed,
                            nullptr, st->gram64[0], st->gram_eff, h_f64, st->scal, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) {
        symnmf_state_destroy(st);
        return fail(ctx, SYMNMF_EDEVICE, "state_create: %s", hipGetErrorString(e));
    }
    st->t0 = std::chrono::steady_clock::now();
    *out = st;
    return SYMNMF_OK;
}

static symnmf_status do_step(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st) {
    const symnmf_params& p = st->p;
    hipStream_t sm = ctx->stream;
    const int64_t t = st->t;
    int kind = 0;   // 0 full, 1 row, 2 block
    if (p.method == SYMNMF_ROW_SVRG) kind = (t % p.snapshot_s == 0) ? 0 : 1;
    if (p.method == SYMNMF_BLOCK_SVRG) kind = (st->phi >= 1.0 || t % p.snapshot_s == 0) ? 0 : 2;
    PlanView pv = plan_view(st->plan, kind == 0, (int32_t)st->tiles, (int32_t)st->chunks, st->P);
    if (kind == 0 && st->tall) {
        pv.tall = 1;
        pv.P = st->P_tall;
    }
    if (kind != 0) {
        PlanRequest r;
        r.mode = kind;
        r.n_tiles = (int32_t)st->tiles;
        r.n_chunks = (int32_t)st->chunks;
        r.tiles_per_block = (int32_t)(p.block_rows / TR);
        r.chunks_per_block = (int32_t)(p.block_rows / KC);
        r.n_blocks = (int32_t)((st->n + p.block_rows - 1) / p.block_rows);
        const double frac = kind == 1 ? p.row_frac : std::sqrt(st->phi);
        r.m = (int32_t)std::min<int64_t>(r.n_blocks, (int64_t)std::ceil(frac * (double)r.n_blocks));
        r.independent = p.independent_blocks;
        r.seed = p.seed;
        r.t = t;
        ProfScope ps(ctx, PK_PLAN);
        HIP_OK(ctx, launch_plan(r, st->plan, st->tiles_I, st->tiles_J, st->counts, sm));
        if (kind == 2)
            HIP_OK(ctx, launch_gram_select(st->k, st->tile_gram, st->tiles_I, st->tiles_J, st->counts, st->gram_eff,
                                           st->h_f64, sm));
    }
    const void* Hc = st->H[st->cur];
    void* Hn = st->H[1 - st->cur];
    if (st->mfma) {
        ProfScope pi(ctx, PK_IMAGE);
        HIP_OK(ctx, launch_h_image((const float*)Hc, S->dtype, st->k, st->chunks, 1.0f, (uint32_t*)st->img[0], sm));
        if (kind == 2)
            HIP_OK(ctx, launch_h_image((const float*)Hc, S->dtype, st->k, st->chunks, 2.0f, (uint32_t*)st->img[1], sm));
    }
    {
        ProfScope ps(ctx, PK_STREAM);
        HIP_OK(ctx, launch_stream(S->data, S->dtype, S->ld, Hc, st->h_f64, st->k, st->part, st->h_f64, pv, sm,
                                  st->img[0], kind == 2 ? st->img[1] : st->img[0]));
    }
    UpdateArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rows = st->rows;
    a.rows_pad = st->rows_pad;
    a.n = st->n;
    a.k = st->k;
    a.row0 = st->row0;
    // Piecewise AdaGrad and the SVRG variants step with the AdaGrad rule
    a.method = (p.method == SYMNMF_PIECEWISE_ADAGRAD || p.method == SYMNMF_ROW_SVRG ||
                p.method == SYMNMF_BLOCK_SVRG) ? SYMNMF_ADAGRAD : p.method;
    a.beta1 = p.beta1;
    a.beta2 = p.beta2;
    a.beta3 = p.beta3;
    {   // bias corrections of step count t + 1
        const double tb = (double)(t + 1);
        a.bc1 = 1.0 - std::pow(p.beta1, tb);
        a.bc2 = 1.0 - std::pow(p.beta2, tb);
        a.bc3 = 1.0 - std::pow(p.beta3, tb);
    }
    a.first = t == 0 ? 1 : 0;
    a.D = st->D;
    a.Gp = st->Gp;
    a.softplus = p.softplus;
    a.eta = p.eta;
    a.eps = p.eps;
    a.alpha = p.alpha;
    a.mu = p.mu;
    a.H = Hc;
    a.Hn = Hn;
    a.G = st->G;
    a.M = st->M;
    a.Theta = st->Theta;
    a.Mu = st->Mu;
    a.Gout = st->Gout;
    a.part = st->part;
    a.gram_eff = st->gram_eff;
    a.cgrad = kind == 2 ? 2.0 : 4.0;
    a.store_mu = (kind == 0 && st->Mu) ? 1 : 0;
    a.fp8 = S->dtype == SYMNMF_S_FP8;
    a.block_step = kind == 2 ? 1 : 0;
    a.panel_scale = S->panel_scale;
    a.diag = S->diag;
    a.panel_rows = S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1;
    a.tile_gram = st->tile_gram;
    a.tile_tr = st->tile_tr;
    a.tile_kkt = st->tile_kkt;
    a.tile_bad = st->tile_bad;
    {
        ProfScope ps(ctx, PK_UPDATE);
        if (p.method == SYMNMF_ADMM) {
            a.rho = p.rho;
            a.minv = st->minv;
            HIP_OK(ctx, launch_admm(a, st->gram64[st->cur], st->h_f64, pv, sm));
        } else {
            HIP_OK(ctx, launch_update(a, st->h_f64, pv, sm));
        }
    }
    const int slot = (int)(t % HCAP);
    ProfScope psf(ctx, PK_FINALIZE);
    HIP_OK(ctx, launch_finalize(st->tiles * SUBT, st->k, st->tile_gram, st->tile_tr, st->tile_kkt, st->tile_bad,
                                st->gram_fixed, st->gram64[st->cur], st->gram64[1 - st->cur], st->gram_eff, st->h_f64,
                                st->ring + slot * 4, sm));
    st->ring_full[slot] = kind == 0;
    st->ring_phi[slot] = st->phi;
    st->cur = 1 - st->cur;
    st->t = t + 1;
    return SYMNMF_OK;
}

// statistics of step t (must be one of the last HCAP steps); synchronises
static symnmf_status read_stats(symnmf_state* st, int64_t t, symnmf_stats* out) {
    symnmf_ctx* ctx = st->ctx;
    const int slot = (int)(t % HCAP);
    double d[4];
    HIP_OK(ctx, hipMemcpyAsync(d, st->ring + slot * 4, 32, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof(*out));
    out->t = t;
    out->full = st->ring_full[slot];
    out->phi = st->ring_phi[slot];
    const double nan = std::nan("");
    if (out->full) {
        out->f = st->S.fro2_stored - 2.0 * d[0] + d[3];
        out->E = out->f / st->S.fro2_stored;
        out->kkt = std::sqrt(d[1]) / ((double)st->rows * (double)st->k);
    } else {
        out->f = nan;
        out->E = nan;
        out->kkt = nan;
    }
    out->stag = nan;
    out->nonfinite = (int32_t)d[2];
    out->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - st->t0).count();
    return SYMNMF_OK;
}

symnmf_status symnmf_step(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st, symnmf_stats* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !st || st->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "step: bad state or context");
    if (S->data != st->S.data || S->n != st->n || S->rows != st->rows)
        return fail(ctx, SYMNMF_EINVAL, "step: S does not match the state");
    symnmf_status s = do_step(ctx, S, st);
    if (s != SYMNMF_OK) return s;
    if (out) {
        s = read_stats(st, st->t - 1, out);
        if (s != SYMNMF_OK) return s;
        st->last = *out;
        if (out->nonfinite) return fail(ctx, SYMNMF_ENUMERIC, "step %lld: %d non-finite gradient entries",
                                        (long long)out->t, out->nonfinite);
    }
    return SYMNMF_OK;
}

symnmf_status symnmf_state_stats(symnmf_ctx* ctx, symnmf_state* st, symnmf_stats* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!st || !out || st->t < 1) return fail(ctx, SYMNMF_EINVAL, "state_stats: no step taken");
    return read_stats(st, st->t - 1, out);
}

symnmf_status symnmf_state_set_phi(symnmf_state* st, double phi) {
    if (!st || !(phi > 0.0 && phi <= 1.0)) return SYMNMF_EINVAL;
    st->phi = phi;
    return SYMNMF_OK;
}

symnmf_status symnmf_state_read(symnmf_ctx* ctx, symnmf_state* st, int32_t which, void* dst) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!st || !dst) return fail(ctx, SYMNMF_EINVAL, "state_read: null argument");
    const void* src = nullptr;
    int64_t count = st->rows * st->k;
    int64_t off = 0;
    switch (which) {
        case 0: src = st->H[st->cur]; count = st->n * st->k; break;
        case 1: src = st->H[1 - st->cur]; count = st->n * st->k; break;
        case 2: src = st->G; break;
        case 3: src = st->M; break;
        case 4: src = st->Theta; break;
        case 5: src = st->Mu; break;
        case 6: src = st->Gout; break;
        case 7: src = st->D; break;
        case 8: src = st->Gp; break;
        default: return fail(ctx, SYMNMF_EINVAL, "state_read: bad buffer id %d", which);
    }
    (void)off;
    if (!src) return fail(ctx, SYMNMF_EINVAL, "state_read: buffer %d not used by this method", which);
    HIP_OK(ctx, hipMemcpyAsync(dst, src, count * st->hsz, hipMemcpyDeviceToDevice, ctx->stream));
    return SYMNMF_OK;
}

}  // extern "C"

// Scratch of objective_terms: FP64 copy of H, the S.H partials, the per-slice
// FP64 partials, the Gram, three effective Grams, the statistics; on the MFMA
// path also the FP32 H and its chunk images.
struct ObjWs {
    int64_t hd, part, tg, ttr, tk, tb, g, gi, sc, hf, img;
    bool mfma;
};
static ObjWs objective_ws(const symnmf_ctx* ctx, const symnmf_S* S, int64_t k, int32_t h_is_f64) {
    ObjWs w;
    const int64_t tiles = S->rows_pad / TR, chunks = S->ld / KC;
    const int32_t P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : 2);
    const int64_t hrows = std::max(round_up(S->n, PAD), S->row0 + S->rows_pad);
    w.hd = hrows * k * 8;
    w.part = ((int64_t)P + tiles) * TR * k * 8;
    w.tg = tiles * k * k * 8;          // one partial per 256-row tile (objective_tiles_kernel)
    w.ttr = tiles * 8;
    w.tk = tiles * 8;
    w.tb = tiles * 4;
    w.g = k * k * 8;
    w.gi = 3 * k * k * 8;
    w.sc = 4 * 8;
    w.mfma = !h_is_f64 && stream_acc64_supported(S->dtype, k);
    w.hf = w.mfma ? hrows * k * 4 : 0;
    w.img = w.mfma ? h_image_words(S->dtype, k, chunks) * 4 : 0;
    return w;
}

symnmf_status objective_terms(symnmf_ctx* ctx, const symnmf_S* S, const void* H, int32_t h_is_f64, int64_t k,
                              double* tr, double* gram_norm2) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !H || k < 1 || k > KMAX) return fail(ctx, SYMNMF_EINVAL, "objective: bad argument");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t tiles = S->rows_pad / TR, chunks = S->ld / KC;
    const int32_t P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : 2);
    const ObjWs w = objective_ws(ctx, S, k, h_is_f64);
    CallScratch scr(ctx);
    void* Hd = scr.get(w.hd);
    void* part = scr.get(w.part, false);
    void* tg = scr.get(w.tg, false);
    void* ttr = scr.get(w.ttr, false);
    void* tk = scr.get(w.tk, false);
    void* tb = scr.get(w.tb, false);
    void* g = scr.get(w.g, false);
    void* gi = scr.get(w.gi, false);
    void* sc = scr.get(w.sc, false);
    void* Hf = w.mfma ? scr.get(w.hf) : nullptr;
    void* img = w.mfma ? scr.get(w.img, false) : nullptr;
    if (scr.err != hipSuccess) return scratch_fail(ctx, scr, "objective");
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(launch_copy_h(H, h_is_f64, Hd, 1, S->n * k, sm));
    PlanView pv = plan_view(nullptr, 1, (int32_t)tiles, (int32_t)chunks, P);
    if (w.mfma) {
        // MFMA products, FP32 within each 256-column chunk, FP64 across chunks
        chk(launch_copy_h(H, 0, Hf, 0, S->n * k, sm));
        chk(launch_h_image((const float*)Hf, S->dtype, k, chunks, 1.0f, (uint32_t*)img, sm));
        chk(launch_stream_acc64(S->data, S->dtype, k, img, (double*)part, pv, sm));
    } else {
        chk(launch_stream(S->data, S->dtype, S->ld, Hd, 1, k, part, 1, pv, sm));
    }
    UpdateArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rows = S->rows;
    a.rows_pad = S->rows_pad;
    a.n = S->n;
    a.k = k;
    a.row0 = S->row0;
    a.H = Hd;
    a.part = part;
    a.fp8 = S->dtype == SYMNMF_S_FP8;
    a.panel_scale = S->panel_scale;
    a.diag = S->diag;
    a.panel_rows = S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1;
    a.tile_gram = (double*)tg;
    a.tile_tr = (double*)ttr;
    a.tile_kkt = (double*)tk;
    a.tile_bad = (int32_t*)tb;
    chk(launch_objective_tiles(a, pv, sm));
    chk(launch_finalize(tiles, k, (double*)tg, (double*)ttr, (double*)tk, (int32_t*)tb, nullptr, nullptr,
                        (double*)g, gi, 1, (double*)sc, sm));
    std::vector<double> gram(k * k);
    double d[4] = {0, 0, 0, 0};
    if (e == hipSuccess) chk(hipMemcpyAsync(gram.data(), g, k * k * 8, hipMemcpyDeviceToHost, sm));
    if (e == hipSuccess) chk(hipMemcpyAsync(d, sc, 32, hipMemcpyDeviceToHost, sm));
    if (e == hipSuccess) chk(hipStreamSynchronize(sm));
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "objective: %s", hipGetErrorString(e));
    double gn = 0.0;
    for (double v : gram) gn += v * v;
    *tr = d[0];
    *gram_norm2 = gn;
    return SYMNMF_OK;
}

extern "C" {

int64_t symnmf_objective_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t k, int32_t h_is_f64) {
    if (!ctx || !S || k < 1 || k > KMAX) return -1;
    const ObjWs w = objective_ws(ctx, S, k, h_is_f64);
    return ws_sum({w.hd, w.part, w.tg, w.ttr, w.tk, w.tb, w.g, w.gi, w.sc}) +
           (w.mfma ? ws_sum({w.hf, w.img}) : 0);
}

symnmf_status symnmf_objective(symnmf_ctx* ctx, const symnmf_S* S, const void* H, int32_t h_is_f64, int64_t k,
                               double* f, double* E) {
    double tr = 0.0, gn = 0.0;
    const symnmf_status s = objective_terms(ctx, S, H, h_is_f64, k, &tr, &gn);
    if (s != SYMNMF_OK) return s;
    const double fv = S->fro2_stored - 2.0 * tr + gn;
    if (f) *f = fv;
    if (E) *E = fv / S->fro2_stored;
    if (!std::isfinite(fv)) return fail(ctx, SYMNMF_ENUMERIC, "objective: non-finite value");
    return SYMNMF_OK;
}

int64_t symnmf_median_workspace(void) { return ws_sum({select_tmp_bytes(), 8}); }

symnmf_status symnmf_median_sq(symnmf_ctx* ctx, const float* g, int64_t m, float* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!g || m < 1 || !out) return fail(ctx, SYMNMF_EINVAL, "median_sq: bad argument");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    CallScratch sc(ctx);
    void* tmp = sc.get(select_tmp_bytes(), false);
    void* res = sc.get(8, false);
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "median_sq");
    double v = 0.0;
    hipError_t e = launch_select(g, 0, 1, m, (m - 1) / 2, tmp, (double*)res, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&v, res, 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "median_sq: %s", hipGetErrorString(e));
    *out = (float)v;
    return SYMNMF_OK;
}

symnmf_status symnmf_median_sq_noalloc(symnmf_ctx* ctx, const float* g, int64_t m, double* out_dev) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!g || !out_dev || m < 1) return fail(ctx, SYMNMF_EINVAL, "median_sq_noalloc: bad argument");
    if (m > SELECT_MAX_M)
        return fail(ctx, SYMNMF_EINVAL, "median_sq_noalloc: m = %lld exceeds the maximum of %lld values",
                    (long long)m, (long long)SELECT_MAX_M);
    hipError_t e = hipSuccess;
    void* scr = noalloc_scratch(ctx->device, &e);
    if (!scr)
        return fail(ctx, SYMNMF_EDEVICE, "median_sq_noalloc: no scratch address on device %d: %s", ctx->device,
                    hipGetErrorString(e));
    HIP_OK(ctx, hipSetDevice(ctx->device));
    HIP_OK(ctx, launch_select(g, 0, 1, m, (m - 1) / 2, scr, out_dev, ctx->stream));
    return SYMNMF_OK;
}

// G <- max(c g^2, c median(g^2)) with g the last step's gradient.
static symnmf_status piecewise_reset_impl(symnmf_state* st, double c, double* median_out) {
    symnmf_ctx* ctx = st->ctx;
    const int64_t m = st->rows * st->k;
    HIP_OK(ctx, launch_select(st->Gout, st->h_f64, 1, m, (m - 1) / 2, st->sel, st->scal, ctx->stream));
    HIP_OK(ctx, launch_piecewise_apply(st->G, st->Gout, st->h_f64, m, c, st->scal, ctx->stream));
    if (median_out) {
        HIP_OK(ctx, hipMemcpyAsync(median_out, st->scal, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return SYMNMF_OK;
}

symnmf_status symnmf_piecewise_reset(symnmf_ctx* ctx, symnmf_state* st, double c, float* median_out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!st || st->t < 1) return fail(ctx, SYMNMF_EINVAL, "piecewise_reset: no step taken");
    double med = 0.0;
    symnmf_status s = piecewise_reset_impl(st, c, &med);
    if (s == SYMNMF_OK && median_out) *median_out = (float)med;
    return s;
}

static symnmf_status device_sum(symnmf_state* st, const void* x, double* out) {
    symnmf_ctx* ctx = st->ctx;
    HIP_OK(ctx, launch_sum(x, st->h_f64, st->rows * st->k, st->scal + 1, ctx->stream));
    HIP_OK(ctx, hipMemcpyAsync(out, st->scal + 1, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    return SYMNMF_OK;
}

static symnmf_status median_of_last_gradient(symnmf_state* st, double* med) {
    symnmf_ctx* ctx = st->ctx;
    const int64_t m = st->rows * st->k;
    HIP_OK(ctx, launch_select(st->Gout, st->h_f64, 1, m, (m - 1) / 2, st->sel, st->scal, ctx->stream));
    HIP_OK(ctx, hipMemcpyAsync(med, st->scal, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    return SYMNMF_OK;
}

// Stop rule and check-time rules for the statistics of a check iteration.
static symnmf_status check_iteration(symnmf_state* st, symnmf_stats* sv) {
    const symnmf_params& p = st->p;
    if (!st->have_E0) {
        st->E0 = sv->E;
        st->have_E0 = true;
    }
    bool stag_ok = false;
    if (st->have_prev) {
        sv->stag = (st->E_prev - sv->E) / st->E0;
        stag_ok = sv->t >= p.warmup && sv->stag < p.tau_stag;
    }
    const double tg = tau_g_of(st);
    sv->converged = (sv->E < p.tau_E && sv->kkt < tg && stag_ok) ? 1 : 0;
    if (!sv->converged) {
        if (p.method == SYMNMF_PIECEWISE_ADAGRAD) {
            bool eligible = true;
            if (st->pw_cool) {
                double gsum = 0.0;
                symnmf_status s = device_sum(st, st->G, &gsum);
                if (s != SYMNMF_OK) return s;
                if (gsum < st->pw_cool_target) eligible = false;
            }
            if (eligible && stag_ok && st->pw_enabled) {
                double med = 0.0;
                symnmf_status s = median_of_last_gradient(st, &med);
                if (s != SYMNMF_OK) return s;
                if (sv->kkt > p.c_r * tg && med > p.eps_med) {
                    if (st->pw_resets > 0 && !(sv->E < st->pw_E_reset * (1.0 - 10.0 * p.tau_stag))) {
                        st->pw_enabled = false;
                    } else {
                        s = piecewise_reset_impl(st, p.c, nullptr);
                        if (s != SYMNMF_OK) return s;
                        double gsum = 0.0;
                        s = device_sum(st, st->G, &gsum);
                        if (s != SYMNMF_OK) return s;
                        st->pw_cool = true;
                        st->pw_cool_target = 2.0 * gsum;
                        st->pw_E_reset = sv->E;
                        st->pw_resets += 1;
                        sv->reset_fired = 1;
                    }
                }
            }
        }
        if (p.method == SYMNMF_BLOCK_SVRG && st->phi < 1.0) {
            st->stag_run = stag_ok ? st->stag_run + 1 : 0;
            if (st->stag_run >= p.grow_checks && sv->kkt > p.c_grow * tg) {
                st->phi = std::min(2.0 * st->phi, 1.0);
                st->stag_run = 0;
            }
        }
    }
    st->E_prev = sv->E;
    st->have_prev = true;
    st->checks.push_back(*sv);
    return SYMNMF_OK;
}

symnmf_status symnmf_solve_to_tol(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st, double f_target,
                                  double rel_tol, symnmf_stats* final_stats, void* H_out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !st || st->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "solve_to_tol: bad state or context");
    if (S->data != st->S.data) return fail(ctx, SYMNMF_EINVAL, "solve_to_tol: S does not match the state");
    const symnmf_params& p = st->p;
    symnmf_stats sv{};
    bool have = false;
    while (st->t < p.max_iter) {
        symnmf_status s = do_step(ctx, S, st);
        if (s != SYMNMF_OK) return s;
        const int64_t t = st->t - 1;
        const bool check = t % p.delta == 0;
        const bool full = st->ring_full[t % HCAP] != 0;
        if (!(check || (f_target > 0.0 && full))) continue;
        s = read_stats(st, t, &sv);
        if (s != SYMNMF_OK) return s;
        have = true;
        if (sv.nonfinite) {
            st->last = sv;
            if (final_stats) *final_stats = sv;
            return fail(ctx, SYMNMF_ENUMERIC, "solve: non-finite gradient at t=%lld", (long long)t);
        }
        if (f_target > 0.0 && full && (sv.f - f_target) / f_target <= rel_tol) {
            // H_t is the buffer the step read: now the "previous" iterate
            if (H_out)
                HIP_OK(ctx, hipMemcpyAsync(H_out, st->H[1 - st->cur], st->n * st->k * st->hsz, hipMemcpyDeviceToDevice,
                                           ctx->stream));
            HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
            st->last = sv;
            if (final_stats) *final_stats = sv;
            return SYMNMF_OK;
        }
        if (check) {
            if (!full) return fail(ctx, SYMNMF_EINVAL, "solve: check iteration %lld was not a full step", (long long)t);
            s = check_iteration(st, &sv);
            if (s != SYMNMF_OK) return s;
            if (sv.converged) {
                if (H_out)
                    HIP_OK(ctx, hipMemcpyAsync(H_out, st->H[1 - st->cur], st->n * st->k * st->hsz,
                                               hipMemcpyDeviceToDevice, ctx->stream));
                HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
                st->last = sv;
                if (final_stats) *final_stats = sv;
                return SYMNMF_OK;
            }
        }
    }
    if (H_out)
        HIP_OK(ctx, hipMemcpyAsync(H_out, st->H[st->cur], st->n * st->k * st->hsz, hipMemcpyDeviceToDevice,
                                   ctx->stream));
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    if (!have && st->t > 0) read_stats(st, st->t - 1, &sv);
    st->last = sv;
    if (final_stats) *final_stats = sv;
    return SYMNMF_ENOTCONV;
}

// Point the state at another storage of the same matrix (same n, rows, row0
// and tiling; FP64 storage only for an FP64 state): the stream launch shape,
// the image and partial buffers follow the new storage type; the optimiser
// state, the iterate and t are kept; the stagnation reference restarts, since
// E changes with the stored matrix.
static symnmf_status rebind_state(symnmf_state* st, const symnmf_S* S) {
    symnmf_ctx* ctx = st->ctx;
    if (S->n != st->n || S->rows != st->rows || S->row0 != st->row0 || S->rows_pad != st->rows_pad ||
        S->ld / KC != st->chunks)
        return fail(ctx, SYMNMF_EINVAL, "state_rebind: S has another shape than the state's");
    if ((S->dtype == SYMNMF_S_FP64) != (st->h_f64 != 0))
        return fail(ctx, SYMNMF_EINVAL, "state_rebind: FP64 storage goes with an FP64 state only");
    const int64_t k = st->k;
    const bool mfma = stream_uses_mfma(S->dtype, st->h_f64, st->h_f64, k) != 0;
    const int32_t P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : stream_wgs_per_cu(S->dtype, k));
    const bool tall = stream_tall_supported(S->dtype, st->h_f64, k) != 0 && std::getenv("SYMNMF_NO_TALL") == nullptr;
    const int32_t P_tall = tall ? tall_wgs(ctx->cus, st->tiles) : ctx->cus;
    const int64_t part_tiles = std::max<int64_t>((int64_t)P + st->tiles,
                                                 tall ? 2 * ((int64_t)P_tall + tall_pairs(st->tiles)) : 0);
    const int64_t part_bytes = part_tiles * TR * k * st->hsz;
    const int64_t img_bytes = mfma ? h_image_words(S->dtype, k, st->chunks) * 4 : 0;
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));   // no kernel of the old shape still reads the buffers
    auto grow = [&](void*& buf, int64_t need) -> symnmf_status {
        void* fresh = nullptr;
        symnmf_status s = state_alloc(st, &fresh, need);
        if (s != SYMNMF_OK) return s;
        for (auto& q : st->allocs)
            if (q == buf) {
                (void)hipFree(q);
                q = nullptr;
            }
        buf = fresh;
        return SYMNMF_OK;
    };
    symnmf_status s = SYMNMF_OK;
    if (part_bytes > st->part_bytes) {
        if ((s = grow(st->part, part_bytes)) != SYMNMF_OK) return s;
        st->part_bytes = part_bytes;
    }
    if (img_bytes > st->img_bytes) {
        if ((s = grow(st->img[0], img_bytes)) != SYMNMF_OK) return s;
        if (st->p.method == SYMNMF_BLOCK_SVRG && (s = grow(st->img[1], img_bytes)) != SYMNMF_OK) return s;
        st->img_bytes = img_bytes;
    }
    st->S = *S;
    st->mfma = mfma;
    st->P = P;
    st->tall = tall;
    st->P_tall = P_tall;
    st->have_prev = false;
    st->stag_run = 0;
    return SYMNMF_OK;
}

symnmf_status symnmf_state_checks(symnmf_ctx* ctx, symnmf_state* st, symnmf_stats* out, int64_t cap,
                                  int64_t* count) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!st || !count || (cap > 0 && !out) || cap < 0) return fail(ctx, SYMNMF_EINVAL, "state_checks: bad argument");
    const int64_t m = (int64_t)st->checks.size();
    *count = m;
    for (int64_t i = 0; i < std::min(m, cap); ++i) out[i] = st->checks[i];
    return SYMNMF_OK;
}

symnmf_status symnmf_state_control(symnmf_ctx* ctx, symnmf_state* st, symnmf_control* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!st || !out) return fail(ctx, SYMNMF_EINVAL, "state_control: null argument");
    std::memset(out, 0, sizeof(*out));
    out->t = st->t;
    out->phi = st->phi;
    out->stag_run = st->stag_run;
    out->pw_resets = st->pw_resets;
    out->pw_enabled = st->pw_enabled ? 1 : 0;
    out->pw_cooling = st->pw_cool ? 1 : 0;
    out->pw_cool_target = st->pw_cool_target;
    out->pw_E_reset = st->pw_E_reset;
    return SYMNMF_OK;
}

symnmf_status symnmf_state_rebind(symnmf_ctx* ctx, symnmf_state* st, const symnmf_S* S) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !st || st->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "state_rebind: bad state or context");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    return rebind_state(st, S);
}

// The loop of symnmf_solve_trace; with S_hi it starts on S and moves the
// state to S_hi at the first check whose stagnation measure falls below
// tau_switch (the precision ladder).
static symnmf_status trace_impl(symnmf_ctx* ctx, const symnmf_S* S, const symnmf_S* S_hi, double tau_switch,
                                int64_t* switched_at, symnmf_state* st, int64_t steps, int64_t save_every,
                                void* H_save, double* ms_out, int64_t* certified_at) {
    const symnmf_params& p = st->p;
    const int64_t nsave = steps / save_every;
    const int64_t hbytes = st->n * st->k * st->hsz;
    std::vector<hipEvent_t> ev(nsave + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    auto cleanup = [&]() {
        for (auto& x : ev)
            if (x) (void)hipEventDestroy(x);
    };
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, SYMNMF_EDEVICE, "solve_trace: %s", hipGetErrorString(e));
    }
    if (certified_at) *certified_at = -1;
    if (switched_at) *switched_at = -1;
    const symnmf_S* cur = S;
    (void)hipEventRecord(ev[0], ctx->stream);
    symnmf_status s = SYMNMF_OK;
    for (int64_t i = 0; i < nsave * save_every && s == SYMNMF_OK; ++i) {
        s = do_step(ctx, cur, st);
        if (s != SYMNMF_OK) break;
        const int64_t t = st->t - 1;
        if ((i + 1) % save_every == 0) {
            const int64_t j = (i + 1) / save_every - 1;
            if (hipMemcpyAsync((char*)H_save + j * hbytes, st->H[st->cur], hbytes, hipMemcpyDeviceToDevice,
                               ctx->stream) != hipSuccess) {
                s = fail(ctx, SYMNMF_EDEVICE, "solve_trace: copy failed");
                break;
            }
            (void)hipEventRecord(ev[j + 1], ctx->stream);
        }
        if (t % p.delta != 0) continue;
        symnmf_stats sv{};
        s = read_stats(st, t, &sv);
        if (s != SYMNMF_OK) break;
        if (sv.nonfinite) {
            s = fail(ctx, SYMNMF_ENUMERIC, "solve_trace: non-finite gradient at t=%lld", (long long)t);
            break;
        }
        if (!sv.full) {
            s = fail(ctx, SYMNMF_EINVAL, "solve_trace: check iteration %lld was not a full step", (long long)t);
            break;
        }
        s = check_iteration(st, &sv);
        st->last = sv;
        const bool low = S_hi && cur != S_hi;
        // certification counts on the final storage only
        if (s == SYMNMF_OK && !low && sv.converged && certified_at && *certified_at < 0) *certified_at = t;
        if (s == SYMNMF_OK && low && sv.t >= p.warmup && !std::isnan(sv.stag) && sv.stag < tau_switch) {
            s = rebind_state(st, S_hi);
            cur = S_hi;
            if (switched_at) *switched_at = t;
        }
    }
    if (s == SYMNMF_OK) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) s = fail(ctx, SYMNMF_EDEVICE, "solve_trace: sync");
        for (int64_t j = 0; j < nsave && s == SYMNMF_OK; ++j) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[0], ev[j + 1]) != hipSuccess) s = fail(ctx, SYMNMF_EDEVICE, "solve_trace: event");
            ms_out[j] = ms;
        }
    }
    cleanup();
    return s;
}

symnmf_status symnmf_solve_trace(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st, int64_t steps,
                                 int64_t save_every, void* H_save, int64_t slots, double* ms_out,
                                 int64_t* certified_at) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !st || st->ctx != ctx || !H_save || !ms_out || save_every < 1 || steps < 0 || slots < steps / save_every)
        return fail(ctx, SYMNMF_EINVAL, "solve_trace: bad argument");
    if (S->data != st->S.data) return fail(ctx, SYMNMF_EINVAL, "solve_trace: S does not match the state");
    return trace_impl(ctx, S, nullptr, 0.0, nullptr, st, steps, save_every, H_save, ms_out, certified_at);
}

symnmf_status symnmf_solve_trace_ladder(symnmf_ctx* ctx, const symnmf_S* S_lo, const symnmf_S* S_hi,
                                        symnmf_state* st, int64_t steps, int64_t save_every, void* H_save,
                                        int64_t slots, double* ms_out, double tau_switch, int64_t* certified_at,
                                        int64_t* switched_at) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S_lo || !S_hi || !st || st->ctx != ctx || !H_save || !ms_out || save_every < 1 || steps < 0 ||
        slots < steps / save_every || !(tau_switch >= 0.0))
        return fail(ctx, SYMNMF_EINVAL, "solve_trace_ladder: bad argument");
    if (S_lo->data != st->S.data) return fail(ctx, SYMNMF_EINVAL, "solve_trace_ladder: S_lo does not match the state");
    if (S_hi->n != S_lo->n || S_hi->rows != S_lo->rows || S_hi->row0 != S_lo->row0 || S_hi->ld != S_lo->ld ||
        S_hi->rows_pad != S_lo->rows_pad || (S_hi->dtype == SYMNMF_S_FP64) != (S_lo->dtype == SYMNMF_S_FP64))
        return fail(ctx, SYMNMF_EINVAL, "solve_trace_ladder: S_lo and S_hi differ in shape or state precision");
    return trace_impl(ctx, S_lo, S_hi, tau_switch, switched_at, st, steps, save_every, H_save, ms_out, certified_at);
}

symnmf_status symnmf_probe_read(symnmf_ctx* ctx, const void* src, void* sink, int64_t sink_words, int64_t bytes) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!src || !sink || bytes < 16 || bytes % 16 || sink_words < 4)
        return fail(ctx, SYMNMF_EINVAL, "probe_read: bad argument");
    HIP_OK(ctx, launch_read_probe(src, bytes, (uint32_t*)sink, sink_words, ctx->stream));
    return SYMNMF_OK;
}

symnmf_status symnmf_probe_copy(symnmf_ctx* ctx, const void* src, void* dst, int64_t bytes) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!src || !dst || bytes < 16 || bytes % 16) return fail(ctx, SYMNMF_EINVAL, "probe_copy: bad arguments");
    HIP_OK(ctx, launch_copy_probe(src, dst, bytes, ctx->stream));
    return SYMNMF_OK;
}

symnmf_status symnmf_profile(symnmf_ctx* ctx, int32_t enable, double* ms_out, int64_t* launches_out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (ms_out || launches_out) {
        HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < PK_COUNT; ++i) {
            if (ms_out) ms_out[i] = 0.0;
            if (launches_out) launches_out[i] = 0;
        }
        for (auto& e : ctx->events) {
            float ms = 0.f;
            HIP_OK(ctx, hipEventElapsedTime(&ms, e.second.first, e.second.second));
            if (ms_out) ms_out[e.first] += ms;
            if (launches_out) launches_out[e.first] += 1;
        }
    }
    for (auto& e : ctx->events) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    ctx->events.clear();
    ctx->profiling = enable != 0;
    return SYMNMF_OK;
}

void symnmf_sample_blocks(uint64_t seed, int64_t t, int32_t stream, int64_t nblocks, int64_t m, int32_t* out) {
    if (!out || nblocks < 1 || m < 1 || m > nblocks) return;
    std::vector<int32_t> perm(nblocks);
    std::vector<uint8_t> flags(nblocks);
    sample_block_flags(seed, t, stream, (int)nblocks, (int)m, perm.data(), flags.data());
    int64_t j = 0;
    for (int64_t b = 0; b < nblocks; ++b)
        if (flags[b]) out[j++] = (int32_t)b;
}

// Library self-check of device instructions whose behaviour the kernels rely
// on: returns the number of FP8 codes the hardware FP8->BF16 conversion
// decodes differently from the E4M3 definition (0 expected), or -1 on error.
int32_t symnmf_selfcheck_fp8(symnmf_ctx* ctx) {
    if (!ctx) return -1;
    CallScratch sc(ctx);
    void* bad = sc.get(4);
    if (sc.err != hipSuccess) return -1;
    int32_t h = -1;
    hipError_t e = launch_fp8_decode_check((int32_t*)bad, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? h : -1;
}

}  // extern "C"
