// C ABI of the learned warm start: sketch, canonical coordinates, the MLP
// (forward, Gram-loss training step with AdamW) and the composed warm start.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace symnmf;

struct symnmf_mlp {
    symnmf_ctx* ctx = nullptr;
    int64_t w = 0, h = 0, k = 0, np = 0, nw = 0;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *V = nullptr;
    uint16_t* Wb = nullptr;   // BF16 copies of W1, W2, W3
    bool bf16_stale = true;
    int32_t residual = 0;     // output max(C + z, 0) over the input's first k columns instead of softplus(z)
    int64_t t = 0;            // AdamW steps taken
    float* split_ws = nullptr;
    int64_t split_floats = 0;
    double* small = nullptr;  // AtA, AtB, BtB (3 k^2) then x^T y slab work
    int64_t small_doubles = 0;
    // activations, grown on demand
    int64_t cap_fwd = 0, cap_train = 0;
    float *a1 = nullptr, *a2 = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr, *out = nullptr, *dA = nullptr, *d3 = nullptr, *da2 = nullptr;

    int64_t off_W1() const { return 0; }
    int64_t off_W2() const { return h * w; }
    int64_t off_W3() const { return h * w + h * h; }
    int64_t off_b1() const { return nw; }
    int64_t off_b2() const { return nw + h; }
    int64_t off_b3() const { return nw + 2 * h; }
};

namespace {

void free_all(std::initializer_list<void*> ps) {
    for (void* p : ps)
        if (p) (void)hipFree(p);
}

symnmf_status ensure_fwd(symnmf_mlp* m, int64_t rows) {
    if (m->cap_fwd >= rows) return SYMNMF_OK;
    free_all({m->a1, m->a2});
    m->a1 = m->a2 = nullptr;
    m->cap_fwd = 0;
    HIP_OK(m->ctx, hipMalloc((void**)&m->a1, rows * m->h * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->a2, rows * m->h * 4));
    m->cap_fwd = rows;
    return SYMNMF_OK;
}

symnmf_status ensure_train(symnmf_mlp* m, int64_t rows) {
    if (m->cap_train >= rows) return SYMNMF_OK;
    free_all({m->z1, m->z2, m->z3, m->out, m->dA, m->d3, m->da2});
    m->z1 = m->z2 = m->z3 = m->out = m->dA = m->d3 = m->da2 = nullptr;
    m->cap_train = 0;
    HIP_OK(m->ctx, hipMalloc((void**)&m->z1, rows * m->h * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->z2, rows * m->h * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->da2, rows * m->h * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->z3, rows * m->k * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->out, rows * m->k * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->dA, rows * m->k * 4));
    HIP_OK(m->ctx, hipMalloc((void**)&m->d3, rows * m->k * 4));
    m->cap_train = rows;
    const int64_t need = 3 * m->k * m->k + xty_work_doubles(rows, m->k, m->k);
    if (m->small_doubles < need) {
        if (m->small) (void)hipFree(m->small);
        m->small = nullptr;
        m->small_doubles = 0;
        HIP_OK(m->ctx, hipMalloc((void**)&m->small, need * 8));
        m->small_doubles = need;
    }
    return SYMNMF_OK;
}

// forward pass; train: keep the pre-activations (z1, z2, z3) for backward
symnmf_status forward(symnmf_mlp* m, const float* X, int64_t rows, bool bf16, bool train, float* A) {
    symnmf_ctx* ctx = m->ctx;
    hipStream_t sm = ctx->stream;
    symnmf_status s = ensure_fwd(m, rows);
    if (s != SYMNMF_OK) return s;
    if (bf16 && m->bf16_stale) {
        HIP_OK(ctx, launch_to_bf16(m->P, m->Wb, m->nw, sm));
        m->bf16_stale = false;
    }
    const void* W1 = bf16 ? (const void*)(m->Wb + m->off_W1()) : (const void*)(m->P + m->off_W1());
    const void* W2 = bf16 ? (const void*)(m->Wb + m->off_W2()) : (const void*)(m->P + m->off_W2());
    const void* W3 = bf16 ? (const void*)(m->Wb + m->off_W3()) : (const void*)(m->P + m->off_W3());
    const int b = bf16 ? 1 : 0;
    HIP_OK(ctx, launch_gemm(0, 0, b, 1, X, W1, m->P + m->off_b1(), m->a1, train ? m->z1 : nullptr, rows, m->h, m->w,
                            1.0f, nullptr, 0, sm));
    HIP_OK(ctx, launch_gemm(0, 0, b, 1, m->a1, W2, m->P + m->off_b2(), m->a2, train ? m->z2 : nullptr, rows, m->h,
                            m->h, 1.0f, nullptr, 0, sm));
    HIP_OK(ctx, launch_gemm(0, 0, b, m->residual ? 0 : 2, m->a2, W3, m->P + m->off_b3(), A, train ? m->z3 : nullptr,
                            rows, m->k, m->h, 1.0f, nullptr, 0, sm));
    if (m->residual) HIP_OK(ctx, launch_residual_relu(X, m->w, A, rows, m->k, sm));
    return SYMNMF_OK;
}

}  // namespace

extern "C" {

int64_t symnmf_mlp_param_count(int64_t width, int64_t hidden, int64_t k) {
    if (width < 1 || width > KMAX || k < 1 || k > KMAX || hidden < 1 || hidden > 1024) return -1;
    return hidden * width + hidden * hidden + k * hidden + 2 * hidden + k;
}

symnmf_status symnmf_mlp_init(symnmf_ctx* ctx, int64_t width, int64_t hidden, int64_t k, uint64_t seed,
                              float* params) {
    if (!ctx) return SYMNMF_EINVAL;
    const int64_t np = symnmf_mlp_param_count(width, hidden, k);
    if (np < 0 || !params) return fail(ctx, SYMNMF_EINVAL, "mlp_init: bad argument");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t rows[3] = {hidden, hidden, k}, cols[3] = {width, hidden, hidden};
    int64_t off = 0;
    for (int l = 0; l < 3; ++l) {
        HIP_OK(ctx, launch_omega(4 * seed + 1 + l, rows[l], rows[l], (int)cols[l], params + off, sm));
        HIP_OK(ctx, launch_scale(params + off, rows[l] * cols[l], (float)(1.0 / std::sqrt((double)cols[l])), sm));
        off += rows[l] * cols[l];
    }
    HIP_OK(ctx, launch_zero(params + off, (np - off) * 4, sm));
    return SYMNMF_OK;
}

symnmf_status symnmf_mlp_create(symnmf_ctx* ctx, int64_t width, int64_t hidden, int64_t k, const float* params,
                                symnmf_mlp** out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!out || !params) return fail(ctx, SYMNMF_EINVAL, "mlp_create: null argument");
    *out = nullptr;
    const int64_t np = symnmf_mlp_param_count(width, hidden, k);
    if (np < 0) return fail(ctx, SYMNMF_EINVAL, "mlp_create: sizes outside w, k in [1, 64], h in [1, 1024]");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    auto* m = new symnmf_mlp();
    m->ctx = ctx;
    m->w = width;
    m->h = hidden;
    m->k = k;
    m->np = np;
    m->nw = hidden * width + hidden * hidden + k * hidden;
    // split-K partials of the weight gradients: at most 64 splits of the largest W
    m->split_floats = 64 * std::max({hidden * width, hidden * hidden, k * hidden});
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMalloc((void**)&m->P, np * 4));
    chk(hipMalloc((void**)&m->G, np * 4));
    chk(hipMalloc((void**)&m->Mm, np * 4));
    chk(hipMalloc((void**)&m->V, np * 4));
    chk(hipMalloc((void**)&m->Wb, m->nw * 2));
    chk(hipMalloc((void**)&m->split_ws, m->split_floats * 4));
    if (e == hipSuccess) chk(hipMemcpyAsync(m->P, params, np * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (e == hipSuccess) chk(launch_zero(m->G, np * 4, ctx->stream));
    if (e == hipSuccess) chk(launch_zero(m->Mm, np * 4, ctx->stream));
    if (e == hipSuccess) chk(launch_zero(m->V, np * 4, ctx->stream));
    if (e != hipSuccess) {
        symnmf_mlp_destroy(m);
        return fail(ctx, e == hipErrorOutOfMemory ? SYMNMF_ENOMEM : SYMNMF_EDEVICE, "mlp_create: %s",
                    hipGetErrorString(e));
    }
    *out = m;
    return SYMNMF_OK;
}

void symnmf_mlp_destroy(symnmf_mlp* m) {
    if (!m) return;
    if (m->ctx) (void)hipStreamSynchronize(m->ctx->stream);
    free_all({m->P, m->G, m->Mm, m->V, m->Wb, m->split_ws, m->small, m->a1, m->a2, m->z1, m->z2, m->z3, m->out, m->dA,
              m->d3, m->da2});
    delete m;
}

symnmf_status symnmf_mlp_set_output(symnmf_ctx* ctx, symnmf_mlp* m, int32_t residual) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!m || m->ctx != ctx || (residual != 0 && residual != 1))
        return fail(ctx, SYMNMF_EINVAL, "mlp_set_output: bad argument");
    if (residual && m->k > m->w) return fail(ctx, SYMNMF_EINVAL, "mlp_set_output: the residual form needs k <= width");
    m->residual = residual;
    return SYMNMF_OK;
}

symnmf_status symnmf_mlp_reserve(symnmf_ctx* ctx, symnmf_mlp* m, int64_t rows, int32_t training) {
    if (!ctx || !m || m->ctx != ctx || rows < 1) return ctx ? fail(ctx, SYMNMF_EINVAL, "mlp_reserve: bad argument")
                                                          : SYMNMF_EINVAL;
    HIP_OK(ctx, hipSetDevice(ctx->device));
    symnmf_status s = ensure_fwd(m, rows);
    if (s == SYMNMF_OK && training) s = ensure_train(m, rows);
    return s;
}

symnmf_status symnmf_mlp_read(symnmf_ctx* ctx, const symnmf_mlp* m, int32_t which, float* dst) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!m || !dst || m->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "mlp_read: bad argument");
    const float* src = which == 0 ? m->P : which == 1 ? m->G : which == 2 ? m->Mm : which == 3 ? m->V : nullptr;
    if (!src) return fail(ctx, SYMNMF_EINVAL, "mlp_read: bad buffer id %d", which);
    HIP_OK(ctx, hipMemcpyAsync(dst, src, m->np * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return SYMNMF_OK;
}

symnmf_status symnmf_mlp_write(symnmf_ctx* ctx, symnmf_mlp* m, const float* params) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!m || !params || m->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "mlp_write: bad argument");
    HIP_OK(ctx, hipMemcpyAsync(m->P, params, m->np * 4, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(ctx, launch_zero(m->Mm, m->np * 4, ctx->stream));
    HIP_OK(ctx, launch_zero(m->V, m->np * 4, ctx->stream));
    m->t = 0;
    m->bf16_stale = true;
    return SYMNMF_OK;
}

symnmf_status symnmf_mlp_forward(symnmf_ctx* ctx, symnmf_mlp* m, const float* X, int64_t rows, int32_t bf16_weights,
                                 float* A) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!m || !X || !A || rows < 1 || m->ctx != ctx) return fail(ctx, SYMNMF_EINVAL, "mlp_forward: bad argument");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    return forward(m, X, rows, bf16_weights != 0, false, A);
}

symnmf_status symnmf_mlp_train_step(symnmf_ctx* ctx, symnmf_mlp* m, const float* X, const float* B, int64_t rows,
                                    const symnmf_adamw* opt, int32_t loss_kind, double* loss) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!m || !X || !B || !opt || rows < 1 || m->ctx != ctx)
        return fail(ctx, SYMNMF_EINVAL, "mlp_train_step: bad argument");
    if (loss_kind != 0 && loss_kind != 1) return fail(ctx, SYMNMF_EINVAL, "mlp_train_step: loss_kind 0 or 1");
    if (!(opt->lr > 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) || !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) ||
        !(opt->eps >= 0.0) || !(opt->weight_decay >= 0.0))
        return fail(ctx, SYMNMF_EINVAL, "mlp_train_step: bad AdamW settings");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    symnmf_status s = ensure_train(m, rows);
    if (s != SYMNMF_OK) return s;
    s = forward(m, X, rows, false, true, m->out);
    if (s != SYMNMF_OK) return s;
    const int64_t k = m->k, h = m->h, w = m->w, kk = k * k;
    double* AtA = m->small;
    double* AtB = m->small + kk;
    double* BtB = m->small + 2 * kk;
    double* work = m->small + 3 * kk;
    HIP_OK(ctx, launch_xty(m->out, k, k, m->out, k, k, rows, work, AtA, sm));
    HIP_OK(ctx, launch_xty(m->out, k, k, B, k, k, rows, work, AtB, sm));
    HIP_OK(ctx, launch_xty(B, k, k, B, k, k, rows, work, BtB, sm));
    std::vector<double> hs(3 * kk);
    HIP_OK(ctx, hipMemcpyAsync(hs.data(), m->small, 3 * kk * 8, hipMemcpyDeviceToHost, sm));
    HIP_OK(ctx, hipStreamSynchronize(sm));
    double naa = 0.0, nab = 0.0, nbb = 0.0;
    for (int64_t e = 0; e < kk; ++e) {
        naa += hs[e] * hs[e];
        nab += hs[kk + e] * hs[kk + e];
        nbb += hs[2 * kk + e] * hs[2 * kk + e];
    }
    if (!(nbb > 0.0) || !std::isfinite(nbb)) return fail(ctx, SYMNMF_EINVAL, "mlp_train_step: target B^T B is zero");
    double L, ca, cb;
    if (loss_kind == 0) {
        // ||A A^T - B B^T||^2 / ||B^T B||^2, gradient 4 (A (A^T A) - B (B^T A)) / ||B^T B||^2
        L = (naa - 2.0 * nab + nbb) / nbb;
        ca = cb = 4.0 / nbb;
    } else {
        // 1 - ||A^T B||^4 / (||A^T A||^2 ||B^T B||^2), gradient
        // (4 b / (a c)) ((b / a) A (A^T A) - B (B^T A)) with a, b, c = naa, nab, nbb
        if (!(naa > 0.0)) return fail(ctx, SYMNMF_ENUMERIC, "mlp_train_step: network output is zero");
        L = 1.0 - nab * nab / (naa * nbb);
        cb = 4.0 * nab / (naa * nbb);
        ca = cb * nab / naa;
    }
    if (loss) *loss = L;
    if (!std::isfinite(L)) return fail(ctx, SYMNMF_ENUMERIC, "mlp_train_step: non-finite loss");
    // backward
    HIP_OK(ctx, launch_gram_loss_grad(m->out, B, AtA, AtB, k, rows, (float)ca, (float)cb, m->dA, sm));
    if (m->residual) HIP_OK(ctx, launch_residual_relu_backward(m->dA, X, w, m->z3, m->d3, rows, k, sm));
    else HIP_OK(ctx, launch_act_backward(m->dA, m->z3, m->d3, rows * k, 2, sm));
    HIP_OK(ctx, launch_gemm(1, 1, 0, 0, m->d3, m->a2, nullptr, m->G + m->off_W3(), nullptr, k, h, rows, 1.0f,
                            m->split_ws, m->split_floats, sm));
    HIP_OK(ctx, launch_colsum(m->d3, rows, k, m->G + m->off_b3(), sm));
    HIP_OK(ctx, launch_gemm(0, 1, 0, 0, m->d3, m->P + m->off_W3(), nullptr, m->da2, nullptr, rows, h, k, 1.0f, nullptr,
                            0, sm));
    HIP_OK(ctx, launch_act_backward(m->da2, m->z2, m->da2, rows * h, 1, sm));        // d2
    HIP_OK(ctx, launch_gemm(1, 1, 0, 0, m->da2, m->a1, nullptr, m->G + m->off_W2(), nullptr, h, h, rows, 1.0f,
                            m->split_ws, m->split_floats, sm));
    HIP_OK(ctx, launch_colsum(m->da2, rows, h, m->G + m->off_b2(), sm));
    // da1 = d2 W2 into a2 (no longer needed), then d1 in place
    HIP_OK(ctx, launch_gemm(0, 1, 0, 0, m->da2, m->P + m->off_W2(), nullptr, m->a2, nullptr, rows, h, h, 1.0f, nullptr,
                            0, sm));
    HIP_OK(ctx, launch_act_backward(m->a2, m->z1, m->a2, rows * h, 1, sm));
    HIP_OK(ctx, launch_gemm(1, 1, 0, 0, m->a2, X, nullptr, m->G + m->off_W1(), nullptr, h, w, rows, 1.0f, m->split_ws,
                            m->split_floats, sm));
    HIP_OK(ctx, launch_colsum(m->a2, rows, h, m->G + m->off_b1(), sm));
    m->t += 1;
    HIP_OK(ctx, launch_adamw(m->P, m->G, m->Mm, m->V, m->np, m->nw, (float)opt->lr, (float)opt->beta1,
                             (float)opt->beta2, (float)opt->eps, (float)opt->weight_decay, m->t, sm));
    m->bf16_stale = true;
    return SYMNMF_OK;
}

// Scratch of symnmf_sketch: Omega (every column of S), the S.Omega partials and
// the chunk images of Omega.
struct SketchWs {
    int64_t om, part, img;
};
static SketchWs sketch_ws(const symnmf_ctx* ctx, const symnmf_S* S, int64_t width) {
    SketchWs w;
    const int64_t tiles = S->rows_pad / TR, chunks = S->ld / KC;
    const int32_t P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : stream_wgs_per_cu(S->dtype, width));
    const int64_t hrows = std::max(S->ld, S->row0 + S->rows_pad);
    w.om = hrows * width * 4;
    w.part = ((int64_t)P + tiles) * TR * width * 4;
    w.img = stream_uses_mfma(S->dtype, 0, 0, width) ? h_image_words(S->dtype, width, chunks) * 4 : 0;
    return w;
}

// Scratch of symnmf_canonical.
static int64_t canonical_ws(int64_t n, int64_t width, int64_t k) {
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    return ws_sum({xty_work_doubles(n, width, width) * 8, width * width * 8, width * width * 8, width * k * 8, k * 8, 8,
                   n * k * 8, nb * 8, nb * 8, k * 8, width * k * 8});
}

int64_t symnmf_sketch_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t width) {
    if (!ctx || !S || width < 1 || width > KMAX) return -1;
    const SketchWs w = sketch_ws(ctx, S, width);
    return ws_sum({w.om, w.part}) + (w.img ? ws_round(w.img) : 0);
}

int64_t symnmf_canonical_workspace(int64_t n, int64_t width, int64_t k) {
    if (n < 1 || width < 1 || width > KMAX || k < 1 || k > width) return -1;
    return canonical_ws(n, width, k);
}

int64_t symnmf_warm_start_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t width, int64_t k) {
    if (!ctx || !S || width < 1 || width > KMAX || k < 1 || k > width) return -1;
    // Y and the coordinates, then (one at a time) the sketch, the canonical
    // coordinates and the objective terms of the alpha rescaling
    const int64_t inner = std::max({symnmf_sketch_workspace(ctx, S, width), canonical_ws(S->n, width, k),
                                    symnmf_objective_workspace(ctx, S, k, 0)});
    return ws_sum({S->n * width * 4, S->n * width * 4}) + inner;
}

int64_t symnmf_subspace_error_workspace(int64_t n, int64_t k) {
    if (n < 1 || k < 1 || k > KMAX) return -1;
    return ws_round((6 * k * k + k + 1 + xty_work_doubles(n, k, k)) * 8 + 16);
}

symnmf_status symnmf_sketch(symnmf_ctx* ctx, const symnmf_S* S, uint64_t omega_seed, int64_t width, float* Y) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !Y || width < 1 || width > KMAX) return fail(ctx, SYMNMF_EINVAL, "sketch: bad argument");
    if (S->dtype == SYMNMF_S_FP64) return fail(ctx, SYMNMF_EUNSUPPORTED, "sketch: FP64 storage is for parity runs");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t tiles = S->rows_pad / TR, chunks = S->ld / KC;
    const int32_t P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu : stream_wgs_per_cu(S->dtype, width));
    const bool mfma = stream_uses_mfma(S->dtype, 0, 0, width) != 0;
    const int64_t hrows = std::max(S->ld, S->row0 + S->rows_pad);
    const SketchWs ws = sketch_ws(ctx, S, width);
    CallScratch sc(ctx);
    void* Om = sc.get(ws.om, false);
    void* part = sc.get(ws.part, false);
    void* img = mfma ? sc.get(ws.img, false) : nullptr;
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "sketch");
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    {
        chk(launch_omega(omega_seed, S->n, hrows, (int)width, (float*)Om, sm));
        if (mfma) chk(launch_h_image((const float*)Om, S->dtype, width, chunks, 1.0f, (uint32_t*)img, sm));
        PlanView pv = plan_view(nullptr, 1, (int32_t)tiles, (int32_t)chunks, P);
        chk(launch_stream(S->data, S->dtype, S->ld, Om, 0, width, part, 0, pv, sm, img, img));
        chk(launch_sh_dense((const float*)part, S->rows, S->rows_pad, width, (int32_t)chunks, P, (const float*)Om,
                            S->row0, S->dtype == SYMNMF_S_FP8 ? S->panel_scale : nullptr, S->diag,
                            S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1, Y, sm));
        chk(hipStreamSynchronize(sm));
    }
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "sketch: %s", hipGetErrorString(e));
    return SYMNMF_OK;
}

symnmf_status symnmf_canonical(symnmf_ctx* ctx, const float* Y, int64_t n, int64_t width, int64_t k, float* X,
                               int64_t* anchors) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!Y || !X || width < 1 || width > KMAX || k < 1 || k > width || n < width)
        return fail(ctx, SYMNMF_EINVAL, "canonical: need 1 <= k <= width <= 64 and n >= width");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    CallScratch sc(ctx);
    void* work = sc.get(xty_work_doubles(n, width, width) * 8, false);
    void* G = sc.get(width * width * 8, false);
    void* V = sc.get(width * width * 8, false);
    void* M = sc.get(width * k * 8, false);
    void* lam = sc.get(k * 8, false);
    void* status = sc.get(8);
    void* R = sc.get(n * k * 8, false);
    void* bval = sc.get(nb * 8, false);
    void* bidx = sc.get(nb * 8, false);
    void* pick = sc.get(k * 8, false);
    void* W = sc.get(width * k * 8, false);
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "canonical");
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    int32_t st[2] = {0, 0};
    {
        chk(launch_xty(Y, width, width, Y, width, width, n, (double*)work, (double*)G, sm));
        chk(launch_jacobi_topk((const double*)G, width, k, (double*)V, (double*)M, (double*)lam, (int32_t*)status, sm));
        chk(launch_project_rows(Y, n, width, (const double*)M, k, k, 1, R, sm));
        chk(launch_spa((double*)R, n, k, (double*)bval, (int64_t*)bidx, nb, (int64_t*)pick, sm));
        chk(launch_anchor_solve(Y, width, (const double*)M, k, (const int64_t*)pick, (double*)W,
                                (int32_t*)status + 1, sm));
        chk(launch_project_rows(Y, n, width, (const double*)W, k, width, 0, X, sm));
        if (anchors) chk(hipMemcpyAsync(anchors, pick, k * 8, hipMemcpyDeviceToDevice, sm));
        chk(hipMemcpyAsync(st, status, 8, hipMemcpyDeviceToHost, sm));
        chk(hipStreamSynchronize(sm));
    }
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "canonical: %s", hipGetErrorString(e));
    if (st[0] == 1) return fail(ctx, SYMNMF_ENUMERIC, "canonical: Y^T Y has a non-positive eigenvalue among the top k");
    if (st[0] == 2) return fail(ctx, SYMNMF_ENUMERIC, "canonical: Jacobi sweeps did not converge");
    if (st[1] == 3) return fail(ctx, SYMNMF_ENUMERIC, "canonical: anchor rows are linearly dependent");
    return SYMNMF_OK;
}

symnmf_status symnmf_warm_start(symnmf_ctx* ctx, const symnmf_S* S, symnmf_mlp* mlp, int64_t width, int64_t k,
                                uint64_t omega_seed, float* H0) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!S || !H0 || width < 1 || width > KMAX || k < 1 || k > width)
        return fail(ctx, SYMNMF_EINVAL, "warm_start: bad argument");
    if (S->rows != S->n || S->row0 != 0)
        return fail(ctx, SYMNMF_EUNSUPPORTED, "warm_start: needs the full matrix, not a row panel");
    if (mlp && (mlp->w != width || mlp->k != k || mlp->ctx != ctx))
        return fail(ctx, SYMNMF_EINVAL, "warm_start: network sizes do not match width and k");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t n = S->n;
    CallScratch sc(ctx);
    float* Y = (float*)sc.get(n * width * 4, false);
    float* X = (float*)sc.get(n * width * 4, false);
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "warm_start");
    symnmf_status s = symnmf_sketch(ctx, S, omega_seed, width, Y);
    if (s == SYMNMF_OK) s = symnmf_canonical(ctx, Y, n, width, k, X, nullptr);
    if (s == SYMNMF_OK) {
        if (mlp) s = forward(mlp, X, n, true, false, H0);
        else if (launch_clip_cols(X, n, width, k, H0, sm) != hipSuccess)
            s = fail(ctx, SYMNMF_EDEVICE, "warm_start: clip launch failed");
    }
    double tr = 0.0, gn = 0.0;
    if (s == SYMNMF_OK) s = objective_terms(ctx, S, H0, 0, k, &tr, &gn);
    if (s != SYMNMF_OK) return s;
    if (!(gn > 0.0) || !std::isfinite(gn) || !std::isfinite(tr))
        return fail(ctx, SYMNMF_ENUMERIC, "warm_start: the initial factor is zero or non-finite");
    const double alpha = std::sqrt(std::max(tr, 0.0) / gn);
    HIP_OK(ctx, launch_scale(H0, n * k, (float)alpha, sm));
    HIP_OK(ctx, hipStreamSynchronize(sm));
    return SYMNMF_OK;
}

symnmf_status symnmf_subspace_error(symnmf_ctx* ctx, const float* A, const float* B, int64_t n, int64_t k,
                                    double* out) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!A || !B || !out || k < 1 || k > KMAX || n < k) return fail(ctx, SYMNMF_EINVAL, "subspace_error: bad argument");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t kk = k * k;
    // AtA, BtB, AtB, V, MA, MB, lam(k), overlap(1), work
    const int64_t work = xty_work_doubles(n, k, k);
    CallScratch sc(ctx);
    double* d = (double*)sc.get((6 * kk + k + 1 + work) * 8 + 16);
    if (sc.err != hipSuccess) return scratch_fail(ctx, sc, "subspace_error");
    double *AtA = d, *BtB = d + kk, *AtB = d + 2 * kk, *V = d + 3 * kk, *MA = d + 4 * kk, *MB = d + 5 * kk;
    double *lam = d + 6 * kk, *ov = lam + k, *wk = ov + 1;
    int32_t* status = (int32_t*)(wk + work);
    int32_t st[2] = {0, 0};
    double overlap = 0.0;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(launch_xty(A, k, k, A, k, k, n, wk, AtA, sm));
    chk(launch_xty(B, k, k, B, k, k, n, wk, BtB, sm));
    chk(launch_xty(A, k, k, B, k, k, n, wk, AtB, sm));
    chk(launch_jacobi_topk(AtA, k, k, V, MA, lam, status, sm));
    chk(launch_jacobi_topk(BtB, k, k, V, MB, lam, status + 1, sm));
    chk(launch_span_overlap(MA, AtB, MB, k, ov, sm));
    chk(hipMemcpyAsync(&overlap, ov, 8, hipMemcpyDeviceToHost, sm));
    chk(hipMemcpyAsync(st, status, 8, hipMemcpyDeviceToHost, sm));
    chk(hipStreamSynchronize(sm));
    if (e != hipSuccess) return fail(ctx, SYMNMF_EDEVICE, "subspace_error: %s", hipGetErrorString(e));
    if (st[0] || st[1]) return fail(ctx, SYMNMF_ENUMERIC, "subspace_error: a factor does not have full column rank");
    *out = std::sqrt(std::max(0.0, 2.0 * (double)k - 2.0 * overlap) / (2.0 * (double)k));
    return SYMNMF_OK;
}

}  // extern "C"
