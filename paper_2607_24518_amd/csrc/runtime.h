// Internal declarations shared by the C-ABI translation units: the context
// object, error reporting and the objective terms helper.
#pragma once
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

// Device scratch of the calls that need temporary buffers (S build, objective,
// median, sketch, canonical coordinates, warm start, subspace error, K-means)
// comes from a pool held by the context.  With a workspace attached
// (symnmf_set_workspace) the pool is that caller-owned buffer and a call that
// needs more fails with ENOMEM; otherwise the pool takes blocks from hipMalloc
// when a call needs more than it holds and keeps them until symnmf_destroy, so
// a call no larger than an earlier one allocates nothing.
struct WsBlock {
    char* p;
    int64_t bytes;
    bool owned;
};

struct symnmf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 256;
    int wgs_per_cu = 0;   // 0: chosen per kernel (SYMNMF_WGS_PER_CU overrides)
    std::string err;
    // optional HIP-event timing of every kernel a step launches
    bool profiling = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;   // (kernel id, start/stop)
    // scratch pool: blocks, and the top of the carved stack (block, offset)
    std::vector<WsBlock> ws;
    bool ws_attached = false;
    size_t ws_top_block = 0;
    int64_t ws_top_off = 0;
    int64_t ws_allocs = 0;   // blocks the pool has taken from hipMalloc
};

// bytes a scratch request occupies in the pool
inline int64_t ws_round(int64_t bytes) { return (std::max<int64_t>(bytes, 16) + 255) / 256 * 256; }
inline int64_t ws_sum(std::initializer_list<int64_t> sizes) {
    int64_t s = 0;
    for (int64_t b : sizes) s += ws_round(b);
    return s;
}

// The scratch of one call: buffers carved from the context pool in stack order
// (a call made inside another carves above its caller's buffers), zeroed on the
// context stream, returned to the pool when the object goes out of scope.
// Calls on one context run in its stream's order, so the next call may reuse
// the memory at once.
class CallScratch {
  public:
    explicit CallScratch(symnmf_ctx* c) : ctx_(c), block0_(c->ws_top_block), off0_(c->ws_top_off) {}
    ~CallScratch() {
        ctx_->ws_top_block = block0_;
        ctx_->ws_top_off = off0_;
    }
    CallScratch(const CallScratch&) = delete;
    CallScratch& operator=(const CallScratch&) = delete;
    void* get(int64_t bytes, bool zero = true);
    hipError_t err = hipSuccess;
    int64_t need = 0;   // bytes asked so far (rounded), also when a request failed

  private:
    symnmf_ctx* ctx_;
    size_t block0_;
    int64_t off0_;
};

// ENOMEM with the size the call needs when the attached workspace is too small,
// else EDEVICE / ENOMEM for the allocation error.
symnmf_status scratch_fail(symnmf_ctx* ctx, const CallScratch& sc, const char* what);

inline symnmf_status fail(symnmf_ctx* ctx, symnmf_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIP_OK(ctx, expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SYMNMF_ENOMEM : SYMNMF_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                             \
    } while (0)

// tr(H^T S H) and ||H^T H||_F^2 of any H (device n x k, float32 or float64),
// accumulated as symnmf_objective does.  Synchronises.
symnmf_status objective_terms(symnmf_ctx* ctx, const symnmf_S* S, const void* H, int32_t h_is_f64, int64_t k,
                              double* tr, double* gram_norm2);
