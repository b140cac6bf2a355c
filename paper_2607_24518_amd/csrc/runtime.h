// Internal declarations shared by the C-ABI translation units: the context
// object, error reporting and the objective terms helper.
#pragma once
#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

struct symnmf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 256;
    int wgs_per_cu = 0;   // 0: chosen per kernel (SYMNMF_WGS_PER_CU overrides)
    std::string err;
    // optional HIP-event timing of every kernel a step launches
    bool profiling = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;   // (kernel id, start/stop)
};

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
