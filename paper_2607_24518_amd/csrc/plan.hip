// Work plan of a sub-sampled step, built on the device so that steps stay
// asynchronous (no host round trip per iteration).
//
// Row-Stochastic SVRG (appendix, family 3): the rows of the sampled blocks I
// take their exact gradient, so their tiles stream every column chunk with
// weight 1.
//
// Block-SVRG AdaptGrow (appendix, family 3): with sampled block sets I and J,
//   g_I = 2 (H_I (H_J^T H_J) - S_IJ H_J),  g_J = 2 (H_J (H_I^T H_I) - S_JI H_I),
// summed on rows in both sets.  Per row tile the S.H term is one weighted sum
// over column chunks:
//   class 0 (rows in I only): chunks of J, weight 1, Gram_eff = Gram_J
//   class 1 (rows in J only): chunks of I, weight 1, Gram_eff = Gram_I
//   class 2 (rows in I and J): chunks of I u J, weight [b in J] + [b in I],
//                              Gram_eff = Gram_I + Gram_J
// so S_IJ and S_JI are read once, in trace form, with no |I| x |J| residual.
#include "common.h"

namespace symnmf {

constexpr int MAX_BLOCKS = 4096;

__global__ void plan_kernel(PlanRequest r, int32_t* __restrict__ base, int32_t* __restrict__ tiles_I,
                            int32_t* __restrict__ tiles_J, int32_t* __restrict__ counts) {
    __shared__ int32_t perm[MAX_BLOCKS];
    __shared__ uint8_t fI[MAX_BLOCKS];
    __shared__ uint8_t fJ[MAX_BLOCKS];
    if (threadIdx.x != 0) return;
    const int nt = r.n_tiles, nc = r.n_chunks;
    int32_t* hdr = base;
    int32_t* active_tile = base + 8;
    int32_t* active_class = active_tile + nt;
    int32_t* unit_offset = active_class + nt;
    int32_t* class_chunks = unit_offset + nt + 1;
    int32_t* class_weight = class_chunks + 3 * nc;
    int32_t* tile_active = class_weight + 3 * nc;

    sample_block_flags(r.seed, r.t, 0, r.n_blocks, r.m, perm, fI);
    if (r.mode == 2 && r.independent) {
        sample_block_flags(r.seed, r.t, 1, r.n_blocks, r.m, perm, fJ);
    } else {
        for (int b = 0; b < r.n_blocks; ++b) fJ[b] = r.mode == 2 ? fI[b] : 0;
    }
    int len[3] = {0, 0, 0};
    if (r.mode == 1) {
        for (int c = 0; c < nc; ++c) {
            class_chunks[c] = c;
            class_weight[c] = 1;
        }
        len[0] = nc;
    } else {
        for (int c = 0; c < nc; ++c) {
            const int b = c / r.chunks_per_block;
            const int inI = fI[b], inJ = fJ[b];
            if (inJ) { class_chunks[len[0]] = c; class_weight[len[0]] = 1; ++len[0]; }
            if (inI) { class_chunks[nc + len[1]] = c; class_weight[nc + len[1]] = 1; ++len[1]; }
            if (inI || inJ) { class_chunks[2 * nc + len[2]] = c; class_weight[2 * nc + len[2]] = inI + inJ; ++len[2]; }
        }
    }
    int na = 0, nI = 0, nJ = 0;
    int64_t U = 0;
    for (int i = 0; i < nt; ++i) {
        const int b = i / r.tiles_per_block;
        const int inI = fI[b], inJ = fJ[b];
        if (inI) tiles_I[nI++] = i;
        if (inJ) tiles_J[nJ++] = i;
        if (!(inI || inJ)) { tile_active[i] = -1; continue; }
        const int cls = r.mode == 1 ? 0 : (inI && inJ ? 2 : (inI ? 0 : 1));
        active_tile[na] = i;
        active_class[na] = cls;
        unit_offset[na] = (int32_t)U;
        tile_active[i] = na;
        U += len[cls];
        ++na;
    }
    unit_offset[na] = (int32_t)U;
    hdr[0] = na;
    hdr[1] = (int32_t)(uint32_t)(U & 0xffffffffu);
    hdr[2] = (int32_t)(U >> 32);
    hdr[3] = len[0];
    hdr[4] = len[1];
    hdr[5] = len[2];
    counts[0] = nI;
    counts[1] = nJ;
}

hipError_t launch_plan(const PlanRequest& r, int32_t* plan_base, int32_t* tiles_I, int32_t* tiles_J,
                       int32_t* counts, hipStream_t stream) {
    if (r.n_blocks > MAX_BLOCKS || r.m < 1 || r.m > r.n_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(64), 0, stream, r, plan_base, tiles_I, tiles_J, counts);
    return hipGetLastError();
}

}  // namespace symnmf
