// S.H row-panel stream: the dominant O(n^2 k) product of every iteration
// (paper section "Computational Methodology": S x H dominates each step).
//
// Work split: see PlanView in common.h.  Each persistent work-group walks its
// unit range; per unit it stages the H rows of one 256-column chunk in LDS
// (permuted into the MFMA B-operand order, scaled by the chunk weight) and
// streams a 256-row x 256-column tile of S from HBM straight into MFMA
// A-operand registers.  Each wave owns 64 rows (4 MFMA row groups) so every
// B fragment read from LDS feeds 4 MFMAs.
//
// MFMA operand layouts used (CDNA3/CDNA4, 64-lane wave, lane l, r = l%16,
// g = l/16):
//   v_mfma_f32_16x16x4_f32 : A[r][g], B[g][r], D[4g+v][r] (v = 0..3)
//   v_mfma_f32_16x16x32_bf16: A[r][8g..8g+7], B[8g..8g+7][r], D as above
// The reduction index of one MFMA may be any permutation of the columns as
// long as A and B agree; each kernel picks the one that lets a lane load a
// contiguous 16-byte piece of its S row.
#include "common.h"

namespace symnmf {

__device__ inline void plan_bounds(const PlanView& p, int64_t& U, int32_t& na) {
    if (p.full) {
        na = p.n_tiles;
        U = (int64_t)p.n_tiles * p.n_chunks;
    } else {
        na = p.hdr[0];
        U = (int64_t)(uint32_t)p.hdr[1] | ((int64_t)p.hdr[2] << 32);
    }
}
__device__ inline int64_t unit_off(const PlanView& p, int32_t a) {
    return p.full ? (int64_t)a * p.n_chunks : (int64_t)p.unit_offset[a];
}
__device__ inline int32_t find_active(const PlanView& p, int64_t u, int32_t na) {
    if (p.full) return (int32_t)(u / p.n_chunks);
    int lo = 0, hi = na - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((int64_t)p.unit_offset[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ inline void unit_chunk(const PlanView& p, int32_t a, int64_t j, int32_t& chunk, float& w) {
    if (p.full) { chunk = (int32_t)j; w = 1.0f; return; }
    int c = p.active_class[a];
    chunk = p.class_chunks[c * p.n_chunks + j];
    w = (float)p.class_weight[c * p.n_chunks + j];
}
__device__ inline int32_t tile_of(const PlanView& p, int32_t a) { return p.full ? a : p.active_tile[a]; }

// ---------------------------------------------------------------------------
// Generic kernel: any storage type, FP32 or FP64 H and accumulation, k <= KB.
// One thread per row of the tile.  Used for FP64 parity runs, ranks that are
// not a multiple of 16, and the FP64-accumulated objective.
// ---------------------------------------------------------------------------
template <typename ST, typename HT, typename AT, int KB>
__global__ __launch_bounds__(256) void stream_generic(const ST* __restrict__ S, int64_t ld,
                                                      const HT* __restrict__ H, int k,
                                                      AT* __restrict__ part, PlanView p) {
    constexpr int SUB = 32;
    __shared__ AT Hs[SUB * KB];
    int64_t U; int32_t na;
    plan_bounds(p, U, na);
    if (U == 0) return;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w = blockIdx.x;
    if (w >= Pe) return;
    int64_t u = wg_start(w, U, Pe);
    const int64_t u1 = wg_start(w + 1, U, Pe);
    int32_t a = find_active(p, u, na);
    const int t = threadIdx.x;
    while (u < u1) {
        const int64_t abase = unit_off(p, a);
        const int64_t run_end = min(u1, unit_off(p, a + 1));
        const int64_t tile = tile_of(p, a);
        AT acc[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[c] = 0;
        const ST* srow = S + (tile * TR + t) * ld;
        for (; u < run_end; ++u) {
            int32_t chunk; float wt;
            unit_chunk(p, a, u - abase, chunk, wt);
            for (int sub = 0; sub < KC; sub += SUB) {
                __syncthreads();
                for (int f = t; f < SUB * k; f += 256) {
                    int kk = f / k, c = f - kk * k;
                    Hs[kk * KB + c] = (AT)H[((int64_t)chunk * KC + sub + kk) * k + c] * (AT)wt;
                }
                __syncthreads();
                const ST* sp = srow + (int64_t)chunk * KC + sub;
                for (int kk = 0; kk < SUB; ++kk) {
                    const AT s = (AT)load_as_f64(sp + kk);
#pragma unroll
                    for (int c = 0; c < KB; ++c)
                        if (c < k) acc[c] += s * Hs[kk * KB + c];
                }
            }
        }
        AT* dst = part + ((w + a) * TR + t) * (int64_t)k;
#pragma unroll
        for (int c = 0; c < KB; ++c)
            if (c < k) dst[c] = acc[c];
        ++a;
    }
}

// ---------------------------------------------------------------------------
// FP32 S: v_mfma_f32_16x16x4_f32.  Lane (r, g) of wave wv holds, for row
// group rg and sub-step s, the float4 S[row][16 s + 4 g .. +3] of row
// 64 wv + 16 rg + r; MFMA number m of the sub-step reduces over columns
// 16 s + 4 g + m.  H is staged as Hs[nt][s][g][c][m].
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256, 2) void stream_mfma_f32(const float* __restrict__ S, int64_t ld,
                                                          const float* __restrict__ H,
                                                          float* __restrict__ part, PlanView p) {
    constexpr int K = 16 * NT;
    __shared__ __attribute__((aligned(16))) float Hs[KC * K];
    int64_t U; int32_t na;
    plan_bounds(p, U, na);
    if (U == 0) return;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w = blockIdx.x;
    if (w >= Pe) return;
    int64_t u = wg_start(w, U, Pe);
    const int64_t u1 = wg_start(w + 1, U, Pe);
    int32_t a = find_active(p, u, na);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    while (u < u1) {
        const int64_t abase = unit_off(p, a);
        const int64_t run_end = min(u1, unit_off(p, a + 1));
        const int64_t tile = tile_of(p, a);
        floatx4 acc[4][NT];
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[rg][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float* sbase = S + (tile * TR + 64 * wv + lr) * ld + 4 * lg;
        for (; u < run_end; ++u) {
            int32_t chunk; float wt;
            unit_chunk(p, a, u - abase, chunk, wt);
            __syncthreads();
            const float* hsrc = H + (int64_t)chunk * KC * K;
            for (int f = threadIdx.x; f < KC * K; f += 256) {
                const int kk = f / K, col = f % K;
                const int nt = col >> 4, c = col & 15, s = kk >> 4, g = (kk >> 2) & 3, m = kk & 3;
                Hs[((((nt * 16 + s) * 4 + g) * 16 + c) << 2) + m] = hsrc[f] * wt;
            }
            __syncthreads();
            const float* sp = sbase + (int64_t)chunk * KC;
#pragma unroll 4
            for (int s = 0; s < 16; ++s) {
                floatx4 av[4];
#pragma unroll
                for (int rg = 0; rg < 4; ++rg)
                    av[rg] = __builtin_nontemporal_load((const floatx4*)(sp + (int64_t)(16 * rg) * ld + 16 * s));
                floatx4 bv[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    bv[nt] = *(const floatx4*)&Hs[(((nt * 16 + s) * 4 + lg) * 16 + lr) << 2];
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[rg][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rg][m], bv[nt][m],
                                                                               acc[rg][nt], 0, 0, 0);
            }
        }
        float* dst = part + (w + a) * (int64_t)TR * K;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dst[(64 * wv + 16 * rg + 4 * lg + v) * K + 16 * nt + lr] = acc[rg][nt][v];
        ++a;
    }
}

// Split x into three bfloat16 pieces hi + mid + lo (each rounded to nearest
// even from the remainder), which carry the 24 significand bits of x.
__device__ inline void split3_bf16(float x, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    hi = f32_to_bf16_bits(x);
    const float r1 = x - bf16_bits_to_f32(hi);
    mid = f32_to_bf16_bits(r1);
    const float r2 = r1 - bf16_bits_to_f32(mid);
    lo = f32_to_bf16_bits(r2);
}

// ---------------------------------------------------------------------------
// BF16 / FP8 S: v_mfma_f32_16x16x32_bf16 with H carried as three bf16 planes
// (H = hi + mid + lo), so S_stored x H is formed to FP32 accuracy with FP32
// accumulation.
//  BF16: sub-step s (0..7) covers 32 columns; lane (r, g) loads the 8 values
//        S[row][32 s + 8 g .. +7]; H staged as Hb[p][nt][s][g][c][i].
//  FP8 : sub-step s (0..3) covers 64 columns; lane (r, g) loads the 16 codes
//        S[row][64 s + 16 g .. +15] and converts them to two bf16x8 halves h;
//        half h reduces over columns 64 s + 16 g + 8 h + i; H staged as
//        Hb[p][nt][s][h][g][c][i].  Codes are unscaled (scale applied by the
//        update kernel) and the unit diagonal is stored as 0.
// ---------------------------------------------------------------------------
template <int NT, bool FP8>
__global__ __launch_bounds__(256, 2) void stream_mfma_lp(const uint8_t* __restrict__ Sbytes, int64_t ld,
                                                         const float* __restrict__ H,
                                                         float* __restrict__ part, PlanView p) {
    constexpr int K = 16 * NT;
    constexpr int PLANE = KC * K;               // bf16 elements per plane
    constexpr int EB = FP8 ? 1 : 2;             // bytes per S element
    __shared__ __attribute__((aligned(16))) uint16_t Hb[3 * PLANE];
    int64_t U; int32_t na;
    plan_bounds(p, U, na);
    if (U == 0) return;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w = blockIdx.x;
    if (w >= Pe) return;
    int64_t u = wg_start(w, U, Pe);
    const int64_t u1 = wg_start(w + 1, U, Pe);
    int32_t a = find_active(p, u, na);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t ldb = ld * EB;
    while (u < u1) {
        const int64_t abase = unit_off(p, a);
        const int64_t run_end = min(u1, unit_off(p, a + 1));
        const int64_t tile = tile_of(p, a);
        floatx4 acc[4][NT];
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[rg][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        const uint8_t* sbase = Sbytes + (tile * TR + 64 * wv + lr) * ldb + 16 * lg;
        for (; u < run_end; ++u) {
            int32_t chunk; float wt;
            unit_chunk(p, a, u - abase, chunk, wt);
            __syncthreads();
            const float* hsrc = H + (int64_t)chunk * KC * K;
            for (int f = threadIdx.x; f < KC * K; f += 256) {
                const int kk = f / K, col = f % K;
                const int nt = col >> 4, c = col & 15;
                int idx;
                if (FP8) {
                    const int s = kk >> 6, g = (kk >> 4) & 3, h = (kk >> 3) & 1, i = kk & 7;
                    idx = (((((nt * 4 + s) * 2 + h) * 4 + g) * 16 + c) << 3) + i;
                } else {
                    const int s = kk >> 5, g = (kk >> 3) & 3, i = kk & 7;
                    idx = ((((nt * 8 + s) * 4 + g) * 16 + c) << 3) + i;
                }
                uint16_t hi, mid, lo;
                split3_bf16(hsrc[f] * wt, hi, mid, lo);
                Hb[idx] = hi;
                Hb[PLANE + idx] = mid;
                Hb[2 * PLANE + idx] = lo;
            }
            __syncthreads();
            const uint8_t* sp = sbase + (int64_t)chunk * KC * EB;
            constexpr int NS = FP8 ? 4 : 8;
#pragma unroll 2
            for (int s = 0; s < NS; ++s) {
                u32x4 raw[4];
#pragma unroll
                for (int rg = 0; rg < 4; ++rg)
                    raw[rg] = __builtin_nontemporal_load((const u32x4*)(sp + (int64_t)(16 * rg) * ldb + 64 * s));
#pragma unroll
                for (int h = 0; h < (FP8 ? 2 : 1); ++h) {
                    bf16x8 av[4];
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        if (FP8) {
                            const uint32_t w0 = h ? raw[rg][2] : raw[rg][0];
                            const uint32_t w1 = h ? raw[rg][3] : raw[rg][1];
                            bf16x2 q0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, false);
                            bf16x2 q1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, true);
                            bf16x2 q2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, false);
                            bf16x2 q3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, true);
                            av[rg] = bf16x8{q0[0], q0[1], q1[0], q1[1], q2[0], q2[1], q3[0], q3[1]};
                        } else {
                            av[rg] = __builtin_bit_cast(bf16x8, raw[rg]);
                        }
                    }
#pragma unroll
                    for (int pl = 0; pl < 3; ++pl) {
                        bf16x8 bv[NT];
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            int idx;
                            if (FP8) idx = (((((nt * 4 + s) * 2 + h) * 4 + lg) * 16 + lr) << 3);
                            else idx = ((((nt * 8 + s) * 4 + lg) * 16 + lr) << 3);
                            bv[nt] = *(const bf16x8*)&Hb[pl * PLANE + idx];
                        }
#pragma unroll
                        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                acc[rg][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rg], bv[nt],
                                                                                      acc[rg][nt], 0, 0, 0);
                    }
                }
            }
        }
        float* dst = part + (w + a) * (int64_t)TR * K;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dst[(64 * wv + 16 * rg + 4 * lg + v) * K + 16 * nt + lr] = acc[rg][nt][v];
        ++a;
    }
}

int stream_uses_mfma(int32_t stype, int h_f64, int acc_f64, int64_t k) {
    if (h_f64 || acc_f64 || stype == SYMNMF_S_FP64) return 0;
    return (k == 16 || k == 32 || k == 64) ? 1 : 0;
}

template <typename ST, typename HT, typename AT>
static hipError_t launch_generic(const void* S, int64_t ld, const void* H, int64_t k, void* part,
                                 const PlanView& p, hipStream_t stream) {
    dim3 grid(p.P), block(256);
    if (k <= 8)
        hipLaunchKernelGGL((stream_generic<ST, HT, AT, 8>), grid, block, 0, stream, (const ST*)S, ld,
                           (const HT*)H, (int)k, (AT*)part, p);
    else if (k <= 16)
        hipLaunchKernelGGL((stream_generic<ST, HT, AT, 16>), grid, block, 0, stream, (const ST*)S, ld,
                           (const HT*)H, (int)k, (AT*)part, p);
    else if (k <= 32)
        hipLaunchKernelGGL((stream_generic<ST, HT, AT, 32>), grid, block, 0, stream, (const ST*)S, ld,
                           (const HT*)H, (int)k, (AT*)part, p);
    else
        hipLaunchKernelGGL((stream_generic<ST, HT, AT, 64>), grid, block, 0, stream, (const ST*)S, ld,
                           (const HT*)H, (int)k, (AT*)part, p);
    return hipGetLastError();
}

template <typename ST>
static hipError_t launch_generic_s(const void* S, int64_t ld, const void* H, int h_f64, int64_t k, void* part,
                                   int acc_f64, const PlanView& p, hipStream_t stream) {
    if (h_f64) return launch_generic<ST, double, double>(S, ld, H, k, part, p, stream);
    if (acc_f64) return launch_generic<ST, float, double>(S, ld, H, k, part, p, stream);
    return launch_generic<ST, float, float>(S, ld, H, k, part, p, stream);
}

hipError_t launch_stream(const void* S, int32_t stype, int64_t ld, const void* H, int h_f64, int64_t k,
                         void* part, int acc_f64, const PlanView& p, hipStream_t stream) {
    if (k < 1 || k > KMAX) return hipErrorInvalidValue;
    if (stream_uses_mfma(stype, h_f64, acc_f64, k)) {
        dim3 grid(p.P), block(256);
        const float* Hf = (const float*)H;
        float* pf = (float*)part;
        if (stype == SYMNMF_S_FP32) {
            if (k == 16) hipLaunchKernelGGL(stream_mfma_f32<1>, grid, block, 0, stream, (const float*)S, ld, Hf, pf, p);
            else if (k == 32) hipLaunchKernelGGL(stream_mfma_f32<2>, grid, block, 0, stream, (const float*)S, ld, Hf, pf, p);
            else hipLaunchKernelGGL(stream_mfma_f32<4>, grid, block, 0, stream, (const float*)S, ld, Hf, pf, p);
        } else if (stype == SYMNMF_S_BF16) {
            const uint8_t* sb = (const uint8_t*)S;
            if (k == 16) hipLaunchKernelGGL((stream_mfma_lp<1, false>), grid, block, 0, stream, sb, ld, Hf, pf, p);
            else if (k == 32) hipLaunchKernelGGL((stream_mfma_lp<2, false>), grid, block, 0, stream, sb, ld, Hf, pf, p);
            else hipLaunchKernelGGL((stream_mfma_lp<4, false>), grid, block, 0, stream, sb, ld, Hf, pf, p);
        } else if (stype == SYMNMF_S_FP8) {
            const uint8_t* sb = (const uint8_t*)S;
            if (k == 16) hipLaunchKernelGGL((stream_mfma_lp<1, true>), grid, block, 0, stream, sb, ld, Hf, pf, p);
            else if (k == 32) hipLaunchKernelGGL((stream_mfma_lp<2, true>), grid, block, 0, stream, sb, ld, Hf, pf, p);
            else hipLaunchKernelGGL((stream_mfma_lp<4, true>), grid, block, 0, stream, sb, ld, Hf, pf, p);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (stype) {
        case SYMNMF_S_FP32: return launch_generic_s<float>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_BF16: return launch_generic_s<uint16_t>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_FP8: return launch_generic_s<uint8_t>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_FP64:
            if (!h_f64) return hipErrorInvalidValue;
            return launch_generic<double, double, double>(S, ld, H, k, part, p, stream);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Device self-check of the FP8 -> BF16 conversion instruction against the
// E4M3 definition (every finite code).  bad[0] counts mismatches.
// ---------------------------------------------------------------------------
__global__ void fp8_decode_check(int32_t* bad) {
    const int code = threadIdx.x;                       // 0..255
    if ((code & 0x7f) == 0x7f) return;                  // NaN codes
    const uint32_t word = (uint32_t)code | ((uint32_t)code << 8) | ((uint32_t)code << 16) | ((uint32_t)code << 24);
    bf16x2 lo = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(word, 1.0f, false);
    bf16x2 hi = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(word, 1.0f, true);
    const float ref = fp8e4m3_to_f32((uint8_t)code);
    const float v[4] = {(float)lo[0], (float)lo[1], (float)hi[0], (float)hi[1]};
    for (int i = 0; i < 4; ++i)
        if (v[i] != ref) atomicAdd(bad, 1);
}

hipError_t launch_fp8_decode_check(int32_t* bad, hipStream_t stream) {
    hipLaunchKernelGGL(fp8_decode_check, dim3(1), dim3(256), 0, stream, bad);
    return hipGetLastError();
}

}  // namespace symnmf
