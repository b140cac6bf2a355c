// S.H row-panel stream: the dominant O(n^2 k) product of every iteration
// (paper section "Computational Methodology": S x H dominates each step).
//
// Work split: see PlanView in common.h.  Each persistent work-group walks its
// unit range; per unit (256-row tile x 256-column chunk) it streams the tile of
// S from HBM straight into MFMA A-operand registers - the tiled storage puts
// every wave's 64 rows of the tile in one contiguous run - while the H rows of
// the chunk sit in LDS in B-operand order.  Once per step a prep kernel writes
// H as "images", one per chunk, already in that LDS order (and, for BF16/FP8
// S, already split into bf16 planes), so staging a chunk is a plain 16-byte
// copy; the image of the next unit is fetched during the current unit and S
// loads run three sub-steps ahead across unit boundaries, so the S stream never
// drains.  Each wave owns 64 rows (4 MFMA row groups) so every B fragment read
// from LDS feeds 4 MFMAs.
//
// MFMA operand layouts used (CDNA3/CDNA4, 64-lane wave, lane l, r = l%16,
// g = l/16):
//   v_mfma_f32_16x16x4_f32 : A[r][g], B[g][r], D[4g+v][r] (v = 0..3)
//   v_mfma_f32_16x16x32_bf16: A[r][8g..8g+7], B[8g..8g+7][r], D as above
// The reduction index of one MFMA may be any permutation of the columns as
// long as A and B agree; each kernel uses the one in which a lane's 16 bytes
// of S are consecutive columns.
#include "common.h"

namespace symnmf {

__device__ inline void plan_bounds(const PlanView& p, int64_t& U, int32_t& na) {
    if (p.full) {
        na = p.tall ? (int32_t)tall_pairs(p.n_tiles) : p.n_tiles;
        U = (int64_t)na * p.n_chunks;
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

// unit u -> (active tile, chunk, weight), a = active tile holding u or a hint below it
__device__ inline void unit_decode(const PlanView& p, int64_t u, int32_t& a, int32_t& chunk, float& w) {
    while (u >= unit_off(p, a + 1)) ++a;
    unit_chunk(p, a, u - unit_off(p, a), chunk, w);
}

// ---------------------------------------------------------------------------
// Generic kernel: any storage type, FP32 or FP64 H and accumulation, k <= KB.
// One thread per row of the tile.  Used for FP64 parity runs, ranks that are
// not a multiple of 16, and the FP64-accumulated objective.
// ---------------------------------------------------------------------------
template <typename ST>
__device__ inline int64_t s_index(int64_t r, int64_t c, int64_t ld, int64_t n_chunks) {
    if (sizeof(ST) == 8) return r * ld + c;
    return tiled_offset(r, c, n_chunks, (int)(16 / sizeof(ST)));
}

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
        const int64_t row = tile * TR + t;
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
                const int64_t col0 = (int64_t)chunk * KC + sub;
                for (int kk = 0; kk < SUB; ++kk) {
                    const AT s = (AT)load_as_f64(S + s_index<ST>(row, col0 + kk, ld, p.n_chunks));
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
// FP64 storage (row-major, leading dimension ld), FP64 H and FP64 accumulation
// on the FP64 matrix cores, k = 16 NT.  v_mfma_f64_16x16x4_f64 (lane l,
// r = l % 16, g = l / 16): A[r][g], B[g][r], D[4v+g][r] (v = 0..3: the four
// output rows of a lane are interleaved, unlike the FP32 16x16x4 form).  A wave
// owns 64 rows of the tile (4 row groups of 16); per sub-step of 8 columns a
// lane loads 16 bytes (2 doubles) of its row in each row group, and the two
// MFMAs of an element e reduce over the columns 2g + e of the sub-step, with
// the matching H rows read from the chunk staged in LDS (scaled by the unit's
// weight).  S loads run one sub-step pair ahead.  Units and partials follow
// the plan as in stream_generic.
// ---------------------------------------------------------------------------
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int NT>
__global__ __launch_bounds__(256, 2) void stream_f64_mfma(const double* __restrict__ S, int64_t ld,
                                                          const double* __restrict__ H,
                                                          double* __restrict__ part, PlanView p) {
    constexpr int K = 16 * NT;
    constexpr int SS = KC / 8;                             // sub-steps of 8 columns per unit
    __shared__ double Hs[KC * K];
    int64_t U; int32_t na;
    plan_bounds(p, U, na);
    if (U == 0) return;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w = blockIdx.x;
    if (w >= Pe) return;
    int64_t u = wg_start(w, U, Pe);
    const int64_t u1 = wg_start(w + 1, U, Pe);
    int32_t a = find_active(p, u, na);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, lr = lane & 15, lg = lane >> 4;
    while (u < u1) {
        const int64_t abase = unit_off(p, a);
        const int64_t run_end = min(u1, unit_off(p, a + 1));
        const int64_t tile = tile_of(p, a);
        doublex4 acc[4][NT];
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[rg][nt] = doublex4{0.0, 0.0, 0.0, 0.0};
        const double* rowp[4];
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
            rowp[rg] = S + (tile * TR + 64 * wv + 16 * rg + lr) * ld + 2 * lg;
        for (; u < run_end; ++u) {
            int32_t chunk; float wt;
            unit_chunk(p, a, u - abase, chunk, wt);
            __syncthreads();
            const double* hsrc = H + (int64_t)chunk * KC * K;
            for (int f = t; f < KC * K; f += 256) Hs[f] = hsrc[f] * (double)wt;
            __syncthreads();
            const int64_t col0 = (int64_t)chunk * KC;
            doublex2 cur[2][4], nxt[2][4];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int rg = 0; rg < 4; ++rg) cur[q][rg] = *(const doublex2*)(rowp[rg] + col0 + 8 * q);
            for (int s = 0; s < SS; s += 2) {
                if (s + 2 < SS) {
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int rg = 0; rg < 4; ++rg)
                            nxt[q][rg] = *(const doublex2*)(rowp[rg] + col0 + 8 * (s + 2 + q));
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int kk = 8 * (s + q) + 2 * lg + e;
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            const double b = Hs[kk * K + 16 * nt + lr];
#pragma unroll
                            for (int rg = 0; rg < 4; ++rg)
                                acc[rg][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[q][rg][e], b, acc[rg][nt],
                                                                                   0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) cur[q][rg] = nxt[q][rg];
            }
        }
        double* dst = part + (w + a) * (int64_t)TR * K;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dst[(64 * wv + 16 * rg + 4 * v + lg) * K + 16 * nt + lr] = acc[rg][nt][v];
        ++a;
    }
}

// ---------------------------------------------------------------------------
// H images.  KIND 0 (FP32 S): floats in the order Hs[nt][s][g][c][m];
// KIND 1 (BF16 S): three bf16 planes, each Hb[nt][s][g][c][i];
// KIND 2 (FP8 S): three bf16 planes, each Hb[nt][s][h][g][c][i].
// (nt = H column / 16, c = H column % 16; the other indices split the chunk
// column kk as the matching kernel's sub-step reads it.)
// ---------------------------------------------------------------------------
__device__ inline void split3_bf16(float x, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    hi = f32_to_bf16_bits(x);
    const float r1 = x - bf16_bits_to_f32(hi);
    mid = f32_to_bf16_bits(r1);
    const float r2 = r1 - bf16_bits_to_f32(mid);
    lo = f32_to_bf16_bits(r2);
}

// First chunk row kk0 and H column of image vector v (16 bytes: 4 floats for
// KIND 0, 8 bf16 of one plane otherwise); the vector holds rows kk0, kk0 + 1, ...
// of that column, in the order given above.
template <int KIND>
__device__ inline void image_vector_origin(int v, int& kk0, int& col) {
    const int c = v & 15, g = (v >> 4) & 3;
    if (KIND == 0) {
        kk0 = 16 * ((v >> 6) & 15) + 4 * g;
        col = 16 * (v >> 10) + c;
    } else if (KIND == 1) {
        kk0 = 32 * ((v >> 6) & 7) + 8 * g;
        col = 16 * (v >> 9) + c;
    } else {
        kk0 = 64 * ((v >> 7) & 3) + 16 * g + 8 * ((v >> 6) & 1);
        col = 16 * (v >> 9) + c;
    }
}

template <int KIND, int K>
struct ImageShape {
    static constexpr int BUFW = KIND == 0 ? KC * K : 3 * KC * K / 2;   // 32-bit words per chunk image
    static constexpr int NV = BUFW / 4;                                 // 16-byte vectors per image
    static constexpr int PLANE = KC * K;                                // bf16 elements per plane
};

// One work-group per (chunk, block of CB columns of H): the block's 256 x CB
// values (scaled by wt) are staged in LDS with 16-byte loads, then every
// thread assembles whole 16-byte image vectors (all three bf16 planes at once
// for KIND 1, 2) and writes them in order.  Each 16-column block is a
// contiguous run of every plane of the image.  At k = 64 a work-group takes
// 16 columns (17 KB of LDS, eight work-groups per CU instead of two); below,
// the whole chunk.
template <int KIND, int K>
constexpr int image_cols_per_wg() { return K == 64 ? 16 : K; }

template <int KIND, int K>
__global__ __launch_bounds__(256) void h_image_kernel(const float* __restrict__ H, float wt,
                                                      u32x4* __restrict__ img) {
    using IS = ImageShape<KIND, K>;
    constexpr int CB = image_cols_per_wg<KIND, K>();
    constexpr int LDH = CB + 1;                           // padded row: column reads spread over banks
    constexpr int EPV = KIND == 0 ? 4 : 8;                // H values per image vector
    constexpr int VP = KC * K / EPV;                      // vectors per plane
    constexpr int VB = VP / (K / CB);                     // ... per plane and column block
    __shared__ float Hs[KC * LDH];
    const int64_t chunk = blockIdx.x;
    const int blk = blockIdx.y;
    const float* src = H + chunk * KC * K + CB * blk;
    for (int q = threadIdx.x; q < KC * CB / 4; q += 256) {
        const int r = q / (CB / 4), c = 4 * (q % (CB / 4));
        const float4 x = *(const float4*)(src + (int64_t)r * K + c);
        float* d = Hs + r * LDH + c;
        d[0] = x.x * wt;
        d[1] = x.y * wt;
        d[2] = x.z * wt;
        d[3] = x.w * wt;
    }
    __syncthreads();
    u32x4* out = img + chunk * IS::NV;
    for (int v = blk * VB + threadIdx.x; v < (blk + 1) * VB; v += 256) {
        int kk0, col;
        image_vector_origin<KIND>(v, kk0, col);
        col -= CB * blk;
        if (KIND == 0) {
            u32x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = __builtin_bit_cast(uint32_t, Hs[(kk0 + e) * LDH + col]);
            out[v] = o;
        } else {
            uint16_t hi[8], mid[8], lo[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) split3_bf16(Hs[(kk0 + e) * LDH + col], hi[e], mid[e], lo[e]);
            u32x4 a, b, c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[e] = (uint32_t)hi[2 * e] | ((uint32_t)hi[2 * e + 1] << 16);
                b[e] = (uint32_t)mid[2 * e] | ((uint32_t)mid[2 * e + 1] << 16);
                c[e] = (uint32_t)lo[2 * e] | ((uint32_t)lo[2 * e + 1] << 16);
            }
            out[v] = a;
            out[VP + v] = b;
            out[2 * VP + v] = c;
        }
    }
}

int64_t h_image_words(int32_t stype, int64_t k, int64_t n_chunks) {
    const int64_t per = stype == SYMNMF_S_FP32 ? KC * k : 3 * KC * k / 2;
    return per * n_chunks;
}

hipError_t launch_h_image(const float* H, int32_t stype, int64_t k, int64_t n_chunks, float wt, uint32_t* img,
                          hipStream_t stream) {
    dim3 grid(n_chunks, k == 64 ? 4 : 1), block(256);
#define IMG(KIND, KK) hipLaunchKernelGGL((h_image_kernel<KIND, KK>), grid, block, 0, stream, H, wt, (u32x4*)img)
    if (stype == SYMNMF_S_FP32) {
        if (k == 16) IMG(0, 16); else if (k == 32) IMG(0, 32); else if (k == 64) IMG(0, 64); else return hipErrorInvalidValue;
    } else if (stype == SYMNMF_S_BF16) {
        if (k == 16) IMG(1, 16); else if (k == 32) IMG(1, 32); else if (k == 64) IMG(1, 64); else return hipErrorInvalidValue;
    } else if (stype == SYMNMF_S_FP8) {
        if (k == 16) IMG(2, 16); else if (k == 32) IMG(2, 32); else if (k == 64) IMG(2, 64); else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
#undef IMG
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MFMA stream kernel.
//
// FP32 S (v_mfma_f32_16x16x4_f32): sub-step s (0..15) covers 16 columns;
//   lane (r, g) holds the float4 S[row][16 s + 4 g .. +3] of row
//   64 wv + 16 rg + r; MFMA number m reduces over columns 16 s + 4 g + m.
// BF16 S (v_mfma_f32_16x16x32_bf16, H = hi + mid + lo in three bf16 planes):
//   sub-step s (0..7) covers 32 columns; lane (r, g) holds S[row][32 s + 8 g
//   .. +7].
// FP8 S: sub-step s (0..3) covers 64 columns; lane (r, g) holds the 16 codes
//   S[row][64 s + 16 g .. +15], widened to two bf16x8 halves h; half h reduces
//   over columns 64 s + 16 g + 8 h + i.  Codes are unscaled (the update kernel
//   applies the panel scale) and the diagonal is stored as 0 (added back from
//   the FP32 diagonal).
// DB: two LDS image buffers (the next image is written while the current one
// is read); PF: the next image is then fetched into registers at the start of
// a unit (otherwise it is copied at the unit boundary).  Without DB the one
// buffer is refilled in QP parts: every (plane, 16-column) block of the image
// holds its sub-steps in order, so once all waves are past the sub-steps of
// part r (a barrier) the next image's part r is written over it (the last part
// at the unit's end); each part is fetched into registers one part ahead.
// ---------------------------------------------------------------------------
// ACC64: FP32 MFMA sums within each 256-column chunk, added into FP64
// accumulators at every chunk boundary; the partials are written as doubles
// (the objective pass).
constexpr int RING_F32 = 8;

// TALL (full plans): 8 waves, the two halves stream row tiles 2q and 2q+1 of a
// (tile pair, chunk) unit against one chunk image, halving image traffic per
// byte of S.
template <int KIND, int NT, bool DB, bool PF, bool ACC64, bool TALL>
__global__ __launch_bounds__(TALL ? 512 : 256, TALL ? 1 : 2) void stream_mfma(const void* __restrict__ Sv,
                                                                             const u32x4* __restrict__ img1,
                                                                             const u32x4* __restrict__ img2,
                                                                             void* __restrict__ part, PlanView plan) {
    // tall kernels only stream full plans: with full fixed at compile time the
    // plan-table lookups (global loads with their waits) drop out of the loop
    PlanView p = plan;
    if (TALL) p.full = 1;
    constexpr int K = 16 * NT;
    constexpr int NTHR = TALL ? 512 : 256;
    using IS = ImageShape<KIND, K>;
    constexpr int NV = IS::NV;
    constexpr int CPT = NV / NTHR;                         // image vectors per thread
    static_assert(NV % NTHR == 0, "image vectors must split evenly over the threads");
    constexpr bool SPLIT = !DB;                            // single buffer, refilled in parts
    constexpr int QP = 4;                                  // parts per image
    constexpr int NSV = NV / ((KIND == 0 ? 1 : 3) * NT);   // vectors per (plane, 16-column) block
    constexpr int HSV = NSV / QP;                          // ... in one part of its sub-steps
    constexpr int CPH = CPT / QP;                          // image vectors per thread and part
    static_assert(!SPLIT || (CPT % QP == 0 && NSV % QP == 0), "image parts must split evenly");
    constexpr int NS = KIND == 0 ? 16 : (KIND == 1 ? 8 : 4);
    constexpr int EB = KIND == 0 ? 4 : (KIND == 1 ? 2 : 1);
    // S prefetch ring and distance (sub-steps): deeper for FP32 S, whose sub-steps
    // are the slowest, to keep more bytes in flight per wave
    constexpr int RING = (KIND <= 1 && NT <= 2 && !ACC64) ? RING_F32 : 4, D = RING - 1;
    static_assert(NS % RING == 0, "ring must divide the sub-steps of a unit");
    static_assert(!SPLIT || NS % QP == 0, "image parts must hold whole sub-steps");
    __shared__ u32x4 lds[(DB ? 2 : 1) * NV];
    int64_t U; int32_t na;
    plan_bounds(p, U, na);
    if (U == 0) return;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w = blockIdx.x;
    if (w >= Pe) return;
    const int64_t u0 = wg_start(w, U, Pe);
    const int64_t u1 = wg_start(w + 1, U, Pe);
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) & 3;
    const int half = TALL ? (int)(threadIdx.x >> 8) : 0;   // tile of the pair (tall)
    const int lr = lane & 15, lg = lane >> 4;
    const int tid = threadIdx.x;

    // this wave's contiguous run of a unit's tile, in 16-byte vectors, plus the
    // lane (tall: the odd last pair has no second tile; that half re-reads the
    // first tile and writes nothing)
    auto s_run = [&](int32_t aa, int32_t ch) -> const u32x4* {
        const int64_t tile = TALL ? min((int64_t)2 * aa + half, (int64_t)p.n_tiles - 1) : (int64_t)tile_of(p, aa);
        return (const u32x4*)((const uint8_t*)Sv + ((int64_t)tile * p.n_chunks + ch) * TILE_ELEMS * EB +
                              (int64_t)wv * (TILE_ELEMS * EB / 4)) + lane;
    };
    auto image = [&](int32_t ch, float wt) -> const u32x4* {
        return (wt > 1.5f ? img2 : img1) + (int64_t)ch * NV;
    };

    int32_t a = find_active(p, u0, na);
    int32_t chunk;
    float wt;
    unit_decode(p, u0, a, chunk, wt);
    {
        const u32x4* src = image(chunk, wt);
        for (int i = tid; i < NV; i += NTHR) lds[i] = src[i];
    }
    const u32x4* sp = s_run(a, chunk);
    u32x4 ring[RING][4];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) ring[d][rg] = __builtin_nontemporal_load(sp + (d * 4 + rg) * 64);
    __syncthreads();

    floatx4 acc[4][NT];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[rg][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    double acc64[ACC64 ? 4 : 1][ACC64 ? NT : 1][ACC64 ? 4 : 1];
    if (ACC64) {
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[ACC64 ? rg : 0][ACC64 ? nt : 0][ACC64 ? v : 0] = 0.0;
    }

    // vector index of the j-th vector of this thread's share of image part r
    auto part_index = [&](int j, int r) -> int {
        const int q = tid + NTHR * j;
        return (q / HSV) * NSV + r * HSV + q % HSV;
    };
    u32x4 hreg[SPLIT ? CPH : (PF ? CPT : 1)];
    int32_t a_next = a;
    for (int64_t u = u0; u < u1; ++u) {
        const int cur = DB ? (int)((u - u0) & 1) : 0;
        const bool more = u + 1 < u1;
        int32_t chunk_n = chunk;
        float wt_n = 1.0f;
        const u32x4* sp_n = sp;
        if (more) {
            unit_decode(p, u + 1, a_next, chunk_n, wt_n);
            sp_n = s_run(a_next, chunk_n);
        }
        // Every load below is issued whether or not a next unit exists (on the
        // last unit they re-read this unit's own image and S run, in bounds and
        // unused): loads under a branch would leave the compiler's wait counts
        // at the joins of the unrolled loop set for the path without them,
        // draining the S prefetch ring near every unit boundary.
        const u32x4* src_n = image(chunk_n, wt_n);
        if (SPLIT) {
#pragma unroll
            for (int j = 0; j < CPH; ++j) hreg[j] = src_n[part_index(j, 0)];
        } else if (PF) {
#pragma unroll
            for (int i = 0; i < CPT; ++i) hreg[i] = src_n[tid + NTHR * i];
        }
        const u32x4* hb = lds + cur * NV;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (SPLIT && s > 0 && s % (NS / QP) == 0) {
                // all waves are done with part r - 1 of the current image, and
                // the last part written at the previous unit's end is visible;
                // on the last unit the write lands in a consumed part, unread
                __syncthreads();
                const int r = s / (NS / QP);
#pragma unroll
                for (int j = 0; j < CPH; ++j) {
                    lds[part_index(j, r - 1)] = hreg[j];
                    hreg[j] = src_n[part_index(j, r)];
                }
            }
            // keep D sub-steps of S in flight, crossing into the next unit
            const int sd = s + D;
            if (sd < NS) {
#pragma unroll
                for (int rg = 0; rg < 4; ++rg)
                    ring[sd % RING][rg] = __builtin_nontemporal_load(sp + (sd * 4 + rg) * 64);
            } else {
#pragma unroll
                for (int rg = 0; rg < 4; ++rg)
                    ring[sd % RING][rg] = __builtin_nontemporal_load(sp_n + ((sd - NS) * 4 + rg) * 64);
            }
            // keep the loads here: the scheduler would otherwise sink them
            // towards their use and shorten the prefetch distance
            __builtin_amdgcn_sched_barrier(0);
            if (KIND == 0) {
                floatx4 bv[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    bv[nt] = __builtin_bit_cast(floatx4, hb[((nt * 16 + s) * 4 + lg) * 16 + lr]);
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const floatx4 av = __builtin_bit_cast(floatx4, ring[s % RING][rg]);
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[rg][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m], bv[nt][m], acc[rg][nt], 0, 0, 0);
                    }
            } else {
#pragma unroll
                for (int h = 0; h < (KIND == 2 ? 2 : 1); ++h) {
                    bf16x8 av[4];
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const u32x4 r = ring[s % RING][rg];
                        if (KIND == 2) {
                            const uint32_t w0 = h ? r[2] : r[0];
                            const uint32_t w1 = h ? r[3] : r[1];
                            bf16x2 q0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, false);
                            bf16x2 q1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, true);
                            bf16x2 q2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, false);
                            bf16x2 q3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, true);
                            av[rg] = bf16x8{q0[0], q0[1], q1[0], q1[1], q2[0], q2[1], q3[0], q3[1]};
                        } else {
                            av[rg] = __builtin_bit_cast(bf16x8, r);
                        }
                    }
#pragma unroll
                    for (int pl = 0; pl < 3; ++pl) {
                        bf16x8 bv[NT];
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            const int v16 = KIND == 2 ? ((((nt * 4 + s) * 2 + h) * 4 + lg) * 16 + lr)
                                                      : (((nt * 8 + s) * 4 + lg) * 16 + lr);
                            bv[nt] = __builtin_bit_cast(bf16x8, hb[pl * (IS::PLANE / 8) + v16]);
                        }
#pragma unroll
                        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                acc[rg][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rg], bv[nt], acc[rg][nt],
                                                                                      0, 0, 0);
                    }
                }
            }
        }
        if (ACC64) {
#pragma unroll
            for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[ACC64 ? rg : 0][ACC64 ? nt : 0][ACC64 ? v : 0] += (double)acc[rg][nt][v];
                    acc[rg][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
        }
        // end of this tile's run: write the partial and start the next tile
        if (!more || a_next != a) {
            const int64_t slot = TALL ? 2 * (w + a) + half : (w + a);
            const bool store = !TALL || 2 * (int64_t)a + half < p.n_tiles;
#pragma unroll
            for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (!store) continue;
                        const int64_t o = slot * (int64_t)TR * K + (64 * wv + 16 * rg + 4 * lg + v) * K + 16 * nt + lr;
                        if (ACC64) {
                            ((double*)part)[o] = acc64[ACC64 ? rg : 0][ACC64 ? nt : 0][ACC64 ? v : 0];
                            acc64[ACC64 ? rg : 0][ACC64 ? nt : 0][ACC64 ? v : 0] = 0.0;
                        } else {
                            ((float*)part)[o] = acc[rg][nt][v];
                        }
                    }
                    acc[rg][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
        }
        if (more && SPLIT) {
            // all waves are done with the last part; the other parts of the
            // next image are visible now, the last one becomes visible at the
            // next unit's first part barrier
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CPH; ++j) lds[part_index(j, QP - 1)] = hreg[j];
            a = a_next;
            chunk = chunk_n;
            sp = sp_n;
        } else if (more) {
            u32x4* dstb = lds + (cur ^ 1) * NV;
            if (PF) {
#pragma unroll
                for (int i = 0; i < CPT; ++i) dstb[tid + NTHR * i] = hreg[i];
            } else {
                const u32x4* src = image(chunk_n, wt_n);
                for (int i = tid; i < NV; i += NTHR) dstb[i] = src[i];
            }
            __syncthreads();
            a = a_next;
            chunk = chunk_n;
            sp = sp_n;
        }
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

// LDS per work-group (image buffers): FP32 k=16/32 double-buffered (32/64 KB),
// k=64 single (64 KB); BF16/FP8 keep three bf16 planes: k=16 double (48 KB),
// k=32 single (48 KB), k=64 single (96 KB, one work-group per CU).
// Tall kernels (one 8-wave work-group per CU) double-buffer the images up to
// k = 32 (FP32 64 KB, BF16 / FP8 96 KB) and FP32 at k = 64 (128 KB); BF16 / FP8
// at k = 64 keep one 96 KB image.
template <int KIND>
static void launch_mfma_kind(const void* S, const u32x4* img1, const u32x4* img2, void* part, int64_t k,
                             const PlanView& p, hipStream_t stream) {
    dim3 grid(p.P);
    if (p.tall) {
        dim3 block(512);
        if (k == 16) hipLaunchKernelGGL((stream_mfma<KIND, 1, true, true, false, true>), grid, block, 0, stream, S, img1, img2, part, p);
        else if (k == 32) hipLaunchKernelGGL((stream_mfma<KIND, 2, true, true, false, true>), grid, block, 0, stream, S, img1, img2, part, p);
        else hipLaunchKernelGGL((stream_mfma<KIND, 4, KIND == 0, false, false, true>), grid, block, 0, stream, S, img1, img2, part, p);
        return;
    }
    dim3 block(256);
    if (k == 16) hipLaunchKernelGGL((stream_mfma<KIND, 1, true, true, false, false>), grid, block, 0, stream, S, img1, img2, part, p);
    else if (k == 32) hipLaunchKernelGGL((stream_mfma<KIND, 2, KIND == 0, true, false, false>), grid, block, 0, stream, S, img1, img2, part, p);
    else hipLaunchKernelGGL((stream_mfma<KIND, 4, false, false, false, false>), grid, block, 0, stream, S, img1, img2, part, p);
}

int stream_tall_supported(int32_t stype, int h_f64, int64_t k) {
    return stream_uses_mfma(stype, h_f64, 0, k);
}

template <int KIND>
static void launch_mfma_kind_acc64(const void* S, const u32x4* img, void* part, int64_t k, const PlanView& p,
                                   hipStream_t stream) {
    dim3 grid(p.P), block(256);
    if (k == 16) hipLaunchKernelGGL((stream_mfma<KIND, 1, true, false, true, false>), grid, block, 0, stream, S, img, img, part, p);
    else hipLaunchKernelGGL((stream_mfma<KIND, 2, KIND == 0, false, true, false>), grid, block, 0, stream, S, img, img, part, p);
}

int stream_acc64_supported(int32_t stype, int64_t k) {
    return (stype == SYMNMF_S_FP32 || stype == SYMNMF_S_BF16 || stype == SYMNMF_S_FP8) && (k == 16 || k == 32);
}

hipError_t launch_stream_acc64(const void* S, int32_t stype, int64_t k, const void* img, double* part,
                               const PlanView& p, hipStream_t stream) {
    if (!stream_acc64_supported(stype, k) || !img || p.tall) return hipErrorInvalidValue;   // 4-wave kernel only
    const u32x4* i1 = (const u32x4*)img;
    if (stype == SYMNMF_S_FP32) launch_mfma_kind_acc64<0>(S, i1, part, k, p, stream);
    else if (stype == SYMNMF_S_BF16) launch_mfma_kind_acc64<1>(S, i1, part, k, p, stream);
    else launch_mfma_kind_acc64<2>(S, i1, part, k, p, stream);
    return hipGetLastError();
}

int stream_wgs_per_cu(int32_t stype, int64_t k) {
    if ((stype == SYMNMF_S_BF16 || stype == SYMNMF_S_FP8) && k == 64) return 1;
    return 2;
}

hipError_t launch_stream(const void* S, int32_t stype, int64_t ld, const void* H, int h_f64, int64_t k,
                         void* part, int acc_f64, const PlanView& p, hipStream_t stream, const void* img1,
                         const void* img2) {
    if (k < 1 || k > KMAX) return hipErrorInvalidValue;
    if (stream_uses_mfma(stype, h_f64, acc_f64, k)) {
        if (!img1) return hipErrorInvalidValue;
        const u32x4* i1 = (const u32x4*)img1;
        const u32x4* i2 = (const u32x4*)(img2 ? img2 : img1);
        float* pf = (float*)part;
        if (stype == SYMNMF_S_FP32) launch_mfma_kind<0>(S, i1, i2, pf, k, p, stream);
        else if (stype == SYMNMF_S_BF16) launch_mfma_kind<1>(S, i1, i2, pf, k, p, stream);
        else if (stype == SYMNMF_S_FP8) launch_mfma_kind<2>(S, i1, i2, pf, k, p, stream);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    switch (stype) {
        case SYMNMF_S_FP32: return launch_generic_s<float>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_BF16: return launch_generic_s<uint16_t>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_FP8: return launch_generic_s<uint8_t>(S, ld, H, h_f64, k, part, acc_f64, p, stream);
        case SYMNMF_S_FP64:
            if (!h_f64) return hipErrorInvalidValue;
            if ((k == 16 || k == 32) && std::getenv("SYMNMF_F64_GENERIC") == nullptr) {
                dim3 grid(p.P), block(256);
                if (k == 16)
                    hipLaunchKernelGGL((stream_f64_mfma<1>), grid, block, 0, stream, (const double*)S, ld,
                                       (const double*)H, (double*)part, p);
                else
                    hipLaunchKernelGGL((stream_f64_mfma<2>), grid, block, 0, stream, (const double*)S, ld,
                                       (const double*)H, (double*)part, p);
                return hipGetLastError();
            }
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

// Plain grid-stride 16-byte copy of `bytes` (a multiple of 16): a kernel of
// known traffic for calibrating hardware byte counters.
__global__ __launch_bounds__(256) void copy_probe_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                         int64_t n16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = __builtin_nontemporal_load(src + i);
}

// Plain read of ``bytes`` (a multiple of 16): grid-stride nontemporal 16-byte
// loads, folded into one word per work-group so the loads stay live.
__global__ __launch_bounds__(256) void read_probe_kernel(const u32x4* __restrict__ src, int64_t count,
                                                         uint32_t* __restrict__ sink) {
    uint32_t acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        const u32x4 v = __builtin_nontemporal_load(src + i);
        acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
    }
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sink[blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}

hipError_t launch_read_probe(const void* src, int64_t bytes, uint32_t* sink, int64_t sink_words,
                             hipStream_t stream) {
    const int64_t blocks = sink_words / 4 < 2048 ? sink_words / 4 : 2048;
    if (blocks < 1 || bytes % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(read_probe_kernel, dim3(blocks), dim3(256), 0, stream, (const u32x4*)src, bytes / 16, sink);
    return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t stream) {
    hipLaunchKernelGGL(copy_probe_kernel, dim3(4096), dim3(256), 0, stream, (const u32x4*)src, (u32x4*)dst, bytes / 16);
    return hipGetLastError();
}

}  // namespace symnmf
