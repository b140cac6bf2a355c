// Learned warm start (an addition to the paper's method): a Gaussian sketch
// Y = S Omega of width 64, canonical per-row coordinates (whitening of Y^T Y
// and successive-projection anchors), an MLP 64 -> 256 -> 256 -> k with
// GELU and a softplus output, and its training with the permutation-invariant
// Gram loss ||A A^T - B B^T||_F^2 and AdamW.  This file holds the kernels; the
// orchestration is in runtime.hip.
#include "common.h"

namespace symnmf {

// Omega_ij = sqrt(-2 ln(1-u)) cos(2 pi v) (Box & Muller 1958), u and v the
// 53-bit uniforms of SplitMix64 outputs 2e and 2e+1 of key seed, e = i*w + j.
__global__ void omega_kernel(uint64_t seed, int64_t n, int64_t rows_alloc, int w, float* __restrict__ out) {
    const int64_t total = rows_alloc * w;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        if (e >= n * w) { out[e] = 0.0f; continue; }
        const double u = (double)(splitmix64(seed, 2 * (uint64_t)e) >> 11) * (1.0 / 9007199254740992.0);
        const double v = (double)(splitmix64(seed, 2 * (uint64_t)e + 1) >> 11) * (1.0 / 9007199254740992.0);
        out[e] = (float)(sqrt(-2.0 * log(1.0 - u)) * cos(6.283185307179586 * v));
    }
}

hipError_t launch_omega(uint64_t seed, int64_t n, int64_t rows_alloc, int w, float* out, hipStream_t stream) {
    int64_t blocks = (rows_alloc * w + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(omega_kernel, dim3(blocks), dim3(256), 0, stream, seed, n, rows_alloc, w, out);
    return hipGetLastError();
}

// Dense S.H rows from the partials of a full pass (FP32 partials), FP8 scale
// and diagonal applied: out (rows x k).
__global__ __launch_bounds__(256) void sh_dense_kernel(const float* __restrict__ part, int64_t rows, int k,
                                                       int32_t n_tiles, int32_t n_chunks, int32_t P,
                                                       const float* __restrict__ H, int64_t row0,
                                                       const float* __restrict__ scale, const float* __restrict__ diag,
                                                       int64_t panel_rows, float* __restrict__ out) {
    const int64_t tile = blockIdx.x;
    const int64_t U = (int64_t)n_tiles * n_chunks;
    const int64_t Pe = U < P ? U : P;
    const int64_t w_lo = wg_owner(tile * n_chunks, U, Pe);
    const int64_t w_hi = wg_owner((tile + 1) * n_chunks - 1, U, Pe);
    for (int f = threadIdx.x; f < TR * k; f += 256) {
        const int r = f / k, c = f - r * k;
        const int64_t prow = tile * TR + r;
        if (prow >= rows) continue;
        float s = 0.0f;
        for (int64_t w = w_lo; w <= w_hi; ++w) s += part[((w + tile) * TR + r) * (int64_t)k + c];
        if (scale) s = s / scale[prow / panel_rows] + diag[prow] * H[(row0 + prow) * k + c];
        out[prow * k + c] = s;
    }
}

hipError_t launch_sh_dense(const float* part, int64_t rows, int64_t rows_pad, int64_t k, int32_t n_chunks, int32_t P,
                           const float* H, int64_t row0, const float* scale, const float* diag, int64_t panel_rows,
                           float* out, hipStream_t stream) {
    hipLaunchKernelGGL(sh_dense_kernel, dim3(rows_pad / TR), dim3(256), 0, stream, part, rows, (int)k,
                       (int32_t)(rows_pad / TR), n_chunks, P, H, row0, scale, diag, panel_rows, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small dense GEMM, FP32 accumulation: C (M x N) = alpha op(A) op(B) + bias,
// then an epilogue.  A: TA = 0 -> M x K row-major, TA = 1 -> K x M.
// B: TB = 0 -> N x K row-major (used transposed), TB = 1 -> K x N.
// B may hold bf16 values (the network weights at inference).  64 x 64 output
// tile, K step 16 staged in LDS; each of the four waves computes a 32 x 32
// quarter as 2 x 2 blocks of v_mfma_f32_16x16x4_f32 (FP32 products and
// accumulation: the bf16 weights are widened exactly).  blockIdx.z splits K
// into ranges of kchunk: with more than one range every range writes its own
// partial C + z M N (no bias, no epilogue) for a fixed-order reduction.
// EPI: 0 none, 1 GELU x Phi(x) (Phi from erfc), 2 softplus.  Z (optional)
// receives the value before the epilogue.
// ---------------------------------------------------------------------------
__device__ inline float normal_cdf_f(float x) { return 0.5f * erfcf(-x * 0.70710678118654752f); }

template <int TA, int TB, typename BT, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(const float* __restrict__ A, const BT* __restrict__ B,
                                                   const float* __restrict__ bias, float* __restrict__ C,
                                                   float* __restrict__ Z, int64_t M, int64_t N, int64_t K,
                                                   int64_t kchunk, float alpha) {
    // row stride 80: the four 16-lane groups of an MFMA operand read (rows kk
    // .. kk + 3) fall on disjoint banks
    __shared__ float As[16][80];
    __shared__ float Bs[16][80];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int rb = 32 * (wv >> 1), cb = 32 * (wv & 1);   // this wave's quarter of the tile
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
    floatx4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = kb; k0 < ke; k0 += 16) {
        __syncthreads();
        for (int f = t; f < 16 * 64; f += 256) {
            const int kr = f >> 6, ir = f & 63;   // index fastest: coalesced for K-major operands
            const int kc = f & 15, ic = f >> 4;   // K fastest: coalesced for row-major operands
            {
                const int64_t m = TA ? m0 + ir : m0 + ic, kx = TA ? k0 + kr : k0 + kc;
                float v = 0.0f;
                if (m < M && kx < ke) v = TA ? A[kx * M + m] : A[m * K + kx];
                if (TA) As[kr][ir] = v; else As[kc][ic] = v;
            }
            {
                const int64_t nn = TB ? n0 + ir : n0 + ic, kx = TB ? k0 + kr : k0 + kc;
                float v = 0.0f;
                if (nn < N && kx < ke) {
                    const int64_t off = TB ? kx * N + nn : nn * K + kx;
                    if constexpr (sizeof(BT) == 2) v = bf16_bits_to_f32(B[off]);
                    else v = B[off];
                }
                if (TB) Bs[kr][ir] = v; else Bs[kc][ic] = v;
            }
        }
        __syncthreads();
        // operand A: lane (i, q) holds A[row i][k = 4 s + q]; operand B: lane
        // (j, q) holds op(B)[k = 4 s + q][column j]
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int kk = 4 * st + lk;
            const float a0 = As[kk][rb + li], a1 = As[kk][rb + 16 + li];
            const float b0 = Bs[kk][cb + li], b1 = Bs[kk][cb + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    const bool split = gridDim.z > 1;
    float* Cz = C + (split ? (int64_t)blockIdx.z * M * N : 0);
    // output: lane (j, q) holds rows 4 q + v, v < 4, of column j of each block
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + rb + 16 * bi + 4 * lk + v, nn = n0 + cb + 16 * bj + li;
            if (m >= M || nn >= N) continue;
            float v_ = alpha * acc[bi][bj][v];
            if (split) { Cz[m * N + nn] = v_; continue; }
            if (bias) v_ += bias[nn];
            if (Z) Z[m * N + nn] = v_;
            if (EPI == 1) v_ = v_ * normal_cdf_f(v_);
            else if (EPI == 2) v_ = fmaxf(v_, 0.0f) + log1pf(expf(-fabsf(v_)));
            Cz[m * N + nn] = v_;
        }
}

// out[e] = sum_z part[z][e] in fixed order
__global__ void sum_split_kernel(const float* __restrict__ part, int splits, int64_t m, float* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int z = 0; z < splits; ++z) s += part[z * m + e];
        out[e] = s;
    }
}

hipError_t launch_gemm(int ta, int tb, int b_bf16, int epi, const float* A, const void* B, const float* bias, float* C,
                       float* Z, int64_t M, int64_t N, int64_t K, float alpha, float* split_ws, int64_t split_ws_floats,
                       hipStream_t stream) {
    if (M < 1 || N < 1 || K < 1) return hipErrorInvalidValue;
    // split K for tall contractions (weight gradients) whose output grid is small
    int64_t splits = 1;
    const int64_t tiles = ((N + 63) / 64) * ((M + 63) / 64);
    if (tiles < 256 && K >= 512 && split_ws) {
        splits = std::min<int64_t>(256 / tiles, K / 256);
        splits = std::min<int64_t>(splits, split_ws_floats / (M * N));
        if (splits < 2 || epi != 0 || bias) splits = 1;
    }
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + 15) / 16 * 16;
    splits = (K + kchunk - 1) / kchunk;
    float* dst = splits > 1 ? split_ws : C;
    dim3 grid((N + 63) / 64, (M + 63) / 64, splits), block(256);
#define G(TA, TB, BT, E)                                                                                       \
    hipLaunchKernelGGL((gemm_kernel<TA, TB, BT, E>), grid, block, 0, stream, A, (const BT*)B, bias, dst, Z, M, N, \
                       K, kchunk, alpha)
    if (b_bf16) {
        if (ta == 0 && tb == 0 && epi == 0) G(0, 0, uint16_t, 0);
        else if (ta == 0 && tb == 0 && epi == 1) G(0, 0, uint16_t, 1);
        else if (ta == 0 && tb == 0 && epi == 2) G(0, 0, uint16_t, 2);
        else return hipErrorInvalidValue;
    } else {
        if (ta == 0 && tb == 0 && epi == 0) G(0, 0, float, 0);
        else if (ta == 0 && tb == 0 && epi == 1) G(0, 0, float, 1);
        else if (ta == 0 && tb == 0 && epi == 2) G(0, 0, float, 2);
        else if (ta == 0 && tb == 1 && epi == 0) G(0, 1, float, 0);
        else if (ta == 1 && tb == 1 && epi == 0) G(1, 1, float, 0);
        else return hipErrorInvalidValue;
    }
#undef G
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t m = M * N;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sum_split_kernel, dim3(blocks), dim3(256), 0, stream, (const float*)split_ws, (int)splits, m, C);
    return hipGetLastError();
}

// dZ = dA * f'(Z): mode 1 GELU' (Phi(z) + z phi(z)), mode 2 softplus' (sigmoid)
__global__ void act_backward_kernel(const float* __restrict__ dA, const float* __restrict__ Zpre, float* __restrict__ dZ,
                                    int64_t m, int mode) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const float z = Zpre[i];
        float d;
        if (mode == 1) d = normal_cdf_f(z) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
        else d = 0.5f * (1.0f + tanhf(0.5f * z));
        dZ[i] = dA[i] * d;
    }
}

hipError_t launch_act_backward(const float* dA, const float* Z, float* dZ, int64_t m, int mode, hipStream_t stream) {
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(act_backward_kernel, dim3(blocks), dim3(256), 0, stream, dA, Z, dZ, m, mode);
    return hipGetLastError();
}

// Residual output A = max(C + z, 0), C the first k columns of the network input
// X (leading dimension ldx): A holds z on entry (rows x k).
__global__ void residual_relu_kernel(const float* __restrict__ X, int64_t ldx, float* __restrict__ A, int64_t rows,
                                     int k) {
    const int64_t m = rows * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k;
        const float v = X[r * ldx + (i - r * k)] + A[i];
        A[i] = v > 0.0f ? v : 0.0f;
    }
}

// dZ = dA [C + z > 0]
__global__ void residual_relu_backward_kernel(const float* __restrict__ dA, const float* __restrict__ X, int64_t ldx,
                                              const float* __restrict__ Z, float* __restrict__ dZ, int64_t rows,
                                              int k) {
    const int64_t m = rows * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k;
        dZ[i] = X[r * ldx + (i - r * k)] + Z[i] > 0.0f ? dA[i] : 0.0f;
    }
}

hipError_t launch_residual_relu(const float* X, int64_t ldx, float* A, int64_t rows, int64_t k, hipStream_t stream) {
    int64_t blocks = (rows * k + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(residual_relu_kernel, dim3(blocks), dim3(256), 0, stream, X, ldx, A, rows, (int)k);
    return hipGetLastError();
}

hipError_t launch_residual_relu_backward(const float* dA, const float* X, int64_t ldx, const float* Z, float* dZ,
                                         int64_t rows, int64_t k, hipStream_t stream) {
    int64_t blocks = (rows * k + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(residual_relu_backward_kernel, dim3(blocks), dim3(256), 0, stream, dA, X, ldx, Z, dZ, rows,
                       (int)k);
    return hipGetLastError();
}

// column sums of an (m x ncol) FP32 matrix (bias gradients), FP64 accumulation
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ X, int64_t m, int ncol, float* __restrict__ out) {
    __shared__ double red[4][64];
    const int lc = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t col = blockIdx.x * 64 + lc;
    double s = 0.0;
    if (col < ncol)
        for (int64_t i = ph; i < m; i += 4) s += (double)X[i * ncol + col];
    red[ph][lc] = s;
    __syncthreads();
    if (ph == 0 && col < ncol) out[col] = (float)(red[0][lc] + red[1][lc] + red[2][lc] + red[3][lc]);
}

hipError_t launch_colsum(const float* X, int64_t m, int64_t ncol, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(colsum_kernel, dim3((ncol + 63) / 64), dim3(256), 0, stream, X, m, (int)ncol, out);
    return hipGetLastError();
}

// AdamW on a flat parameter vector; the first n_decay entries get decoupled
// weight decay.  t = step number (1, 2, ...).
__global__ void adamw_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                             float* __restrict__ V, int64_t m, int64_t n_decay, float lr, float b1, float b2,
                             float eps, float wd, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = G[i];
        const float mi = b1 * Mm[i] + (1.0f - b1) * g;
        const float vi = b2 * V[i] + (1.0f - b2) * g * g;
        Mm[i] = mi;
        V[i] = vi;
        float p = P[i];
        if (i < n_decay) p -= lr * wd * p;
        p -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        P[i] = p;
    }
}

hipError_t launch_adamw(float* P, const float* G, float* M, float* V, int64_t m, int64_t n_decay, float lr, float b1,
                        float b2, float eps, float wd, int64_t t, hipStream_t stream) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(adamw_kernel, dim3(blocks), dim3(256), 0, stream, P, G, M, V, m, n_decay, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t m) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_bits(x[i]);
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t m, hipStream_t stream) {
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks), dim3(256), 0, stream, x, y, m);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Successive projection (Gillis & Vavasis 2014) on the rows of R (m x k, FP64
// working copy): argmax of the residual row norms (lowest index on ties) in
// two passes, then every row is projected off the chosen row's direction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void spa_argmax_blocks(const double* __restrict__ R, int64_t m, int k,
                                                         double* __restrict__ bval, int64_t* __restrict__ bidx) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += R[i * k + c] * R[i * k + c];
        if (s > best) { best = s; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + off];
            const int64_t ia = si[threadIdx.x], ib = si[threadIdx.x + off];
            if (b > a || (b == a && ib < ia)) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { bval[blockIdx.x] = sv[0]; bidx[blockIdx.x] = si[0]; }
}

__global__ void spa_argmax_final(const double* __restrict__ bval, const int64_t* __restrict__ bidx, int nb,
                                 int64_t* __restrict__ pick, int step) {
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int64_t bi = 0;
    for (int b = 0; b < nb; ++b)
        if (bval[b] > best || (bval[b] == best && bidx[b] < bi)) { best = bval[b]; bi = bidx[b]; }
    pick[step] = bi;
}

__global__ __launch_bounds__(256) void spa_project(double* __restrict__ R, int64_t m, int k, const int64_t* __restrict__ pick,
                                                   int step) {
    __shared__ double u[KMAX];
    __shared__ double nrm;
    const int64_t p = pick[step];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += R[p * k + c] * R[p * k + c];
        nrm = sqrt(s);
    }
    __syncthreads();
    if ((int)threadIdx.x < k) u[threadIdx.x] = nrm > 0.0 ? R[p * k + threadIdx.x] / nrm : 0.0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        if (i == p) continue;
        double d = 0.0;
        for (int c = 0; c < k; ++c) d += R[i * k + c] * u[c];
        for (int c = 0; c < k; ++c) R[i * k + c] -= d * u[c];
    }
}

__global__ void spa_zero_row(double* __restrict__ R, int k, const int64_t* __restrict__ pick, int step) {
    const int64_t p = pick[step];
    if ((int)threadIdx.x < k) R[p * k + threadIdx.x] = 0.0;
}

hipError_t launch_spa(double* R, int64_t m, int64_t k, double* bval, int64_t* bidx, int nb, int64_t* pick,
                      hipStream_t stream) {
    for (int s = 0; s < k; ++s) {
        hipLaunchKernelGGL(spa_argmax_blocks, dim3(nb), dim3(256), 0, stream, (const double*)R, m, (int)k, bval, bidx);
        hipLaunchKernelGGL(spa_argmax_final, dim3(1), dim3(64), 0, stream, (const double*)bval, (const int64_t*)bidx, nb, pick, s);
        hipLaunchKernelGGL(spa_project, dim3(nb), dim3(256), 0, stream, R, m, (int)k, (const int64_t*)pick, s);
        hipLaunchKernelGGL(spa_zero_row, dim3(1), dim3(64), 0, stream, R, (int)k, (const int64_t*)pick, s);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 products X^T Y (kx x ky, both <= 64) of two row-major FP32 matrices
// over m rows: 64-row slabs staged through LDS, every thread accumulating 16
// entries of the slab's product; slab partials reduced in slab order.
// ---------------------------------------------------------------------------
constexpr int XTY_ROWS = 64;

__global__ __launch_bounds__(256) void xty_slab_kernel(const float* __restrict__ X, int64_t ldx, int kx,
                                                       const float* __restrict__ Y, int64_t ldy, int ky, int64_t m,
                                                       double* __restrict__ part) {
    __shared__ float xs[XTY_ROWS][KMAX + 1];
    __shared__ float ys[XTY_ROWS][KMAX + 1];
    const int64_t r0 = (int64_t)blockIdx.x * XTY_ROWS;
    for (int f = threadIdx.x; f < XTY_ROWS * KMAX; f += 256) {
        const int r = f / KMAX, c = f - r * KMAX;
        const bool in = r0 + r < m;
        xs[r][c] = (in && c < kx) ? X[(r0 + r) * ldx + c] : 0.0f;
        ys[r][c] = (in && c < ky) ? Y[(r0 + r) * ldy + c] : 0.0f;
    }
    __syncthreads();
    double* dst = part + (int64_t)blockIdx.x * kx * ky;
    for (int e = threadIdx.x; e < kx * ky; e += 256) {
        const int a = e / ky, b = e - a * ky;
        double sum = 0.0;
        for (int r = 0; r < XTY_ROWS; ++r) sum += (double)xs[r][a] * (double)ys[r][b];
        dst[e] = sum;
    }
}

__global__ void sum_slabs_kernel(const double* __restrict__ part, int64_t slabs, int entries, double* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    double s = 0.0;
    for (int64_t b = 0; b < slabs; ++b) s += part[b * entries + e];
    out[e] = s;
}

int64_t xty_work_doubles(int64_t m, int64_t kx, int64_t ky) { return ((m + XTY_ROWS - 1) / XTY_ROWS) * kx * ky; }

hipError_t launch_xty(const float* X, int64_t ldx, int64_t kx, const float* Y, int64_t ldy, int64_t ky, int64_t m,
                      double* work, double* out, hipStream_t stream) {
    if (kx < 1 || ky < 1 || kx > KMAX || ky > KMAX || m < 1) return hipErrorInvalidValue;
    const int64_t slabs = (m + XTY_ROWS - 1) / XTY_ROWS;
    hipLaunchKernelGGL(xty_slab_kernel, dim3(slabs), dim3(256), 0, stream, X, ldx, (int)kx, Y, ldy, (int)ky, m, work);
    const int entries = (int)(kx * ky);
    hipLaunchKernelGGL(sum_slabs_kernel, dim3((entries + 255) / 256), dim3(256), 0, stream, (const double*)work, slabs,
                       entries, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric eigen-decomposition of a w x w FP64 matrix (w <= 64) in one
// work-group: cyclic two-sided Jacobi rotations (Golub & Van Loan, Matrix
// Computations, symmetric Schur decomposition of 2 x 2 blocks) in the
// round-robin parallel order, w/2 disjoint rotations at a time.  Then the k
// largest eigenvalues (descending, lower index first on ties) and
// M = V_k diag(lambda)^-1/2 (w x k).  status[0] = 1 when a selected
// eigenvalue is not positive and finite, 2 when the sweeps do not converge.
// V: w x w FP64 device scratch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void jacobi_topk_kernel(const double* __restrict__ G, int w, int k,
                                                          double* __restrict__ V, double* __restrict__ Mout,
                                                          double* __restrict__ lam_out, int32_t* __restrict__ status) {
    __shared__ double A[KMAX][KMAX + 1];
    __shared__ int order[KMAX];
    __shared__ int done;
    __shared__ double floor_abs;
    __shared__ double cs_s[KMAX / 2], sn_s[KMAX / 2];
    __shared__ int p_s[KMAX / 2], q_s[KMAX / 2];
    const int t = threadIdx.x;
    for (int e = t; e < w * w; e += 256) {
        const int i = e / w, j = e - i * w;
        A[i][j] = 0.5 * (G[i * w + j] + G[j * w + i]);
        V[e] = i == j ? 1.0 : 0.0;
    }
    const int wp = w + (w & 1);    // even player count; index w (odd w) is a bye
    const int half = wp / 2;
    // a pair is rotated when |a_pq| > max(1e-14 sqrt(|a_pp a_qq|), 1e-15 ||G||_F)
    // (the relative criterion of Demmel & Veselic 1992, with an absolute floor
    // so that rounding noise inside a null space of a semidefinite G does not
    // keep the sweeps going); converged after a sweep with no rotation
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < w; ++i)
            for (int j = 0; j < w; ++j) s += A[i][j] * A[i][j];
        floor_abs = 1e-15 * sqrt(s);
    }
    int sweep = 0;
    for (; sweep < 60; ++sweep) {
        __syncthreads();
        if (t == 0) done = 1;
        __syncthreads();
        for (int r = 0; r < wp - 1; ++r) {
            // pair i of round r: (wp-1, r) for i = 0, else ((r+i) mod (wp-1), (r-i) mod (wp-1));
            // every rotation is computed from the block before any row is changed
            if (t < half) {
                int p, q;
                if (t == 0) { p = wp - 1; q = r; }
                else { p = (r + t) % (wp - 1); q = (r - t + (wp - 1)) % (wp - 1); }
                if (p > q) { const int tmp = p; p = q; q = tmp; }
                double c = 1.0, sn = 0.0;
                if (q < w) {
                    const double apq = A[p][q];
                    if (fabs(apq) > fmax(1e-14 * sqrt(fabs(A[p][p] * A[q][q])), floor_abs)) {
                        done = 0;
                        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * c;
                    }
                }
                cs_s[t] = c; sn_s[t] = sn; p_s[t] = p; q_s[t] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int f = t; f < half * w; f += 256) {
                const int pi = f / w, col = f - pi * w;
                const int p = p_s[pi], q = q_s[pi];
                if (q >= w || sn_s[pi] == 0.0) continue;
                const double c = cs_s[pi], sn = sn_s[pi];
                const double ap = A[p][col], aq = A[q][col];
                A[p][col] = c * ap - sn * aq;
                A[q][col] = sn * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int f = t; f < half * w; f += 256) {
                const int pi = f / w, row = f - pi * w;
                const int p = p_s[pi], q = q_s[pi];
                if (q >= w || sn_s[pi] == 0.0) continue;
                const double c = cs_s[pi], sn = sn_s[pi];
                const double ap = A[row][p], aq = A[row][q];
                A[row][p] = c * ap - sn * aq;
                A[row][q] = sn * ap + c * aq;
                const double vp = V[row * w + p], vq = V[row * w + q];
                V[row * w + p] = c * vp - sn * vq;
                V[row * w + q] = sn * vp + c * vq;
            }
            __syncthreads();
        }
        if (done) break;
    }
    __syncthreads();
    if (t == 0) {
        int32_t st = sweep >= 60 ? 2 : 0;
        bool used[KMAX];
        for (int i = 0; i < w; ++i) used[i] = false;
        for (int c = 0; c < k; ++c) {
            int best = -1;
            for (int i = 0; i < w; ++i)
                if (!used[i] && (best < 0 || A[i][i] > A[best][best])) best = i;
            used[best] = true;
            order[c] = best;
            const double l = A[best][best];
            lam_out[c] = l;
            if (!(l > 0.0) || !isfinite(l)) st = 1;
        }
        status[0] = st;
    }
    __syncthreads();
    for (int e = t; e < w * k; e += 256) {
        const int i = e / k, c = e - i * k;
        const double l = A[order[c]][order[c]];
        Mout[e] = l > 0.0 ? V[i * w + order[c]] / sqrt(l) : 0.0;
    }
}

hipError_t launch_jacobi_topk(const double* G, int64_t w, int64_t k, double* V, double* M, double* lam,
                              int32_t* status, hipStream_t stream) {
    if (w < 1 || w > KMAX || k < 1 || k > w) return hipErrorInvalidValue;
    hipLaunchKernelGGL(jacobi_topk_kernel, dim3(1), dim3(256), 0, stream, G, (int)w, (int)k, V, M, lam, status);
    return hipGetLastError();
}

// out (m x ldo) = Y (m x w, FP32) W (w x k, FP64): FP64 sums; OUT = double
// writes k columns (ldo = k), OUT = float writes ldo columns, zero past k.
template <typename OUT>
__global__ __launch_bounds__(256) void project_rows_kernel(const float* __restrict__ Y, int64_t m, int w,
                                                           const double* __restrict__ W, int k, int ldo,
                                                           OUT* __restrict__ out) {
    __shared__ double Ws[KMAX * KMAX];
    for (int e = threadIdx.x; e < w * k; e += 256) Ws[e] = W[e];
    __syncthreads();
    const int64_t total = m * ldo;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / ldo;
        const int c = (int)(e - i * ldo);
        double s = 0.0;
        if (c < k)
            for (int l = 0; l < w; ++l) s += (double)Y[i * w + l] * Ws[l * k + c];
        out[e] = (OUT)s;
    }
}

hipError_t launch_project_rows(const float* Y, int64_t m, int64_t w, const double* W, int64_t k, int64_t ldo,
                               int out_f64, void* out, hipStream_t stream) {
    if (w > KMAX || k > KMAX || ldo < k) return hipErrorInvalidValue;
    int64_t blocks = (m * ldo + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (out_f64)
        hipLaunchKernelGGL(project_rows_kernel<double>, dim3(blocks), dim3(256), 0, stream, Y, m, (int)w, W, (int)k,
                           (int)ldo, (double*)out);
    else
        hipLaunchKernelGGL(project_rows_kernel<float>, dim3(blocks), dim3(256), 0, stream, Y, m, (int)w, W, (int)k,
                           (int)ldo, (float*)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Anchor basis in one work-group: A = Y[anchors] M (k x k, FP64), LU with
// partial pivoting, then W = M A^-1 (w x k) by solving A^T w_l = m_l for every
// row l of M.  C = Y W then equals Z A^-1 with Z = Y M.  status[0] = 0, or 3
// when a pivot is below 1e-13 times the largest entry of A.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void anchor_solve_kernel(const float* __restrict__ Y, int w,
                                                           const double* __restrict__ M, int k,
                                                           const int64_t* __restrict__ anchors, double* __restrict__ W,
                                                           int32_t* __restrict__ status) {
    __shared__ double LU[KMAX][KMAX + 1];
    __shared__ int perm[KMAX];
    __shared__ double amax;
    __shared__ int piv, singular;
    const int t = threadIdx.x;
    if (t == 0) singular = 0;
    for (int e = t; e < k * k; e += 256) {
        const int j = e / k, c = e - j * k;
        const int64_t row = anchors[j];
        double s = 0.0;
        for (int l = 0; l < w; ++l) s += (double)Y[row * w + l] * M[l * k + c];
        LU[j][c] = s;
    }
    if (t < k) perm[t] = t;
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int j = 0; j < k; ++j)
            for (int c = 0; c < k; ++c) m = fmax(m, fabs(LU[j][c]));
        amax = m;
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            int p = j;
            for (int i = j + 1; i < k; ++i)
                if (fabs(LU[i][j]) > fabs(LU[p][j])) p = i;
            piv = p;
            if (!(fabs(LU[p][j]) > 1e-13 * amax)) singular = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != j) {
            for (int c = t; c < k; c += 256) {
                const double tmp = LU[j][c];
                LU[j][c] = LU[p][c];
                LU[p][c] = tmp;
            }
            if (t == 0) { const int tp = perm[j]; perm[j] = perm[p]; perm[p] = tp; }
        }
        __syncthreads();
        const double d = LU[j][j];
        for (int i = j + 1 + t; i < k; i += 256) LU[i][j] = d != 0.0 ? LU[i][j] / d : 0.0;
        __syncthreads();
        for (int e = t; e < (k - j - 1) * (k - j - 1); e += 256) {
            const int i = j + 1 + e / (k - j - 1), c = j + 1 + e % (k - j - 1);
            LU[i][c] -= LU[i][j] * LU[j][c];
        }
        __syncthreads();
    }
    // P A = L U  =>  A^T = U^T L^T P.  For row l of M: U^T y = m (forward),
    // L^T x = y (backward, unit diagonal), w = P^T x, i.e. w[perm[i]] = x[i].
    for (int l = t; l < w; l += 256) {
        double x[KMAX];
        for (int i = 0; i < k; ++i) {
            double s = M[l * k + i];
            for (int j = 0; j < i; ++j) s -= LU[j][i] * x[j];
            x[i] = LU[i][i] != 0.0 ? s / LU[i][i] : 0.0;
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = x[i];
            for (int j = i + 1; j < k; ++j) s -= LU[j][i] * x[j];
            x[i] = s;
        }
        for (int i = 0; i < k; ++i) W[l * k + perm[i]] = x[i];
    }
    if (t == 0) status[0] = singular ? 3 : 0;
}

hipError_t launch_anchor_solve(const float* Y, int64_t w, const double* M, int64_t k, const int64_t* anchors,
                               double* W, int32_t* status, hipStream_t stream) {
    if (w > KMAX || k > KMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(anchor_solve_kernel, dim3(1), dim3(256), 0, stream, Y, (int)w, M, (int)k, anchors, W, status);
    return hipGetLastError();
}

// Gram-loss gradient rows: dA_ic = ca sum_j A_ij AtA_jc - cb sum_j B_ij AtB_cj,
// the per-row form of ca A (A^T A) - cb B (B^T A) (both Gram losses have it).
__global__ __launch_bounds__(256) void gram_loss_grad_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                             const double* __restrict__ AtA,
                                                             const double* __restrict__ AtB, int k, int64_t m,
                                                             float ca, float cb, float* __restrict__ dA) {
    __shared__ float P[KMAX * KMAX];
    __shared__ float Q[KMAX * KMAX];
    for (int e = threadIdx.x; e < k * k; e += 256) {
        P[e] = (float)AtA[e];
        const int c = e / k, j = e - c * k;
        Q[j * k + c] = (float)AtB[c * k + j];   // Q[j][c] = (A^T B)_cj
    }
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < m * k; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / k;
        const int c = (int)(e - i * k);
        float sa = 0.0f, sb = 0.0f;
        for (int j = 0; j < k; ++j) {
            sa += A[i * k + j] * P[j * k + c];
            sb += B[i * k + j] * Q[j * k + c];
        }
        dA[e] = ca * sa - cb * sb;
    }
}

hipError_t launch_gram_loss_grad(const float* A, const float* B, const double* AtA, const double* AtB, int64_t k,
                                 int64_t m, float ca, float cb, float* dA, hipStream_t stream) {
    if (k > KMAX) return hipErrorInvalidValue;
    int64_t blocks = (m * k + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(gram_loss_grad_kernel, dim3(blocks), dim3(256), 0, stream, A, B, AtA, AtB, (int)k, m, ca, cb, dA);
    return hipGetLastError();
}

// out (m x k) = max(X[:, :k], 0) for X (m x w)
__global__ void clip_cols_kernel(const float* __restrict__ X, int64_t m, int w, int k, float* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * k; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / k;
        const int c = (int)(e - i * k);
        out[e] = fmaxf(X[i * w + c], 0.0f);
    }
}

hipError_t launch_clip_cols(const float* X, int64_t m, int64_t w, int64_t k, float* out, hipStream_t stream) {
    int64_t blocks = (m * k + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(clip_cols_kernel, dim3(blocks), dim3(256), 0, stream, X, m, (int)w, (int)k, out);
    return hipGetLastError();
}

__global__ void scale_kernel(float* __restrict__ x, int64_t m, float a) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= a;
}

hipError_t launch_scale(float* x, int64_t m, float a, hipStream_t stream) {
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(scale_kernel, dim3(blocks), dim3(256), 0, stream, x, m, a);
    return hipGetLastError();
}

// ||M_A^T (A^T B) M_B||_F^2 for k x k FP64 matrices (one work-group); with
// M_X^T (X^T X) M_X = I this is ||Q_A^T Q_B||_F^2 of orthonormal bases of the
// column spans of A and B.
__global__ __launch_bounds__(256) void span_overlap_kernel(const double* __restrict__ MA,
                                                           const double* __restrict__ AtB,
                                                           const double* __restrict__ MB, int k,
                                                           double* __restrict__ out) {
    __shared__ double T[KMAX * KMAX];
    __shared__ double red[4];
    for (int e = threadIdx.x; e < k * k; e += 256) {
        const int i = e / k, j = e - i * k;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s += AtB[i * k + l] * MB[l * k + j];
        T[e] = s;   // (A^T B M_B)_ij
    }
    __syncthreads();
    double acc = 0.0;
    for (int e = threadIdx.x; e < k * k; e += 256) {
        const int i = e / k, j = e - i * k;
        double q = 0.0;
        for (int l = 0; l < k; ++l) q += MA[l * k + i] * T[l * k + j];
        acc += q * q;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_span_overlap(const double* MA, const double* AtB, const double* MB, int64_t k, double* out,
                               hipStream_t stream) {
    if (k < 1 || k > KMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(span_overlap_kernel, dim3(1), dim3(256), 0, stream, MA, AtB, MB, (int)k, out);
    return hipGetLastError();
}

}  // namespace symnmf
