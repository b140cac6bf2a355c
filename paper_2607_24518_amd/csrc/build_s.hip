// S construction on the device (paper appendix "Benchmark Data Generation",
// correlation and TPDM construction; section "Empirical Estimation").
//
//   |corr| : column means and centred norms in FP64, Z = (X - mean) / norm
//            (so Z^T Z is the Pearson correlation), S = |Z^T Z|, S_ii = 1.
//   TPDM   : per column, ranks of the (negated, for the lower tail) samples
//            with ties to the lower sample; Pareto(2) margins
//            x = (1 - r/(T+1))^-1/2; FP64 radial norm of every sample; the
//            floor(qT) largest norms kept (ties to the lower sample); angular
//            rows w_t = x_t / ||x_t||; columns scaled so that the Gram has unit
//            diagonal, i.e. S = D^-1/2 (Omega^T Omega) D^-1/2; S_ii = 1.
// Both finish with the same MFMA SYRK (v_mfma_f32_16x16x4_f32, FP32
// accumulation) whose epilogue takes |.|, sets the unit diagonal, rounds to
// the storage type and accumulates FP64 sums of S and S^2.
#include "common.h"

namespace symnmf {

// ---------------------------------------------------------------------------
// |corr|: standardised columns
// ---------------------------------------------------------------------------
template <typename ZT>
__global__ __launch_bounds__(256) void standardise_kernel(const float* __restrict__ X, int64_t T, int64_t n,
                                                          ZT* __restrict__ Z, int64_t ldz,
                                                          int32_t* __restrict__ bad) {
    __shared__ double red[4][64];
    const int lc = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t col = blockIdx.x * 64 + lc;
    const bool valid = col < n;
    double s = 0.0;
    if (valid)
        for (int64_t t = ph; t < T; t += 4) s += (double)X[t * n + col];
    red[ph][lc] = s;
    __syncthreads();
    const double mean = (red[0][lc] + red[1][lc] + red[2][lc] + red[3][lc]) / (double)T;
    __syncthreads();
    double ss = 0.0;
    if (valid)
        for (int64_t t = ph; t < T; t += 4) {
            const double d = (double)X[t * n + col] - mean;
            ss += d * d;
        }
    red[ph][lc] = ss;
    __syncthreads();
    const double c = sqrt(red[0][lc] + red[1][lc] + red[2][lc] + red[3][lc]);
    if (!valid) return;
    if (!isfinite(c)) {                      // a NaN or infinity in the column
        if (ph == 0) atomicOr(bad, BAD_NONFINITE);
        return;
    }
    if (!(c > 0.0)) {
        if (ph == 0) atomicAdd(bad, 1);
        return;
    }
    for (int64_t t = ph; t < T; t += 4) Z[t * ldz + col] = (ZT)(((double)X[t * n + col] - mean) / c);
}

// Raises BAD_NONFINITE in *flag when any of the count values is NaN or
// infinite and, when sign != 0, BAD_NEGATIVE when some sign * X[i] < 0.
__global__ __launch_bounds__(256) void check_input_kernel(const float* __restrict__ X, int64_t count, float sign,
                                                          int32_t* __restrict__ flag) {
    bool nonfinite = false, negative = false;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        const float v = X[i];
        nonfinite |= !isfinite(v);
        negative |= sign * v < 0.0f;
    }
    if (nonfinite) atomicOr(flag, BAD_NONFINITE);
    if (negative) atomicOr(flag, BAD_NEGATIVE);
}

hipError_t launch_check_input(const float* X, int64_t count, float sign, int32_t* flag, hipStream_t stream) {
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    if (blocks > 0) hipLaunchKernelGGL(check_input_kernel, dim3(blocks), dim3(256), 0, stream, X, count, sign, flag);
    return hipGetLastError();
}

hipError_t launch_standardise(const float* X, int64_t T, int64_t n, void* Z, int z_f64, int64_t ldz, int32_t* bad,
                              hipStream_t stream) {
    if (z_f64)
        hipLaunchKernelGGL(standardise_kernel<double>, dim3((n + 63) / 64), dim3(256), 0, stream, X, T, n, (double*)Z, ldz, bad);
    else
        hipLaunchKernelGGL(standardise_kernel<float>, dim3((n + 63) / 64), dim3(256), 0, stream, X, T, n, (float*)Z, ldz, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// TPDM pieces
// ---------------------------------------------------------------------------
// dst (cols x rows) = sign * src (rows x cols)^T, 64 x 64 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, int64_t rows, int64_t cols,
                                                        T* __restrict__ dst, T sign) {
    __shared__ T tile[64][65];
    const int64_t r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = src[r * cols + c] * sign;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) dst[c * rows + r] = tile[tx][i];
    }
}

// Unsigned key ordered like the float value; -0.0 and +0.0 get the same key
// (they are equal values and tie like any other equal pair).
__device__ inline uint32_t sortable_key(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7fffffffu) == 0) u = 0;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One work-group per column: bitonic sort of the column's keys in LDS, then
// rank r_t = 1 + #{keys < key_t} + #{t' < t : key_t' = key_t}.
constexpr int RANK_MAX_T = 32768;
__global__ __launch_bounds__(1024) void rank_kernel(const float* __restrict__ Xt, int64_t T, int32_t* __restrict__ R) {
    extern __shared__ uint32_t keys[];
    const int64_t col = blockIdx.x;
    const float* x = Xt + col * T;
    int P2 = 1;
    while (P2 < T) P2 <<= 1;
    for (int i = threadIdx.x; i < P2; i += blockDim.x) keys[i] = i < T ? sortable_key(x[i]) : 0xffffffffu;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (P2 >> 1); i += blockDim.x) {
                const int lo = 2 * stride * (i / stride) + (i % stride);
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint32_t a = keys[lo], b = keys[hi];
                if ((a > b) == asc) { keys[lo] = b; keys[hi] = a; }
            }
            __syncthreads();
        }
    }
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
        const uint32_t k = sortable_key(x[t]);
        int lo = 0, hi = (int)T;                 // first index with keys[idx] >= k
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (keys[mid] < k) lo = mid + 1; else hi = mid;
        }
        int32_t rank = lo + 1;
        const bool tie = (lo + 1 < T && keys[lo + 1] == k);
        if (tie)
            for (int64_t s = 0; s < t; ++s) rank += (sortable_key(x[s]) == k) ? 1 : 0;
        R[col * T + t] = rank;
    }
}

// Radial norm of sample t from its ranks (row t of Rt, n values), FP64.
__global__ __launch_bounds__(256) void norms_kernel(const int32_t* __restrict__ Rt, int64_t T, int64_t n,
                                                    double* __restrict__ norms) {
    __shared__ double red[4];
    const int64_t t = blockIdx.x;
    const double Tp1 = (double)T + 1.0;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double x = pow(1.0 - (double)Rt[t * n + j] / Tp1, -0.5);
        s += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) norms[t] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// Indices of the n_exc largest norms in increasing t (ties to the lower t),
// given v* = the n_exc-th largest norm.
__global__ void compact_kernel(const double* __restrict__ norms, int64_t T, int64_t n_exc,
                               const double* __restrict__ vstar, int32_t* __restrict__ idx) {
    if (threadIdx.x != 0) return;
    const double v = vstar[0];
    int64_t greater = 0;
    for (int64_t t = 0; t < T; ++t) greater += norms[t] > v ? 1 : 0;
    int64_t equal_left = n_exc - greater, a = 0;
    for (int64_t t = 0; t < T && a < n_exc; ++t) {
        if (norms[t] > v) idx[a++] = (int32_t)t;
        else if (norms[t] == v && equal_left > 0) { idx[a++] = (int32_t)t; --equal_left; }
    }
}

// Omega_aj = x(R[t_a][j]) / ||x_{t_a}||, then column j scaled to unit norm.
template <typename ZT>
__global__ __launch_bounds__(256) void omega_kernel(const int32_t* __restrict__ Rt, int64_t T, int64_t n,
                                                    const double* __restrict__ norms,
                                                    const int32_t* __restrict__ idx, int64_t n_exc,
                                                    ZT* __restrict__ Om, int64_t ldz) {
    __shared__ double red[4][64];
    const int lc = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t col = blockIdx.x * 64 + lc;
    const double Tp1 = (double)T + 1.0;
    double ss = 0.0;
    if (col < n)
        for (int64_t a = ph; a < n_exc; a += 4) {
            const int64_t t = idx[a];
            const double w = pow(1.0 - (double)Rt[t * n + col] / Tp1, -0.5) / norms[t];
            ss += w * w;
        }
    red[ph][lc] = ss;
    __syncthreads();
    const double c = sqrt(red[0][lc] + red[1][lc] + red[2][lc] + red[3][lc]);
    if (col >= n) return;
    for (int64_t a = ph; a < n_exc; a += 4) {
        const int64_t t = idx[a];
        const double w = pow(1.0 - (double)Rt[t * n + col] / Tp1, -0.5) / norms[t];
        Om[a * ldz + col] = (ZT)(w / c);
    }
}

// Raw marginals: radial norm of sample t straight from row t of X, FP64.
__global__ __launch_bounds__(256) void norms_raw_kernel(const float* __restrict__ X, int64_t n,
                                                        double* __restrict__ norms) {
    __shared__ double red[4];
    const int64_t t = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double x = (double)X[t * n + j];
        s += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) norms[t] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// Raw marginals: Omega_aj = sign * X[t_a][j] / ||x_{t_a}||, column j scaled to unit norm.
template <typename ZT>
__global__ __launch_bounds__(256) void omega_raw_kernel(const float* __restrict__ X, int64_t n, float sign,
                                                        const double* __restrict__ norms,
                                                        const int32_t* __restrict__ idx, int64_t n_exc,
                                                        ZT* __restrict__ Om, int64_t ldz) {
    __shared__ double red[4][64];
    const int lc = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t col = blockIdx.x * 64 + lc;
    double ss = 0.0;
    if (col < n)
        for (int64_t a = ph; a < n_exc; a += 4) {
            const int64_t t = idx[a];
            const double w = (double)X[t * n + col] / norms[t];
            ss += w * w;
        }
    red[ph][lc] = ss;
    __syncthreads();
    const double c = sqrt(red[0][lc] + red[1][lc] + red[2][lc] + red[3][lc]);
    if (col >= n) return;
    for (int64_t a = ph; a < n_exc; a += 4) {
        const int64_t t = idx[a];
        const double w = (double)sign * (double)X[t * n + col] / norms[t];
        Om[a * ldz + col] = (ZT)(w / c);
    }
}

int64_t tpdm_work_bytes(int64_t T, int64_t n, int raw) {
    const int64_t planes = raw ? 0 : round_up(T * n * 4, 256) * 2;
    return planes + round_up(T * 8, 256) + round_up(T * 4, 256) + round_up(select_tmp_bytes(), 256) + 256;
}

hipError_t launch_tpdm_omega(const float* X, int64_t T, int64_t n, int lower, int raw, void* Omega, int z_f64,
                             int64_t ldz, int64_t n_exc, void* work, hipStream_t stream) {
    if (!raw && T > RANK_MAX_T) return hipErrorInvalidValue;
    char* w = (char*)work;
    float* Xt = (float*)w;                       // n x T, later reused for Rt (T x n)
    int32_t* R = nullptr;                        // n x T
    if (!raw) {
        w += round_up(T * n * 4, 256);
        R = (int32_t*)w;
        w += round_up(T * n * 4, 256);
    }
    double* norms = (double*)w;
    w += round_up(T * 8, 256);
    int32_t* idx = (int32_t*)w;
    w += round_up(T * 4, 256);
    void* sel = w;
    w += round_up(select_tmp_bytes(), 256);
    double* vstar = (double*)w;
    dim3 tb(256);
    if (raw) {
        const float sign = lower ? -1.0f : 1.0f;
        hipLaunchKernelGGL(norms_raw_kernel, dim3(T), tb, 0, stream, X, n, norms);
        hipError_t e = launch_select(norms, 1, 0, T, T - n_exc, sel, vstar, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(64), 0, stream, (const double*)norms, T, n_exc,
                           (const double*)vstar, idx);
        if (z_f64)
            hipLaunchKernelGGL(omega_raw_kernel<double>, dim3((n + 63) / 64), tb, 0, stream, X, n, sign,
                               (const double*)norms, (const int32_t*)idx, n_exc, (double*)Omega, ldz);
        else
            hipLaunchKernelGGL(omega_raw_kernel<float>, dim3((n + 63) / 64), tb, 0, stream, X, n, sign,
                               (const double*)norms, (const int32_t*)idx, n_exc, (float*)Omega, ldz);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(transpose_kernel<float>, dim3((n + 63) / 64, (T + 63) / 64), tb, 0, stream, X, T, n, Xt,
                       lower ? -1.0f : 1.0f);
    int P2 = 1;
    while (P2 < T) P2 <<= 1;
    if (P2 * 4 > 65536) {
        hipError_t ea = hipFuncSetAttribute((const void*)rank_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            P2 * 4);
        if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(rank_kernel, dim3(n), dim3(1024), (size_t)P2 * 4, stream, (const float*)Xt, T, R);
    int32_t* Rt = (int32_t*)Xt;
    hipLaunchKernelGGL(transpose_kernel<int32_t>, dim3((T + 63) / 64, (n + 63) / 64), tb, 0, stream,
                       (const int32_t*)R, n, T, Rt, (int32_t)1);
    hipLaunchKernelGGL(norms_kernel, dim3(T), tb, 0, stream, (const int32_t*)Rt, T, n, norms);
    hipError_t e = launch_select(norms, 1, 0, T, T - n_exc, sel, vstar, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(64), 0, stream, (const double*)norms, T, n_exc,
                       (const double*)vstar, idx);
    if (z_f64)
        hipLaunchKernelGGL(omega_kernel<double>, dim3((n + 63) / 64), tb, 0, stream, (const int32_t*)Rt, T, n,
                           (const double*)norms, (const int32_t*)idx, n_exc, (double*)Omega, ldz);
    else
        hipLaunchKernelGGL(omega_kernel<float>, dim3((n + 63) / 64), tb, 0, stream, (const int32_t*)Rt, T, n,
                           (const double*)norms, (const int32_t*)idx, n_exc, (float*)Omega, ldz);
    return hipGetLastError();
}

// XCD-aware order of the 128 x 128 output tiles of the S-building GEMMs.
// Work-groups are dispatched round-robin over the 8 XCDs, so the 64 work-groups
// w = x + 8 (64 g + q), q = 0..63, all land on XCD x; they take the 8 x 8 block
// of tiles number 8 g + x (in row-major order of 8 x 8 blocks), and per K slab
// read 8 row blocks and 8 column blocks of Z through that XCD's L2 instead of
// one row block and 64 column blocks.  False for the padding work-groups.
__device__ inline bool syrk_tile(int64_t w, int64_t n_ti, int64_t n_tj, int64_t& ti, int64_t& tj) {
    const int64_t x = w & 7, l = w >> 3;
    const int64_t blk = (l >> 6) * 8 + x, q = l & 63;
    const int64_t bcols = (n_tj + 7) >> 3;
    const int64_t br = blk / bcols, bc = blk - br * bcols;
    ti = br * 8 + (q >> 3);
    tj = bc * 8 + (q & 7);
    return ti < n_ti && tj < n_tj;
}
inline int64_t syrk_grid(int64_t n_ti, int64_t n_tj) {
    const int64_t blocks = ((n_ti + 7) >> 3) * ((n_tj + 7) >> 3);
    return (blocks + 7) / 8 * 8 * 64;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// A full square S (no row panel) is symmetric, so the S-building GEMMs
// compute only the 128 x 128 tiles with ti <= tj; the work-group of an
// off-diagonal tile also stores its transpose.  The transposed value is
// bitwise the one the (tj, ti) tile would compute: the products commute and
// the reduction runs over the same samples in the same order.  Work-groups of
// tiles below the diagonal only clear their sum slot.
__device__ inline bool syrk_symmetric(const BuildOut& o) { return o.row0 == 0 && o.rows == o.n; }

// Epilogue of the S-building GEMMs: |.|, unit diagonal, storage rounding into
// the tiled layout, FP64 sums per work-group (MODE 1), or the FP8 panel
// maxima (MODE 0).  acc[a][b][v] holds element (64 wr + 16 a + 4 lg + v,
// 64 wc + 16 b + lr) of the work-group's 128 x 128 tile (the D layout of the
// 16 x 16 MFMAs).  With mirror, element (j, i) of the transposed tile is
// stored too: a lane's four v values are four consecutive columns of row j,
// one aligned piece of a 16-byte vector of the tiled layout.
// tab: 128 + 128 words of work-group scratch (MODE 0: row and column maxima;
// FP8 MODE 1: the scales of the tile's rows and of the mirrored rows), inv:
// 256 doubles (FP8 MODE 1: their reciprocals).
template <int MODE, int DT>
__device__ __attribute__((always_inline)) inline void syrk_epilogue(const floatx4 (&acc)[4][4], int64_t i0, int64_t j0, bool mirror,
                                     const BuildOut& o, double* __restrict__ wg_sums,
                                     uint32_t* __restrict__ panel_max, uint32_t* tab, double* inv,
                                     double (*red)[4], int64_t slot) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1, lr = lane & 15, lg = lane >> 4;
    // |S_ij| of an off-diagonal element inside the matrix, else 0
    auto offdiag = [&](int a, int b, int v) -> float {
        const int64_t i = i0 + 64 * wr + 16 * a + 4 * lg + v, j = j0 + 64 * wc + 16 * b + lr;
        const bool valid = i < o.rows && j < o.n && o.row0 + i != j;
        return valid ? __builtin_fabsf(acc[a][b][v]) : 0.0f;
    };
    if (MODE == 0) {
        // maxima of non-negative floats compare as their bit patterns; rows
        // reduce over b in registers and over the 16 lanes lr, columns over
        // a and v in registers and over the 4 lanes lg, then one LDS atomic
        // per row (column) and wave
        uint32_t* rowmax = tab;
        uint32_t* colmax = tab + 128;
        if (t < 128) {
            rowmax[t] = 0;
            colmax[t] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float r = 0.0f;
#pragma unroll
                for (int b = 0; b < 4; ++b) r = fmaxf(r, offdiag(a, b, v));
#pragma unroll
                for (int sh = 1; sh < 16; sh <<= 1) r = fmaxf(r, __shfl_xor(r, sh, 64));
                if (lr == 0 && r > 0.0f) atomicMax(&rowmax[64 * wr + 16 * a + 4 * lg + v], __builtin_bit_cast(uint32_t, r));
            }
        if (mirror) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float c = 0.0f;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int v = 0; v < 4; ++v) c = fmaxf(c, offdiag(a, b, v));
                c = fmaxf(c, __shfl_xor(c, 16, 64));
                c = fmaxf(c, __shfl_xor(c, 32, 64));
                if (lg == 0 && c > 0.0f) atomicMax(&colmax[64 * wc + 16 * b + lr], __builtin_bit_cast(uint32_t, c));
            }
        }
        __syncthreads();
        // one device atomic per scale panel that the tile's rows (and the
        // mirrored rows) touch: the thread of the first such row of a panel
        // reduces the panel's rows of the tile
        const int q = t & 127;
        const bool col = t >= 128;
        const int64_t base = col ? j0 : i0, r = base + q;
        if ((!col || mirror) && r < o.rows) {
            const int64_t pnl = r / o.panel_rows, first = pnl * o.panel_rows;
            if (q == 0 || r == first) {
                const uint32_t* mx = col ? colmax : rowmax;
                const int64_t end = min(min(first + o.panel_rows, o.rows), base + 128) - base;
                uint32_t m = 0;
                for (int u = q; u < end; ++u) m = max(m, mx[u]);
                if (m) atomicMax(&panel_max[pnl], m);
            }
        }
        return;
    }
    float* srow = (float*)tab;            // FP8: scale of tile row li
    float* scol = (float*)tab + 128;      // FP8: scale of mirrored row lj
    if constexpr (DT == SYMNMF_S_FP8) {
        const int64_t r = t < 128 ? i0 + t : j0 + (t - 128);
        float sc = 1.0f;
        if (r < o.rows && (t < 128 || mirror)) sc = o.scale[r / o.panel_rows];
        tab[t] = __builtin_bit_cast(uint32_t, sc);
        inv[t] = 1.0 / (double)sc;
        __syncthreads();
    }
    constexpr int E = DT == SYMNMF_S_FP32 ? 4 : (DT == SYMNMF_S_BF16 ? 8 : 16);
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    // per 16 x 16 block (a, b): the tile's elements, then (mirror) the
    // transposed block, row j with four consecutive columns per lane (never a
    // diagonal element, i < j; an FP8 element takes the scale of row j); the
    // block's accumulators are dead after it, which keeps register pressure
    // at the level of the tile alone
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int lj = 64 * wc + 16 * b + lr;
            const int64_t j = j0 + lj;                         // column (mirror: row)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int li = 64 * wr + 16 * a + 4 * lg + v;
                const int64_t i = i0 + li;                     // panel row
                const bool valid = i < o.rows && j < o.n;
                const bool diag = valid && o.row0 + i == j;
                float val = valid ? __builtin_fabsf(acc[a][b][v]) : 0.0f;
                if (diag) val = 1.0f;
                const int64_t off = tiled_offset(i, j, o.ld / KC, E);
                double stored;
                if constexpr (DT == SYMNMF_S_FP32) {
                    ((float*)o.data)[off] = val;
                    stored = val;
                } else if constexpr (DT == SYMNMF_S_BF16) {
                    const uint16_t bits = f32_to_bf16_bits(val);
                    ((uint16_t*)o.data)[off] = bits;
                    stored = bf16_bits_to_f32(bits);
                } else {
                    if (diag) {
                        ((uint8_t*)o.data)[off] = 0;
                        o.diag[i] = val;
                        stored = val;
                    } else if (valid) {
                        const uint8_t code = f32_to_fp8e4m3(val * srow[li]);
                        ((uint8_t*)o.data)[off] = code;
                        stored = (double)fp8e4m3_to_f32(code) * inv[li];
                    } else {
                        ((uint8_t*)o.data)[off] = 0;
                        stored = 0.0;
                    }
                }
                s1 += val;
                s2 += (double)val * (double)val;
                s3 += stored * stored;
            }
            if (mirror) {
                uint32_t mw[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t i = i0 + 64 * wr + 16 * a + 4 * lg + v;
                    const bool valid = i < o.rows && j < o.n;
                    const float val = valid ? __builtin_fabsf(acc[a][b][v]) : 0.0f;
                    double stored;
                    if constexpr (DT == SYMNMF_S_FP32) {
                        mw[v] = __builtin_bit_cast(uint32_t, val);
                        stored = val;
                    } else if constexpr (DT == SYMNMF_S_BF16) {
                        const uint16_t bits = f32_to_bf16_bits(val);
                        mw[v] = bits;
                        stored = bf16_bits_to_f32(bits);
                    } else {
                        const uint8_t code = valid ? f32_to_fp8e4m3(val * scol[lj]) : (uint8_t)0;
                        mw[v] = code;
                        stored = (double)fp8e4m3_to_f32(code) * inv[128 + lj];
                    }
                    s1 += val;
                    s2 += (double)val * (double)val;
                    s3 += stored * stored;
                }
                const int64_t off = tiled_offset(j, i0 + 64 * wr + 16 * a + 4 * lg, o.ld / KC, E);
                if constexpr (DT == SYMNMF_S_FP32) {
                    *(u32x4*)((float*)o.data + off) = u32x4{mw[0], mw[1], mw[2], mw[3]};
                } else if constexpr (DT == SYMNMF_S_BF16) {
                    *(u32x2*)((uint16_t*)o.data + off) = u32x2{mw[0] | (mw[1] << 16), mw[2] | (mw[3] << 16)};
                } else {
                    *(uint32_t*)((uint8_t*)o.data + off) = mw[0] | (mw[1] << 8) | (mw[2] << 16) | (mw[3] << 24);
                }
            }
        }
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_down(s1, off, 64);
        s2 += __shfl_down(s2, off, 64);
        s3 += __shfl_down(s3, off, 64);
    }
    if (lane == 0) { red[0][wv] = s1; red[1][wv] = s2; red[2][wv] = s3; }
    __syncthreads();
    if (t < 3) wg_sums[slot * 3 + t] = red[t][0] + red[t][1] + red[t][2] + red[t][3];
}

// ---------------------------------------------------------------------------
// SYRK: S[i][j] = |sum_t Z[t][row0+i] Z[t][j]| for the panel rows, 128 x 128
// output tile per work-group (2 x 2 waves of 64 x 64), K in steps of 16.
// MODE 0 only finds the largest off-diagonal |S| of every FP8 scale panel;
// MODE 1 stores and sums.
// ---------------------------------------------------------------------------
template <int MODE, int DT>
__global__ __launch_bounds__(256, 2) void syrk_kernel(const float* __restrict__ Z, int64_t K, int64_t ldz, BuildOut o,
                                                   int64_t n_ti, int64_t n_tj, double* __restrict__ wg_sums,
                                                   uint32_t* __restrict__ panel_max) {
    __shared__ float As[2][16][128 + 4];
    __shared__ float Bs[2][16][128 + 4];
    __shared__ uint32_t tab[256];
    __shared__ double inv[(MODE == 1 && DT == SYMNMF_S_FP8) ? 256 : 1];
    __shared__ double red[3][4];
    int64_t ti, tj;
    if (!syrk_tile(blockIdx.x, n_ti, n_tj, ti, tj)) return;
    const bool sym = syrk_symmetric(o);
    if (sym && ti > tj) {
        if (MODE == 1 && threadIdx.x < 3) wg_sums[(ti * n_tj + tj) * 3 + threadIdx.x] = 0.0;
        return;
    }
    const int64_t i0 = ti * 128, j0 = tj * 128;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1, lr = lane & 15, lg = lane >> 4;
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* Za = Z + o.row0 + i0;
    const float* Zb = Z + j0;
    // the next K slab is loaded into registers while the current one is
    // multiplied; LDS is double buffered, so one barrier per slab suffices
    float ra[8], rb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = t + 256 * q;
        const int kk = f >> 7, ii = f & 127;
        ra[q] = Za[kk * ldz + ii];
        rb[q] = Zb[kk * ldz + ii];
    }
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        const int buf = (int)((k0 >> 4) & 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int f = t + 256 * q;
            const int kk = f >> 7, ii = f & 127;
            As[buf][kk][ii] = ra[q];
            Bs[buf][kk][ii] = rb[q];
        }
        __syncthreads();
        if (k0 + 16 < K) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int f = t + 256 * q;
                const int kk = f >> 7, ii = f & 127;
                ra[q] = Za[(k0 + 16 + kk) * ldz + ii];
                rb[q] = Zb[(k0 + 16 + kk) * ldz + ii];
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = 4 * s + lg;
            float av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][64 * wr + 16 * a + lr];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kk][64 * wc + 16 * b + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    syrk_epilogue<MODE, DT>(acc, i0, j0, sym && ti < tj, o, wg_sums, panel_max, tab, inv, red,
                            ti * n_tj + tj);
}

// ---------------------------------------------------------------------------
// Split-precision SYRK on the bf16 matrix cores for BF16 and FP8 storage
// (Henry, Tang & Heinecke 2019): every float is split into two bf16 "planes"
// z = h + m, h = bf16(z), m = bf16(z - h), and S = sum h h + h m + m h with the
// plane products exact in the FP32 accumulator; the dropped m m term and the
// residual are ~2^-16 relative, far below the BF16 (2^-9) or FP8 storage
// rounding that follows.  (FP32 storage uses the FP32-MFMA kernel above.)
// The planes are stored per column with the samples contiguous,
// P[p][c][kk] (Kp = samples rounded up to 32, zero padded), so every lane of
// v_mfma_f32_16x16x32_bf16 loads its 8 consecutive samples as one 16-byte
// vector straight from memory: A[r][8g..8g+7] of row r = lane % 16 and
// g = lane / 16, B the same for the columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void split_planes_kernel(const float* __restrict__ Z, int64_t K, int64_t ldz,
                                                           int64_t Kp, uint16_t* __restrict__ P) {
    __shared__ float tile[32][64 + 1];
    const int64_t c0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * 32;
    const int t = threadIdx.x;
    for (int f = t; f < 32 * 64; f += 256) {
        const int kk = f >> 6, c = f & 63;
        tile[kk][c] = k0 + kk < K ? Z[(k0 + kk) * ldz + c0 + c] : 0.0f;
    }
    __syncthreads();
    const int64_t plane = ldz * Kp;
    for (int f = t; f < 32 * 64; f += 256) {
        const int c = f >> 5, kk = f & 31;
        const float x = tile[kk][c];
        const uint16_t h = f32_to_bf16_bits(x);
        const int64_t o = (c0 + c) * Kp + k0 + kk;
        P[o] = h;
        P[plane + o] = f32_to_bf16_bits(x - bf16_bits_to_f32(h));
    }
}

// Operands are staged through LDS: per 32-sample slab the work-group's 128
// rows and 128 columns in both planes (32 KB) are loaded with 16-byte vectors
// into registers one slab ahead, written to one of two LDS buffers, and every
// wave reads its MFMA fragments from there, so each operand byte is fetched
// from L2 once per work-group instead of once per wave.  The MFMA sequence of
// a slab is unchanged, so the result does not depend on the staging.
constexpr int SPLIT_VECS = 8;   // 16-byte vectors per thread and slab (2 sides x 2 planes x 128 rows x 4)

template <int MODE, int DT>
__global__ __launch_bounds__(256, 2) void syrk_split_kernel(const uint16_t* __restrict__ P, int64_t Kp, int64_t ldz,
                                                            BuildOut o, int64_t n_ti, int64_t n_tj,
                                                            double* __restrict__ wg_sums,
                                                            uint32_t* __restrict__ panel_max) {
    // [buffer][side A/B][plane][row][16-byte part]: 2 x 2 x 2 x 128 x 4 vectors;
    // vector q of thread t sits at f = t + 256 q of its buffer: side q / 4,
    // plane (q / 2) % 2, row t / 4 + 64 (q % 2), part t % 4
    __shared__ u32x4 lds[2 * 2048];
    __shared__ uint32_t tab[256];
    __shared__ double inv[(MODE == 1 && DT == SYMNMF_S_FP8) ? 256 : 1];
    __shared__ double red[3][4];
    int64_t ti, tj;
    if (!syrk_tile(blockIdx.x, n_ti, n_tj, ti, tj)) return;
    const bool sym = syrk_symmetric(o);
    if (sym && ti > tj) {
        if (MODE == 1 && threadIdx.x < 3) wg_sums[(ti * n_tj + tj) * 3 + threadIdx.x] = 0.0;
        return;
    }
    const int64_t i0 = ti * 128, j0 = tj * 128;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1, lr = lane & 15, lg = lane >> 4;
    const int64_t plane = ldz * Kp;
    const uint16_t* tp = P + (int64_t)(t >> 2) * Kp + 8 * (t & 3);
    // work-group-uniform offsets of the 8 vectors (elements)
    auto voff = [&](int q) -> int64_t {
        return ((q >> 2) ? j0 : o.row0 + i0) * Kp + (q & 1) * 64 * Kp + ((q >> 1) & 1) * plane;
    };
    // hh products accumulate in acc; the cross terms of one 32-sample block
    // are formed in two fresh MFMAs (x from the row's lower planes, y from the
    // column's) and added as x + y, so that element (j, i) repeats the exact
    // operations of (i, j) with x and y exchanged: S stays exactly symmetric.
    floatx4 acc[4][4], crs[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
            crs[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    u32x4 reg[SPLIT_VECS];
#pragma unroll
    for (int q = 0; q < SPLIT_VECS; ++q) reg[q] = *(const u32x4*)(tp + voff(q));
    for (int64_t k0 = 0; k0 < Kp; k0 += 32) {
        u32x4* lb = lds + ((k0 >> 5) & 1) * 2048;
#pragma unroll
        for (int q = 0; q < SPLIT_VECS; ++q) lb[t + 256 * q] = reg[q];
        __syncthreads();
        if (k0 + 32 < Kp) {
#pragma unroll
            for (int q = 0; q < SPLIT_VECS; ++q) reg[q] = *(const u32x4*)(tp + voff(q) + k0 + 32);
        }
        // fragment of row / column block a of plane p, side sd:
        // lb[((sd * 2 + p) * 128 + 64 w + 16 a + lr) * 4 + lg]
        bf16x8 bv[2][4];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                bv[p][b] = __builtin_bit_cast(bf16x8, lb[((2 + p) * 128 + 64 * wc + 16 * b + lr) * 4 + lg]);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const bf16x8 a0 = __builtin_bit_cast(bf16x8, lb[(64 * wr + 16 * a + lr) * 4 + lg]);
            const bf16x8 a1 = __builtin_bit_cast(bf16x8, lb[(128 + 64 * wr + 16 * a + lr) * 4 + lg]);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const floatx4 x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv[0][b], zero, 0, 0, 0);
                const floatx4 y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv[1][b], zero, 0, 0, 0);
                crs[a][b] += x + y;
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv[0][b], acc[a][b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += crs[a][b];
    syrk_epilogue<MODE, DT>(acc, i0, j0, sym && ti < tj, o, wg_sums, panel_max, tab, inv, red,
                            ti * n_tj + tj);
}

// FP64 S (parity runs): plain FP64 FMAs, 64 x 64 tile per work-group, each
// thread a 4 x 4 block, K in steps of 16 through LDS.
__global__ __launch_bounds__(256) void syrk_f64_kernel(const double* __restrict__ Z, int64_t K, int64_t ldz,
                                                       BuildOut o, double* __restrict__ wg_sums) {
    __shared__ double As[16][64];
    __shared__ double Bs[16][64];
    __shared__ double red[3][4];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x, ti = t >> 4, tj = t & 15;
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        __syncthreads();
        for (int f = t; f < 16 * 64; f += 256) {
            const int kk = f >> 6, ii = f & 63;
            As[kk][ii] = Z[(k0 + kk) * ldz + o.row0 + i0 + ii];
            Bs[kk][ii] = Z[(k0 + kk) * ldz + j0 + ii];
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) acc[a][b] += As[kk][4 * ti + a] * Bs[kk][4 * tj + b];
    }
    double s1 = 0.0, s2 = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const int64_t i = i0 + 4 * ti + a, j = j0 + 4 * tj + b;
            const bool valid = i < o.rows && j < o.n;
            double v = valid ? fabs(acc[a][b]) : 0.0;
            if (valid && o.row0 + i == j) v = 1.0;
            ((double*)o.data)[i * o.ld + j] = v;
            s1 += v;
            s2 += v * v;
        }
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_down(s1, off, 64);
        s2 += __shfl_down(s2, off, 64);
    }
    const int wv = t >> 6;
    if ((t & 63) == 0) { red[0][wv] = s1; red[1][wv] = s2; red[2][wv] = s2; }
    __syncthreads();
    if (t < 3) {
        const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        wg_sums[wg * 3 + t] = red[t][0] + red[t][1] + red[t][2] + red[t][3];
    }
}

// scale_p = 448 / max off-diagonal |S| of panel p (1 when the panel is all zero)
__global__ void fp8_scales_kernel(const uint32_t* __restrict__ panel_max, int64_t panels, float* __restrict__ scale) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= panels) return;
    const float m = __builtin_bit_cast(float, panel_max[p]);
    scale[p] = m > 0.0f ? 448.0f / m : 1.0f;
}

// column sums of an (m x 3) FP64 array in a fixed order
__global__ __launch_bounds__(1024) void sum3_kernel(const double* __restrict__ x, int64_t m, double* __restrict__ out) {
    __shared__ double red[3][16];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < m; i += 1024)
        for (int c = 0; c < 3; ++c) s[c] += x[i * 3 + c];
    for (int c = 0; c < 3; ++c) {
        double v = s[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double r = 0.0;
        for (int i = 0; i < 16; ++i) r += red[threadIdx.x][i];
        out[threadIdx.x] = r;
    }
}

static hipError_t finish_sums(const double* wg_sums, int64_t wgs, double* sums, hipStream_t stream) {
    hipLaunchKernelGGL(sum3_kernel, dim3(1), dim3(1024), 0, stream, wg_sums, wgs, sums);
    return hipGetLastError();
}

int64_t syrk_sum_words(const BuildOut& o) {
    return 4 + 3 * (o.ld / 64) * (o.rows_pad / 64);
}

hipError_t launch_syrk_store(const void* Zv, int z_f64, int64_t K, int64_t ldz, const BuildOut& o, double* sums,
                             uint32_t* panel_max, hipStream_t stream) {
    // sums: [0..2] results, then 3 * wgs partial words
    if (z_f64) {
        if (o.dtype != SYMNMF_S_FP64) return hipErrorInvalidValue;
        dim3 grid(o.ld / 64, o.rows_pad / 64), block(256);
        hipLaunchKernelGGL(syrk_f64_kernel, grid, block, 0, stream, (const double*)Zv, K, ldz, o, sums + 4);
        return finish_sums(sums + 4, (int64_t)grid.x * grid.y, sums, stream);
    }
    if (o.dtype == SYMNMF_S_FP64) return hipErrorInvalidValue;
    const float* Z = (const float*)Zv;
    const int64_t n_ti = o.rows_pad / 128, n_tj = o.ld / 128;
    dim3 grid(syrk_grid(n_ti, n_tj)), block(256);
    const int64_t wgs = n_ti * n_tj;
    double* wg_sums = sums + 4;
    if (o.dtype == SYMNMF_S_FP8) {
        const int64_t panels = (o.rows + o.panel_rows - 1) / o.panel_rows;
        hipLaunchKernelGGL((syrk_kernel<0, SYMNMF_S_FP8>), grid, block, 0, stream, Z, K, ldz, o, n_ti, n_tj, wg_sums,
                           panel_max);
        hipLaunchKernelGGL(fp8_scales_kernel, dim3((panels + 255) / 256), dim3(256), 0, stream,
                           (const uint32_t*)panel_max, panels, o.scale);
        hipLaunchKernelGGL((syrk_kernel<1, SYMNMF_S_FP8>), grid, block, 0, stream, Z, K, ldz, o, n_ti, n_tj, wg_sums,
                           panel_max);
    } else if (o.dtype == SYMNMF_S_BF16) {
        hipLaunchKernelGGL((syrk_kernel<1, SYMNMF_S_BF16>), grid, block, 0, stream, Z, K, ldz, o, n_ti, n_tj, wg_sums,
                           panel_max);
    } else {
        hipLaunchKernelGGL((syrk_kernel<1, SYMNMF_S_FP32>), grid, block, 0, stream, Z, K, ldz, o, n_ti, n_tj, wg_sums,
                           panel_max);
    }
    return finish_sums(wg_sums, wgs, sums, stream);
}

int64_t syrk_split_ws_bytes(int64_t K, int64_t ldz) { return 2 * ldz * round_up(K, 32) * 2; }

hipError_t launch_syrk_split_store(const float* Z, int64_t K, int64_t ldz, const BuildOut& o, double* sums,
                                   uint32_t* panel_max, void* ws, hipStream_t stream) {
    if (o.dtype != SYMNMF_S_BF16 && o.dtype != SYMNMF_S_FP8) return hipErrorInvalidValue;
    const int64_t Kp = round_up(K, 32);
    uint16_t* P = (uint16_t*)ws;
    hipLaunchKernelGGL(split_planes_kernel, dim3(ldz / 64, Kp / 32), dim3(256), 0, stream, Z, K, ldz, Kp, P);
    const int64_t n_ti = o.rows_pad / 128, n_tj = o.ld / 128;
    dim3 grid(syrk_grid(n_ti, n_tj)), block(256);
    const int64_t wgs = n_ti * n_tj;
    double* wg_sums = sums + 4;
    if (o.dtype == SYMNMF_S_FP8) {
        const int64_t panels = (o.rows + o.panel_rows - 1) / o.panel_rows;
        hipLaunchKernelGGL((syrk_split_kernel<0, SYMNMF_S_FP8>), grid, block, 0, stream, (const uint16_t*)P, Kp, ldz,
                           o, n_ti, n_tj, wg_sums, panel_max);
        hipLaunchKernelGGL(fp8_scales_kernel, dim3((panels + 255) / 256), dim3(256), 0, stream,
                           (const uint32_t*)panel_max, panels, o.scale);
        hipLaunchKernelGGL((syrk_split_kernel<1, SYMNMF_S_FP8>), grid, block, 0, stream, (const uint16_t*)P, Kp, ldz,
                           o, n_ti, n_tj, wg_sums, panel_max);
    } else {
        hipLaunchKernelGGL((syrk_split_kernel<1, SYMNMF_S_BF16>), grid, block, 0, stream, (const uint16_t*)P, Kp, ldz,
                           o, n_ti, n_tj, wg_sums, panel_max);
    }
    return finish_sums(wg_sums, wgs, sums, stream);
}

// ---------------------------------------------------------------------------
// Store a given dense panel (rows x n, FP32 or FP64, row-major).
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void store_dense_kernel(const T* __restrict__ src, BuildOut o,
                                                          double* __restrict__ wg_sums, uint32_t* __restrict__ panel_max) {
    __shared__ double red[3][4];
    const int64_t i = blockIdx.x;   // panel row (padded range)
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    uint32_t mx = 0;
    for (int64_t j = threadIdx.x; j < o.ld; j += 256) {
        const bool valid = i < o.rows && j < o.n;
        const bool diag = valid && (o.row0 + i == j);
        const double v = valid ? (double)src[i * o.n + j] : 0.0;
        if (MODE == 0) {
            if (valid && !diag) {
                const uint32_t b = __builtin_bit_cast(uint32_t, (float)fabs(v));
                mx = b > mx ? b : mx;
            }
            continue;
        }
        const int E = o.dtype == SYMNMF_S_FP32 ? 4 : (o.dtype == SYMNMF_S_BF16 ? 8 : 16);
        const int64_t off = o.dtype == SYMNMF_S_FP64 ? i * o.ld + j : tiled_offset(i, j, o.ld / KC, E);
        double stored;
        if (o.dtype == SYMNMF_S_FP64) { ((double*)o.data)[off] = v; stored = v; }
        else if (o.dtype == SYMNMF_S_FP32) { ((float*)o.data)[off] = (float)v; stored = (float)v; }
        else if (o.dtype == SYMNMF_S_BF16) {
            const uint16_t bits = f32_to_bf16_bits((float)v);
            ((uint16_t*)o.data)[off] = bits;
            stored = bf16_bits_to_f32(bits);
        } else {
            if (diag) { ((uint8_t*)o.data)[off] = 0; o.diag[i] = (float)v; stored = (float)v; }
            else if (valid) {
                const float sc = o.scale[i / o.panel_rows];
                const uint8_t code = f32_to_fp8e4m3((float)v * sc);
                ((uint8_t*)o.data)[off] = code;
                stored = (double)fp8e4m3_to_f32(code) / (double)sc;
            } else { ((uint8_t*)o.data)[off] = 0; stored = 0.0; }
        }
        s1 += v;
        s2 += v * v;
        s3 += stored * stored;
    }
    if (MODE == 0) {
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t other = __shfl_down(mx, off, 64);
            mx = other > mx ? other : mx;
        }
        if ((threadIdx.x & 63) == 0 && i < o.rows && mx) atomicMax(&panel_max[i / o.panel_rows], mx);
        return;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_down(s1, off, 64);
        s2 += __shfl_down(s2, off, 64);
        s3 += __shfl_down(s3, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][wv] = s1; red[1][wv] = s2; red[2][wv] = s3; }
    __syncthreads();
    if (threadIdx.x < 3)
        wg_sums[i * 3 + threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

hipError_t launch_store_dense(const void* src, int src_f64, const BuildOut& o, double* sums, uint32_t* panel_max,
                              hipStream_t stream) {
    dim3 grid(o.rows_pad), block(256);
    double* wg_sums = sums + 4;
    if (o.dtype == SYMNMF_S_FP8) {
        const int64_t panels = (o.rows + o.panel_rows - 1) / o.panel_rows;
        if (src_f64) hipLaunchKernelGGL((store_dense_kernel<double, 0>), grid, block, 0, stream, (const double*)src, o, wg_sums, panel_max);
        else hipLaunchKernelGGL((store_dense_kernel<float, 0>), grid, block, 0, stream, (const float*)src, o, wg_sums, panel_max);
        hipLaunchKernelGGL(fp8_scales_kernel, dim3((panels + 255) / 256), dim3(256), 0, stream,
                           (const uint32_t*)panel_max, panels, o.scale);
    }
    if (src_f64) hipLaunchKernelGGL((store_dense_kernel<double, 1>), grid, block, 0, stream, (const double*)src, o, wg_sums, panel_max);
    else hipLaunchKernelGGL((store_dense_kernel<float, 1>), grid, block, 0, stream, (const float*)src, o, wg_sums, panel_max);
    return finish_sums(wg_sums, o.rows_pad, sums, stream);
}

}  // namespace symnmf
