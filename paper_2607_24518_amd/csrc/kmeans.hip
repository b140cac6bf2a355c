// Spherical K-means (Lloyd) on the rows of S and the cosine silhouette
// (paper section "Clustering": spherical K-means as constrained SymNMF and
// the computational comparison, table tab:kmeans).
//
// The points are the unit rows s^_i = s_i / ||s_i|| of the stored S.  Since S
// is symmetric, both products Lloyd needs are S.H passes of the stream kernel
// with an n x K factor:
//   assignment:  cos(s^_i, c_k) = (S C)_ik / ||s_i||, argmax over k;
//   update:      sum_{j in k} s^_j = (S W)_{:,k} with W_jk = [label_j = k] / ||s_j||,
//                then c_k = that sum / its length.
// Factors live slice-major, [slice][rows_pad][w] with w = 16, 32 or 64, so
// every slice is one stream pass at a rank the MFMA kernels support and K is
// not limited to 64.  FP64 storage uses FP64 factors and the generic stream
// (parity runs); the other storage types use FP32 factors, and the argmax is
// taken on the FP32 products.  Sums of the objective and the silhouette are
// FP64 in a fixed order, so results do not depend on scheduling.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace symnmf {

namespace {

constexpr int KT = 256;   // threads of every kernel below

// --------------------------------------------------------------------------
// Row lengths.  Pass 1 writes FP64 sums of S_ij^2 per (row, 256-column
// chunk); pass 2 adds the chunks of every row in increasing order.
// --------------------------------------------------------------------------
template <int DT>   // 0 FP32, 1 BF16, 2 FP8 tiled storage
__global__ __launch_bounds__(KT) void rowsq_tiled_kernel(const uint8_t* __restrict__ S, int64_t n_chunks,
                                                         int64_t rows_pad, double* __restrict__ part) {
    constexpr int EB = DT == 0 ? 4 : (DT == 1 ? 2 : 1);   // bytes per element
    constexpr int E = 16 / EB;                              // elements per lane load
    constexpr int NS = 256 / (4 * E);                       // sub-steps per tile
    const int64_t R = blockIdx.x / n_chunks, C = blockIdx.x - R * n_chunks;
    const u32x4* tile = (const u32x4*)(S + (R * n_chunks + C) * TILE_ELEMS * EB);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
            // lane l holds E columns of tile row 64 wv + 16 rg + l % 16
            const u32x4 v = __builtin_nontemporal_load(tile + ((int64_t)(wv * NS + s) * 4 + rg) * 64 + l);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t word = v[q];
                if (DT == 0) {
                    const double x = (double)__builtin_bit_cast(float, word);
                    acc[rg] += x * x;
                } else if (DT == 1) {
                    const double x0 = (double)bf16_bits_to_f32((uint16_t)(word & 0xffffu));
                    const double x1 = (double)bf16_bits_to_f32((uint16_t)(word >> 16));
                    acc[rg] += x0 * x0 + x1 * x1;
                } else {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double x = (double)fp8e4m3_to_f32((uint8_t)((word >> (8 * b)) & 0xffu));
                        acc[rg] += x * x;
                    }
                }
            }
        }
    }
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same rows
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) {
        acc[rg] += __shfl_xor(acc[rg], 16, 64);
        acc[rg] += __shfl_xor(acc[rg], 32, 64);
    }
    if (l < 16) {
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) part[C * rows_pad + R * TR + 64 * wv + 16 * rg + l] = acc[rg];
    }
}

// FP64 storage: row-major, leading dimension ld; wave w takes rows w, w + 4, ...
__global__ __launch_bounds__(KT) void rowsq_f64_kernel(const double* __restrict__ S, int64_t ld, int64_t n_chunks,
                                                       int64_t rows_pad, double* __restrict__ part) {
    const int64_t R = blockIdx.x / n_chunks, C = blockIdx.x - R * n_chunks;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int r = wv; r < TR; r += 4) {
        const double* row = S + (R * TR + r) * ld + C * KC;
        double a = 0.0;
        for (int j = l; j < KC; j += 64) a += row[j] * row[j];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (l == 0) part[C * rows_pad + R * TR + r] = a;
    }
}

// norms[i] = sqrt(sum over chunks); FP8 storage: codes / scale plus the
// diagonal kept aside (its code is 0).  bad[0] counts zero or non-finite rows.
__global__ __launch_bounds__(KT) void rownorm_finish_kernel(const double* __restrict__ part, int64_t n_chunks,
                                                            int64_t rows_pad, int64_t rows,
                                                            const float* __restrict__ scale,
                                                            const float* __restrict__ diag, int64_t panel_rows,
                                                            double* __restrict__ norms, int32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int64_t c = 0; c < n_chunks; ++c) s += part[c * rows_pad + i];
    if (scale) {
        const double sc = (double)scale[i / panel_rows], d = (double)diag[i];
        s = s / (sc * sc) + d * d;
    }
    if (!(s > 0.0) || !(s < INFINITY)) atomicAdd(bad, 1);
    norms[i] = sqrt(s);
}

// --------------------------------------------------------------------------
// Dense S.X of one slice from the stream's partial tiles (fixed order over
// the work-groups that streamed each tile).  FP8: partial / scale + S_ii X_i.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(KT) void slice_dense_kernel(const T* __restrict__ part, int64_t rows, int w, PlanView p,
                                                         const float* __restrict__ scale,
                                                         const float* __restrict__ diag, int64_t panel_rows,
                                                         const T* __restrict__ X, T* __restrict__ Y) {
    const int32_t tile = blockIdx.x;
    int64_t w_lo, w_hi, sb, sm;
    partial_slots(p, tile, w_lo, w_hi, sb, sm);
    for (int f = threadIdx.x; f < TR * w; f += KT) {
        const int r = f / w, c = f - r * w;
        const int64_t row = (int64_t)tile * TR + r;
        if (row >= rows) continue;
        T s = 0;
        for (int64_t q = w_lo; q <= w_hi; ++q) s += part[((sm * q + sb) * TR + r) * (int64_t)w + c];
        if (scale) s = s / (T)scale[row / panel_rows] + (T)diag[row] * X[row * w + c];
        Y[row * w + c] = s;
    }
}

// --------------------------------------------------------------------------
// Factor preparation
// --------------------------------------------------------------------------
// W[s][j][c] = [label_j = s w + c] / ||s_j|| (zero in padding rows / columns)
template <typename T>
__global__ __launch_bounds__(KT) void weights_kernel(const int32_t* __restrict__ labels,
                                                     const double* __restrict__ norms, int64_t n, int64_t rows_pad,
                                                     int w, int64_t total, T* __restrict__ W) {
    for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * KT) {
        const int64_t s = idx / (rows_pad * w), rem = idx - s * rows_pad * w;
        const int64_t j = rem / w, c = rem - j * w;
        T v = 0;
        if (j < n && (int64_t)labels[j] == s * w + c) v = (T)(1.0 / norms[j]);
        W[idx] = v;
    }
}

// counts[c] = members of cluster c; bad[0] counts labels outside [lo, K)
__global__ __launch_bounds__(KT) void count_kernel(const int32_t* __restrict__ labels, int64_t n, int64_t K, int lo,
                                                   int32_t* __restrict__ counts, int32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i >= n) return;
    const int32_t c = labels[i];
    if (c < lo || (int64_t)c >= K) {
        atomicAdd(bad, 1);
        return;
    }
    if (c >= 0) atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(KT) void fill_labels_kernel(int32_t* __restrict__ labels, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i < n) labels[i] = -1;
}
__global__ __launch_bounds__(KT) void seed_labels_kernel(int32_t* __restrict__ labels, const int64_t* __restrict__ rows,
                                                         int64_t K) {
    const int64_t c = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (c < K) labels[rows[c]] = (int32_t)c;
}

// Column sums of squares of M over 256-row blocks (FP64), in a fixed order.
template <typename T>
__global__ __launch_bounds__(KT) void colsq_kernel(const T* __restrict__ M, int64_t rows_pad, int w, int64_t ncol,
                                                   double* __restrict__ part) {
    __shared__ double red[KT];
    const int64_t b = blockIdx.x;        // row block
    const int s = blockIdx.y;            // slice
    const int t = threadIdx.x, groups = KT / w, c = t % w, g = t / w;
    const T* base = M + ((int64_t)s * rows_pad + b * TR) * w;
    double a = 0.0;
    for (int r = g; r < TR; r += groups) {
        const double v = (double)base[(int64_t)r * w + c];
        a += v * v;
    }
    red[t] = a;
    __syncthreads();
    if (t < w) {
        double tot = 0.0;
        for (int q = 0; q < groups; ++q) tot += red[q * w + t];
        part[b * ncol + (int64_t)s * w + t] = tot;
    }
}

// inv[col] = 1 / ||M_col|| for clusters with members and a non-zero sum, else
// 0 (the column keeps its previous centroid)
__global__ __launch_bounds__(KT) void colnorm_finish_kernel(const double* __restrict__ part, int64_t blocks,
                                                            int64_t ncol, int64_t K, const int32_t* __restrict__ counts,
                                                            double* __restrict__ inv) {
    const int64_t col = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (col >= ncol) return;
    double s = 0.0;
    for (int64_t b = 0; b < blocks; ++b) s += part[b * ncol + col];
    inv[col] = (col < K && counts[col] > 0 && s > 0.0 && s < INFINITY) ? 1.0 / sqrt(s) : 0.0;
}

template <typename T>
__global__ __launch_bounds__(KT) void normalise_kernel(const T* __restrict__ M, const double* __restrict__ inv,
                                                       int64_t rows_pad, int w, int64_t total,
                                                       const T* __restrict__ Cprev, T* __restrict__ C) {
    for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * KT) {
        const int64_t s = idx / (rows_pad * w), c = idx % w;
        const double iv = inv[s * w + c];
        C[idx] = iv > 0.0 ? (T)((double)M[idx] * iv) : (Cprev ? Cprev[idx] : (T)0);
    }
}

// slices <-> n x K row-major
template <typename T>
__global__ __launch_bounds__(KT) void pack_kernel(const T* __restrict__ src, int64_t n, int64_t K, int64_t rows_pad,
                                                  int w, int64_t total, T* __restrict__ dst) {
    for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * KT) {
        const int64_t s = idx / (rows_pad * w), rem = idx - s * rows_pad * w;
        const int64_t j = rem / w, kk = s * w + (rem - j * w);
        dst[idx] = (j < n && kk < K) ? src[j * K + kk] : (T)0;
    }
}
template <typename T>
__global__ __launch_bounds__(KT) void unpack_kernel(const T* __restrict__ src, int64_t n, int64_t K, int64_t rows_pad,
                                                    int w, T* __restrict__ dst) {
    for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < n * K; idx += (int64_t)gridDim.x * KT) {
        const int64_t j = idx / K, kk = idx - j * K, s = kk / w;
        dst[idx] = src[(s * rows_pad + j) * w + (kk - s * w)];
    }
}

// --------------------------------------------------------------------------
// Assignment and silhouette (one thread per row; FP64 block sums)
// --------------------------------------------------------------------------
__device__ inline void block_sum2(double a, int64_t b, double* out_a, int64_t* out_b) {
    __shared__ double sa[KT / 64];
    __shared__ int64_t sb[KT / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0;
        int64_t tb = 0;
        for (int q = 0; q < KT / 64; ++q) {
            ta += sa[q];
            tb += sb[q];
        }
        *out_a = ta;
        if (out_b) *out_b = tb;
    }
}

template <typename T>
__global__ __launch_bounds__(KT) void assign_kernel(const T* __restrict__ P, const double* __restrict__ norms,
                                                    int64_t n, int64_t rows_pad, int w, int64_t K,
                                                    int32_t* __restrict__ labels, T* __restrict__ best,
                                                    int32_t* __restrict__ counts, double* __restrict__ jpart,
                                                    int64_t* __restrict__ chpart, int track) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    double jl = 0.0;
    int64_t ch = 0;
    if (i < n) {
        T bv = P[i * w];
        int32_t bk = 0;
        for (int64_t kk = 1; kk < K; ++kk) {
            const int64_t s = kk / w;
            const T v = P[(s * rows_pad + i) * w + (kk - s * w)];
            if (v > bv) {   // strict: ties keep the lower index
                bv = v;
                bk = (int32_t)kk;
            }
        }
        const double cv = (double)bv / norms[i];
        jl = 1.0 - cv;
        ch = (track && labels[i] != bk) ? 1 : 0;   // labels hold the previous assignment only when tracked
        labels[i] = bk;
        if (best) best[i] = (T)cv;
        atomicAdd(&counts[bk], 1);
    }
    block_sum2(jl, ch, jpart + blockIdx.x, chpart + blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(KT) void silhouette_kernel(const T* __restrict__ Q, const double* __restrict__ norms,
                                                        const int32_t* __restrict__ labels,
                                                        const int32_t* __restrict__ counts, int64_t n,
                                                        int64_t rows_pad, int w, int64_t K,
                                                        double* __restrict__ spart) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    double si = 0.0;
    if (i < n) {
        const int32_t la = labels[i];
        const double na = (double)counts[la];
        if (na > 1.0) {
            const double inv = 1.0 / norms[i];
            auto dot = [&](int64_t kk) {   // s^_i . m_kk
                const int64_t s = kk / w;
                return (double)Q[(s * rows_pad + i) * w + (kk - s * w)] * inv;
            };
            const double a = (na - dot(la)) / (na - 1.0);
            double b = INFINITY;
            for (int64_t kk = 0; kk < K; ++kk) {
                if (kk == la || counts[kk] == 0) continue;
                b = fmin(b, 1.0 - dot(kk) / (double)counts[kk]);
            }
            const double mx = fmax(a, b);
            si = mx > 0.0 ? (b - a) / mx : 0.0;
        }
    }
    block_sum2(si, 0, spart + blockIdx.x, nullptr);
}

// out[0] = sum a, out[1] = sum b (b may be NULL), fixed order
__global__ __launch_bounds__(KT) void sum_parts_kernel(const double* __restrict__ a, const int64_t* __restrict__ b,
                                                       int64_t m, double* __restrict__ out) {
    __shared__ double sa[KT];
    __shared__ double sb[KT];
    const int t = threadIdx.x;
    double x = 0.0, y = 0.0;
    for (int64_t i = t; i < m; i += KT) {
        x += a[i];
        if (b) y += (double)b[i];
    }
    sa[t] = x;
    sb[t] = y;
    __syncthreads();
    for (int o = KT / 2; o > 0; o >>= 1) {
        if (t < o) {
            sa[t] += sa[t + o];
            sb[t] += sb[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

// --------------------------------------------------------------------------
// Spectral diagnostic: trace and power iteration on the first column of a
// 16-wide factor slice.
// --------------------------------------------------------------------------
template <int DT>   // 0 FP32, 1 BF16, 2 FP8 tiled storage, 3 FP64 row-major
__global__ __launch_bounds__(KT) void diag_sum_kernel(const void* __restrict__ S, int64_t n, int64_t ld,
                                                      int64_t n_chunks, const float* __restrict__ diag,
                                                      double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        if (DT == 3) v = ((const double*)S)[i * ld + i];
        else if (DT == 2) v = (double)diag[i];
        else if (DT == 1) v = (double)bf16_bits_to_f32(((const uint16_t*)S)[tiled_offset(i, i, n_chunks, 8)]);
        else v = (double)((const float*)S)[tiled_offset(i, i, n_chunks, 4)];
    }
    block_sum2(v, 0, part + blockIdx.x, nullptr);
}

// partials of v . y and y . y over rows i < n (column 0 of 16-wide slices)
template <typename T>
__global__ __launch_bounds__(KT) void power_dots_kernel(const T* __restrict__ X, const T* __restrict__ Y, int64_t n,
                                                        int w, double* __restrict__ pvy, double* __restrict__ pyy) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    double vy = 0.0, yy = 0.0;
    if (i < n) {
        const double v = (double)X[i * w], y = (double)Y[i * w];
        vy = v * y;
        yy = y * y;
    }
    block_sum2(vy, 0, pvy + blockIdx.x, nullptr);
    __syncthreads();
    block_sum2(yy, 0, pyy + blockIdx.x, nullptr);
}

template <typename T>
__global__ __launch_bounds__(KT) void power_scale_kernel(const T* __restrict__ Y, int64_t n, int w, double scale,
                                                         T* __restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i < n) X[i * w] = (T)((double)Y[i * w] * scale);
}

template <typename T>
__global__ __launch_bounds__(KT) void fill_col0_kernel(T* __restrict__ X, int64_t n, int w, double value) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i < n) X[i * w] = (T)value;
}

template <typename T>
__global__ __launch_bounds__(KT) void copy_col0_kernel(const T* __restrict__ X, int64_t n, int w,
                                                       float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i < n) out[i] = (float)X[i * w];
}

// --------------------------------------------------------------------------
// k-means++ seeding: row c of the stored S scaled by 1 / ||s_c|| into column 0
// of a 16-wide slice, then d_j <- min(d_j, 1 - cos) after one S pass.
// --------------------------------------------------------------------------
template <int DT, typename T>   // DT: 0 FP32, 1 BF16, 2 FP8 tiled, 3 FP64 row-major
__global__ __launch_bounds__(KT) void gather_row_kernel(const void* __restrict__ S, int64_t n, int64_t ld,
                                                        int64_t n_chunks, const float* __restrict__ scale,
                                                        const float* __restrict__ diag, int64_t panel_rows,
                                                        int64_t c, double inv_norm, int w, T* __restrict__ X) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (j >= n) return;
    double v;
    if (DT == 3) v = ((const double*)S)[c * ld + j];
    else if (DT == 2) v = j == c ? (double)diag[c]
                                 : (double)fp8e4m3_to_f32(((const uint8_t*)S)[tiled_offset(c, j, n_chunks, 16)]) /
                                       (double)scale[c / panel_rows];
    else if (DT == 1) v = (double)bf16_bits_to_f32(((const uint16_t*)S)[tiled_offset(c, j, n_chunks, 8)]);
    else v = (double)((const float*)S)[tiled_offset(c, j, n_chunks, 4)];
    X[j * w] = (T)(v * inv_norm);
}

// d_j = min(d_j, max(1 - (S x)_j / ||s_j||, 0)), 0 at the seeds; FP64 block sums
template <typename T>
__global__ __launch_bounds__(KT) void kpp_update_kernel(const T* __restrict__ P, const double* __restrict__ norms,
                                                        const uint8_t* __restrict__ chosen, int64_t n, int w,
                                                        double* __restrict__ d, double* __restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    double v = 0.0;
    if (j < n) {
        const double dist = fmax(1.0 - (double)P[j * w] / norms[j], 0.0);
        v = chosen[j] ? 0.0 : fmin(d[j], dist);
        d[j] = v;
    }
    block_sum2(v, 0, part + blockIdx.x, nullptr);
}

__global__ void mark_kernel(uint8_t* __restrict__ chosen, int64_t c) { chosen[c] = 1; }

inline unsigned blocks_for(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + KT - 1) / KT, 65536)); }

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
// Device allocations of one call, zero-filled, freed on scope exit.
// Scratch of one K-means call, from the context pool (zeroed buffers).
struct Scratch {
    CallScratch cs;
    hipError_t& err;
    explicit Scratch(symnmf_ctx* c) : cs(c), err(cs.err) {}
    void* get(int64_t bytes) { return cs.get(bytes, true); }
};

// Everything one K-means call needs to multiply S by n x K factors.
struct KCall {
    const symnmf_S* S;
    hipStream_t sm;
    int64_t n, rows_pad, tiles, chunks, K, w, nsl, ncol;
    bool f64, mfma;
    int64_t esz;
    PlanView pv;
    void* part = nullptr;    // stream partials
    void* img = nullptr;     // chunk images of one slice
    double* norms = nullptr; // rows_pad
    int32_t* counts = nullptr;
    int32_t* bad = nullptr;
    double* scal = nullptr;  // [0] sum, [1] second sum
    double* jpart = nullptr;
    int64_t* chpart = nullptr;
    double* colpart = nullptr;
    double* inv = nullptr;

    int64_t factor_elems() const { return nsl * rows_pad * w; }
    int64_t factor_bytes() const { return factor_elems() * esz; }
    int64_t row_blocks() const { return (n + KT - 1) / KT; }
};

int64_t slice_width(int64_t K) { return K <= 16 ? 16 : (K <= 32 ? 32 : 64); }

symnmf_status kcall_setup(symnmf_ctx* ctx, const symnmf_S* S, int64_t K, Scratch& sc, KCall& kc) {
    if (!S || !S->data) return fail(ctx, SYMNMF_EINVAL, "kmeans: S is NULL");
    if (S->rows != S->n || S->row0 != 0)
        return fail(ctx, SYMNMF_EUNSUPPORTED, "kmeans: needs the full matrix (rows == n), not a row panel");
    if (K < 1 || K > S->n) return fail(ctx, SYMNMF_EINVAL, "kmeans: need 1 <= K <= n (K = %lld, n = %lld)",
                                       (long long)K, (long long)S->n);
    if (S->rows_pad != S->ld || S->rows_pad % TR != 0 || S->rows_pad < S->n)
        return fail(ctx, SYMNMF_EINVAL, "kmeans: inconsistent S descriptor");
    HIP_OK(ctx, hipSetDevice(ctx->device));
    kc.S = S;
    kc.sm = ctx->stream;
    kc.n = S->n;
    kc.rows_pad = S->rows_pad;
    kc.tiles = S->rows_pad / TR;
    kc.chunks = S->ld / KC;
    kc.K = K;
    kc.w = slice_width(K);
    kc.nsl = (K + kc.w - 1) / kc.w;
    kc.ncol = kc.nsl * kc.w;
    kc.f64 = S->dtype == SYMNMF_S_FP64;
    kc.esz = kc.f64 ? 8 : 4;
    kc.mfma = stream_uses_mfma(S->dtype, kc.f64, kc.f64, kc.w) != 0;
    kc.pv = plan_view(nullptr, 1, (int32_t)kc.tiles, (int32_t)kc.chunks, 0);
    int64_t part_tiles;
    if (kc.mfma && stream_tall_supported(S->dtype, 0, kc.w)) {
        kc.pv.tall = 1;
        kc.pv.P = tall_wgs(ctx->cus, kc.tiles);
        part_tiles = 2 * ((int64_t)kc.pv.P + tall_pairs(kc.tiles));
    } else {
        kc.pv.P = ctx->cus * (ctx->wgs_per_cu > 0 ? ctx->wgs_per_cu
                                                  : (kc.f64 ? 2 : stream_wgs_per_cu(S->dtype, kc.w)));
        part_tiles = (int64_t)kc.pv.P + kc.tiles;
    }
    kc.part = sc.get(part_tiles * TR * kc.w * kc.esz);
    if (kc.mfma) kc.img = sc.get(h_image_words(S->dtype, kc.w, kc.chunks) * 4);
    kc.norms = (double*)sc.get(kc.rows_pad * 8);
    kc.counts = (int32_t*)sc.get(kc.ncol * 4);
    kc.bad = (int32_t*)sc.get(16);
    kc.scal = (double*)sc.get(4 * 8);
    kc.jpart = (double*)sc.get(kc.row_blocks() * 8);
    kc.chpart = (int64_t*)sc.get(kc.row_blocks() * 8);
    kc.colpart = (double*)sc.get(kc.tiles * kc.ncol * 8);
    kc.inv = (double*)sc.get(kc.ncol * 8);
    if (sc.err != hipSuccess)
        return fail(ctx, sc.err == hipErrorOutOfMemory ? SYMNMF_ENOMEM : SYMNMF_EDEVICE, "kmeans: %s",
                    hipGetErrorString(sc.err));
    return SYMNMF_OK;
}

hipError_t launch_row_norms(const KCall& kc, double* part) {
    const symnmf_S* S = kc.S;
    const unsigned grid = (unsigned)(kc.tiles * kc.chunks);
    if (S->dtype == SYMNMF_S_FP32)
        hipLaunchKernelGGL(rowsq_tiled_kernel<0>, dim3(grid), dim3(KT), 0, kc.sm, (const uint8_t*)S->data, kc.chunks,
                           kc.rows_pad, part);
    else if (S->dtype == SYMNMF_S_BF16)
        hipLaunchKernelGGL(rowsq_tiled_kernel<1>, dim3(grid), dim3(KT), 0, kc.sm, (const uint8_t*)S->data, kc.chunks,
                           kc.rows_pad, part);
    else if (S->dtype == SYMNMF_S_FP8)
        hipLaunchKernelGGL(rowsq_tiled_kernel<2>, dim3(grid), dim3(KT), 0, kc.sm, (const uint8_t*)S->data, kc.chunks,
                           kc.rows_pad, part);
    else
        hipLaunchKernelGGL(rowsq_f64_kernel, dim3(grid), dim3(KT), 0, kc.sm, (const double*)S->data, S->ld,
                           kc.chunks, kc.rows_pad, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool fp8 = S->dtype == SYMNMF_S_FP8;
    hipLaunchKernelGGL(rownorm_finish_kernel, dim3((unsigned)((kc.n + KT - 1) / KT)), dim3(KT), 0, kc.sm, part,
                       kc.chunks, kc.rows_pad, kc.n, fp8 ? S->panel_scale : nullptr, fp8 ? S->diag : nullptr,
                       S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1, kc.norms, kc.bad);
    return hipGetLastError();
}

// Row lengths into kc.norms; EINVAL on a zero or non-finite row.  Synchronises.
symnmf_status compute_norms(symnmf_ctx* ctx, KCall& kc, Scratch& sc) {
    double* part = (double*)sc.get(kc.chunks * kc.rows_pad * 8);
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "kmeans: %s", hipGetErrorString(sc.err));
    HIP_OK(ctx, launch_row_norms(kc, part));
    int32_t bad = 0;
    HIP_OK(ctx, hipMemcpyAsync(&bad, kc.bad, 4, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    if (bad) return fail(ctx, SYMNMF_EINVAL, "kmeans: %d rows of S are zero or non-finite", bad);
    return SYMNMF_OK;
}

// Y = S X for slice-major factors (every slice one stream pass)
hipError_t s_times(const KCall& kc, const void* X, void* Y) {
    const symnmf_S* S = kc.S;
    const bool fp8 = S->dtype == SYMNMF_S_FP8;
    for (int64_t s = 0; s < kc.nsl; ++s) {
        const char* Xs = (const char*)X + s * kc.rows_pad * kc.w * kc.esz;
        char* Ys = (char*)Y + s * kc.rows_pad * kc.w * kc.esz;
        hipError_t e = hipSuccess;
        if (kc.mfma) e = launch_h_image((const float*)Xs, S->dtype, kc.w, kc.chunks, 1.0f, (uint32_t*)kc.img, kc.sm);
        if (e == hipSuccess)
            e = launch_stream(S->data, S->dtype, S->ld, Xs, kc.f64, kc.w, kc.part, kc.f64, kc.pv, kc.sm, kc.img, kc.img);
        if (e != hipSuccess) return e;
        const float* scale = fp8 ? S->panel_scale : nullptr;
        const float* diag = fp8 ? S->diag : nullptr;
        const int64_t pr = S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1;
        if (kc.f64)
            hipLaunchKernelGGL(slice_dense_kernel<double>, dim3((unsigned)kc.tiles), dim3(KT), 0, kc.sm,
                               (const double*)kc.part, kc.n, (int)kc.w, kc.pv, scale, diag, pr, (const double*)Xs,
                               (double*)Ys);
        else
            hipLaunchKernelGGL(slice_dense_kernel<float>, dim3((unsigned)kc.tiles), dim3(KT), 0, kc.sm,
                               (const float*)kc.part, kc.n, (int)kc.w, kc.pv, scale, diag, pr, (const float*)Xs,
                               (float*)Ys);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_weights_t(const KCall& kc, const int32_t* labels, void* W) {
    hipLaunchKernelGGL(weights_kernel<T>, dim3(blocks_for(kc.factor_elems())), dim3(KT), 0, kc.sm, labels, kc.norms,
                       kc.n, kc.rows_pad, (int)kc.w, kc.factor_elems(), (T*)W);
    return hipGetLastError();
}

hipError_t launch_counts(const KCall& kc, const int32_t* labels, int lo) {
    hipError_t e = launch_zero(kc.counts, kc.ncol * 4, kc.sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)kc.row_blocks()), dim3(KT), 0, kc.sm, labels, kc.n, kc.K, lo,
                       kc.counts, kc.bad);
    return hipGetLastError();
}

// C = normalised S W(labels); clusters without members keep Cprev (may be NULL).
// kc.counts must hold the member counts of labels.
template <typename T>
hipError_t centroid_step(const KCall& kc, const int32_t* labels, void* W, void* M, const void* Cprev, void* C) {
    hipError_t e = launch_weights_t<T>(kc, labels, W);
    if (e == hipSuccess) e = s_times(kc, W, M);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsq_kernel<T>, dim3((unsigned)kc.tiles, (unsigned)kc.nsl), dim3(KT), 0, kc.sm, (const T*)M,
                       kc.rows_pad, (int)kc.w, kc.ncol, kc.colpart);
    hipLaunchKernelGGL(colnorm_finish_kernel, dim3(blocks_for(kc.ncol)), dim3(KT), 0, kc.sm, kc.colpart, kc.tiles,
                       kc.ncol, kc.K, kc.counts, kc.inv);
    hipLaunchKernelGGL(normalise_kernel<T>, dim3(blocks_for(kc.factor_elems())), dim3(KT), 0, kc.sm, (const T*)M,
                       kc.inv, kc.rows_pad, (int)kc.w, kc.factor_elems(), (const T*)Cprev, (T*)C);
    return hipGetLastError();
}

// labels = argmax_k (S C)_ik; kc.counts = the new member counts; scal[0] = J,
// scal[1] = labels changed.
template <typename T>
hipError_t assign_step(const KCall& kc, const void* C, void* Pbuf, int32_t* labels, void* best, int track = 1) {
    hipError_t e = s_times(kc, C, Pbuf);
    if (e == hipSuccess) e = launch_zero(kc.counts, kc.ncol * 4, kc.sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(assign_kernel<T>, dim3((unsigned)kc.row_blocks()), dim3(KT), 0, kc.sm, (const T*)Pbuf,
                       kc.norms, kc.n, kc.rows_pad, (int)kc.w, kc.K, labels, (T*)best, kc.counts, kc.jpart,
                       kc.chpart, track);
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(KT), 0, kc.sm, kc.jpart, kc.chpart, kc.row_blocks(), kc.scal);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pack(const KCall& kc, const void* src, void* dst) {
    hipLaunchKernelGGL(pack_kernel<T>, dim3(blocks_for(kc.factor_elems())), dim3(KT), 0, kc.sm, (const T*)src, kc.n,
                       kc.K, kc.rows_pad, (int)kc.w, kc.factor_elems(), (T*)dst);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_unpack(const KCall& kc, const void* src, void* dst) {
    hipLaunchKernelGGL(unpack_kernel<T>, dim3(blocks_for(kc.n * kc.K)), dim3(KT), 0, kc.sm, (const T*)src, kc.n,
                       kc.K, kc.rows_pad, (int)kc.w, (T*)dst);
    return hipGetLastError();
}

symnmf_status read_scal(symnmf_ctx* ctx, const KCall& kc, double out[2]) {
    HIP_OK(ctx, hipMemcpyAsync(out, kc.scal, 16, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    return SYMNMF_OK;
}

symnmf_status check_bad(symnmf_ctx* ctx, const KCall& kc, const char* what) {
    int32_t bad = 0;
    HIP_OK(ctx, hipMemcpyAsync(&bad, kc.bad, 4, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    if (bad) return fail(ctx, SYMNMF_EINVAL, "%s: %d labels out of range", what, bad);
    return SYMNMF_OK;
}

// Forgy seeds: partial Fisher-Yates over [0, n) on 53-bit SplitMix64 uniforms
std::vector<int64_t> forgy_rows(uint64_t seed, int64_t n, int64_t K) {
    std::vector<int64_t> a((size_t)n);
    for (int64_t i = 0; i < n; ++i) a[(size_t)i] = i;
    for (int64_t i = 0; i < K; ++i) {
        const double u = (double)(splitmix64(seed, (uint64_t)i) >> 11) * 0x1.0p-53;
        int64_t j = i + (int64_t)(u * (double)(n - i));
        if (j > n - 1) j = n - 1;
        std::swap(a[(size_t)i], a[(size_t)j]);
    }
    a.resize((size_t)K);
    return a;
}

template <typename T>
symnmf_status kmeans_run(symnmf_ctx* ctx, KCall& kc, Scratch& sc, const std::vector<int64_t>& rows, double tol,
                         int64_t max_iter, int32_t* labels, void* C_out, symnmf_kmeans_stats* st,
                         std::chrono::steady_clock::time_point t0) {
    void* W = sc.get(kc.factor_bytes());
    void* M = sc.get(kc.factor_bytes());
    void* C = sc.get(kc.factor_bytes());
    void* Pb = sc.get(kc.factor_bytes());
    int64_t* rows_d = (int64_t*)sc.get(kc.K * 8);
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "kmeans: %s", hipGetErrorString(sc.err));
    symnmf_status r = compute_norms(ctx, kc, sc);
    if (r != SYMNMF_OK) return r;
    HIP_OK(ctx, hipMemcpyAsync(rows_d, rows.data(), kc.K * 8, hipMemcpyHostToDevice, kc.sm));
    hipLaunchKernelGGL(fill_labels_kernel, dim3((unsigned)kc.row_blocks()), dim3(KT), 0, kc.sm, labels, kc.n);
    hipLaunchKernelGGL(seed_labels_kernel, dim3(blocks_for(kc.K)), dim3(KT), 0, kc.sm, labels, rows_d, kc.K);
    HIP_OK(ctx, hipGetLastError());
    // seed centroids: the unit seed rows, through the same update step
    HIP_OK(ctx, launch_counts(kc, labels, -1));
    HIP_OK(ctx, centroid_step<T>(kc, labels, W, M, nullptr, C));
    HIP_OK(ctx, assign_step<T>(kc, C, Pb, labels, nullptr));
    double sv[2];
    if ((r = read_scal(ctx, kc, sv)) != SYMNMF_OK) return r;
    double J = sv[0];
    const double J0 = J;
    int64_t changed = (int64_t)sv[1], it = 0;
    bool converged = false;
    if (!std::isfinite(J)) return fail(ctx, SYMNMF_ENUMERIC, "kmeans: non-finite objective");
    while (it < max_iter) {
        HIP_OK(ctx, centroid_step<T>(kc, labels, W, M, C, C));   // counts are those of labels
        HIP_OK(ctx, assign_step<T>(kc, C, Pb, labels, nullptr));
        if ((r = read_scal(ctx, kc, sv)) != SYMNMF_OK) return r;
        ++it;
        const double Jn = sv[0];
        changed = (int64_t)sv[1];
        if (!std::isfinite(Jn)) return fail(ctx, SYMNMF_ENUMERIC, "kmeans: non-finite objective");
        const bool stop = J <= 0.0 || (J - Jn) < tol * J;
        J = Jn;
        if (stop) {
            converged = true;
            break;
        }
    }
    if (C_out) HIP_OK(ctx, launch_unpack<T>(kc, C, C_out));
    std::vector<int32_t> counts((size_t)kc.ncol);
    HIP_OK(ctx, hipMemcpyAsync(counts.data(), kc.counts, kc.ncol * 4, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    if (st) {
        st->iters = it;
        st->J0 = J0;
        st->J = J;
        st->changed = changed;
        st->converged = converged ? 1 : 0;
        st->empty = 0;
        for (int64_t c = 0; c < kc.K; ++c) st->empty += counts[(size_t)c] == 0 ? 1 : 0;
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!converged) return fail(ctx, SYMNMF_ENOTCONV, "kmeans: no convergence within %lld iterations",
                                (long long)max_iter);
    return SYMNMF_OK;
}

template <typename T>
symnmf_status spectral_run(symnmf_ctx* ctx, KCall& kc, Scratch& sc, int64_t max_iter, double tol, double* lambda1,
                           double* trace, double* r_eff, double* collapse, double* collapse_rows, int64_t* iters,
                           float* u1) {
    const symnmf_S* S = kc.S;
    void* X = sc.get(kc.factor_bytes());
    void* Y = sc.get(kc.factor_bytes());
    double* p1 = (double*)sc.get(kc.row_blocks() * 8);
    double* p2 = (double*)sc.get(kc.row_blocks() * 8);
    double* out = (double*)sc.get(4 * 8);
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "spectral: %s", hipGetErrorString(sc.err));
    const unsigned nb = (unsigned)kc.row_blocks();
    // trace
    switch (S->dtype) {
        case SYMNMF_S_FP32:
            hipLaunchKernelGGL(diag_sum_kernel<0>, dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld, kc.chunks,
                               S->diag, p1);
            break;
        case SYMNMF_S_BF16:
            hipLaunchKernelGGL(diag_sum_kernel<1>, dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld, kc.chunks,
                               S->diag, p1);
            break;
        case SYMNMF_S_FP8:
            hipLaunchKernelGGL(diag_sum_kernel<2>, dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld, kc.chunks,
                               S->diag, p1);
            break;
        default:
            hipLaunchKernelGGL(diag_sum_kernel<3>, dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld, kc.chunks,
                               S->diag, p1);
    }
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(KT), 0, kc.sm, p1, nullptr, kc.row_blocks(), out);
    HIP_OK(ctx, hipGetLastError());
    double tr[2];
    HIP_OK(ctx, hipMemcpyAsync(tr, out, 16, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    // power iteration from the normalised all-ones vector (S >= 0: its
    // Perron vector is non-negative, so the start is never orthogonal to it)
    hipLaunchKernelGGL(fill_col0_kernel<T>, dim3(nb), dim3(KT), 0, kc.sm, (T*)X, kc.n, (int)kc.w,
                       1.0 / std::sqrt((double)kc.n));
    HIP_OK(ctx, hipGetLastError());
    double lam = 0.0, yy = 0.0;
    int64_t it = 0;
    for (; it < max_iter;) {
        HIP_OK(ctx, s_times(kc, X, Y));
        hipLaunchKernelGGL(power_dots_kernel<T>, dim3(nb), dim3(KT), 0, kc.sm, (const T*)X, (const T*)Y, kc.n,
                           (int)kc.w, p1, p2);
        hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(KT), 0, kc.sm, p1, nullptr, kc.row_blocks(), out);
        hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(KT), 0, kc.sm, p2, nullptr, kc.row_blocks(), out + 2);
        HIP_OK(ctx, hipGetLastError());
        double d[4];
        HIP_OK(ctx, hipMemcpyAsync(d, out, 32, hipMemcpyDeviceToHost, kc.sm));
        HIP_OK(ctx, hipStreamSynchronize(kc.sm));
        ++it;
        const double lam_new = d[0];   // Rayleigh quotient v^T S v with ||v|| = 1
        yy = d[2];
        if (!std::isfinite(lam_new) || !(yy > 0.0))
            return fail(ctx, SYMNMF_ENUMERIC, "spectral: power iteration broke down (S v = 0 or non-finite)");
        hipLaunchKernelGGL(power_scale_kernel<T>, dim3(nb), dim3(KT), 0, kc.sm, (const T*)Y, kc.n, (int)kc.w,
                           1.0 / std::sqrt(yy), (T*)X);
        HIP_OK(ctx, hipGetLastError());
        const bool done = it > 1 && std::fabs(lam_new - lam) <= tol * std::fabs(lam_new);
        lam = lam_new;
        if (done) break;
    }
    if (u1) {
        hipLaunchKernelGGL(copy_col0_kernel<T>, dim3(nb), dim3(KT), 0, kc.sm, (const T*)X, kc.n, (int)kc.w, u1);
        HIP_OK(ctx, hipGetLastError());
    }
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    const double fro2 = S->fro2_stored;
    if (lambda1) *lambda1 = lam;
    if (trace) *trace = tr[0];
    if (r_eff) *r_eff = tr[0] / lam;
    if (collapse) *collapse = (fro2 - lam * lam) / fro2;
    // from the rows: sum_i ||s_i||^2 sin^2(theta_i) = ||S||^2 - sum_i (u . s_i)^2 = ||S||^2 - ||S u||^2
    if (collapse_rows) *collapse_rows = (fro2 - yy) / fro2;
    if (iters) *iters = it;
    return SYMNMF_OK;
}

// k-means++ seed rows (host vector) on the unit rows of the stored S
template <typename T>
symnmf_status kpp_run(symnmf_ctx* ctx, KCall& kc, Scratch& sc, uint64_t seed, std::vector<int64_t>& rows) {
    const symnmf_S* S = kc.S;
    void* X = sc.get(kc.factor_bytes());
    void* Pb = sc.get(kc.factor_bytes());
    double* d = (double*)sc.get(kc.rows_pad * 8);
    uint8_t* chosen = (uint8_t*)sc.get(kc.rows_pad);
    double* part = (double*)sc.get(kc.row_blocks() * 8);
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "kmeans_seed_pp: %s", hipGetErrorString(sc.err));
    symnmf_status r = compute_norms(ctx, kc, sc);
    if (r != SYMNMF_OK) return r;
    std::vector<double> norms_h((size_t)kc.n);
    HIP_OK(ctx, hipMemcpyAsync(norms_h.data(), kc.norms, kc.n * 8, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    const unsigned nb = (unsigned)kc.row_blocks();
    const bool fp8 = S->dtype == SYMNMF_S_FP8;
    const int64_t pr = S->fp8_panel_rows > 0 ? S->fp8_panel_rows : 1;
    auto draw = [&](int64_t i) { return (double)(splitmix64(seed, (uint64_t)i) >> 11) * 0x1.0p-53; };
    auto add_seed = [&](int64_t c) -> hipError_t {
        const double inv = 1.0 / norms_h[(size_t)c];
        switch (S->dtype) {
            case SYMNMF_S_FP32:
                hipLaunchKernelGGL((gather_row_kernel<0, T>), dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld,
                                   kc.chunks, S->panel_scale, S->diag, pr, c, inv, (int)kc.w, (T*)X);
                break;
            case SYMNMF_S_BF16:
                hipLaunchKernelGGL((gather_row_kernel<1, T>), dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld,
                                   kc.chunks, S->panel_scale, S->diag, pr, c, inv, (int)kc.w, (T*)X);
                break;
            case SYMNMF_S_FP8:
                hipLaunchKernelGGL((gather_row_kernel<2, T>), dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld,
                                   kc.chunks, S->panel_scale, S->diag, pr, c, inv, (int)kc.w, (T*)X);
                break;
            default:
                hipLaunchKernelGGL((gather_row_kernel<3, T>), dim3(nb), dim3(KT), 0, kc.sm, S->data, kc.n, S->ld,
                                   kc.chunks, S->panel_scale, S->diag, pr, c, inv, (int)kc.w, (T*)X);
        }
        hipLaunchKernelGGL(mark_kernel, dim3(1), dim3(1), 0, kc.sm, chosen, c);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = s_times(kc, X, Pb);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kpp_update_kernel<T>, dim3(nb), dim3(KT), 0, kc.sm, (const T*)Pb, kc.norms, chosen, kc.n,
                           (int)kc.w, d, part);
        return hipGetLastError();
    };
    (void)fp8;
    // d starts at +infinity (the first update takes the distances to seed 0)
    {
        std::vector<double> inf((size_t)kc.n, INFINITY);
        HIP_OK(ctx, hipMemcpyAsync(d, inf.data(), kc.n * 8, hipMemcpyHostToDevice, kc.sm));
        HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    }
    std::vector<uint8_t> chosen_h((size_t)kc.n, 0);
    rows.clear();
    int64_t first = (int64_t)(draw(0) * (double)kc.n);
    if (first > kc.n - 1) first = kc.n - 1;
    rows.push_back(first);
    chosen_h[(size_t)first] = 1;
    HIP_OK(ctx, add_seed(first));
    std::vector<double> parts(nb), blk(KT);
    for (int64_t i = 1; i < kc.K; ++i) {
        HIP_OK(ctx, hipMemcpyAsync(parts.data(), part, nb * 8, hipMemcpyDeviceToHost, kc.sm));
        HIP_OK(ctx, hipStreamSynchronize(kc.sm));
        double total = 0.0;
        for (unsigned b = 0; b < nb; ++b) total += parts[b];
        if (!std::isfinite(total)) return fail(ctx, SYMNMF_ENUMERIC, "kmeans_seed_pp: non-finite distances");
        int64_t j = -1;
        if (total > 0.0) {
            // smallest j with sum_{l <= j} d_l > u_i * total
            const double target = draw(i) * total;
            double acc = 0.0;
            unsigned b = 0;
            while (b + 1 < nb && acc + parts[b] <= target) acc += parts[b++];
            const int64_t r0 = (int64_t)b * KT;
            const int64_t cnt = std::min<int64_t>(KT, kc.n - r0);
            HIP_OK(ctx, hipMemcpyAsync(blk.data(), d + r0, cnt * 8, hipMemcpyDeviceToHost, kc.sm));
            HIP_OK(ctx, hipStreamSynchronize(kc.sm));
            j = r0 + cnt - 1;
            for (int64_t q = 0; q < cnt; ++q) {
                acc += blk[(size_t)q];
                if (acc > target) {
                    j = r0 + q;
                    break;
                }
            }
        } else {
            for (int64_t q = 0; q < kc.n; ++q)
                if (!chosen_h[(size_t)q]) {
                    j = q;
                    break;
                }
        }
        rows.push_back(j);
        chosen_h[(size_t)j] = 1;
        if (i + 1 < kc.K) HIP_OK(ctx, add_seed(j));
    }
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    return SYMNMF_OK;
}

}  // namespace
}  // namespace symnmf

using namespace symnmf;

extern "C" {

symnmf_status symnmf_kmeans_seed_rows(uint64_t seed, int64_t n, int64_t K, int64_t* out) {
    if (!out || K < 1 || K > n) return SYMNMF_EINVAL;
    const std::vector<int64_t> rows = forgy_rows(seed, n, K);
    std::copy(rows.begin(), rows.end(), out);
    return SYMNMF_OK;
}

symnmf_status symnmf_kmeans_seed_pp(symnmf_ctx* ctx, const symnmf_S* S, int64_t K, uint64_t seed, int64_t* rows) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!rows) return fail(ctx, SYMNMF_EINVAL, "kmeans_seed_pp: rows is NULL");
    Scratch sc(ctx);
    KCall kc;
    // one-column passes: K = 1 sets up a 16-wide slice; the seed count is K
    symnmf_status r = kcall_setup(ctx, S, 1, sc, kc);
    if (r != SYMNMF_OK) return r;
    if (K < 1 || K > kc.n) return fail(ctx, SYMNMF_EINVAL, "kmeans_seed_pp: need 1 <= K <= n");
    kc.K = K;
    std::vector<int64_t> v;
    r = kc.f64 ? kpp_run<double>(ctx, kc, sc, seed, v) : kpp_run<float>(ctx, kc, sc, seed, v);
    if (r != SYMNMF_OK) return r;
    std::copy(v.begin(), v.end(), rows);
    return SYMNMF_OK;
}

symnmf_status symnmf_row_norms(symnmf_ctx* ctx, const symnmf_S* S, double* norms) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!norms) return fail(ctx, SYMNMF_EINVAL, "row_norms: norms is NULL");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, 1, sc, kc);
    if (r == SYMNMF_OK) r = compute_norms(ctx, kc, sc);
    if (r != SYMNMF_OK) return r;
    HIP_OK(ctx, hipMemcpyAsync(norms, kc.norms, kc.n * 8, hipMemcpyDeviceToDevice, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    return SYMNMF_OK;
}

symnmf_status symnmf_kmeans_assign(symnmf_ctx* ctx, const symnmf_S* S, const void* C, int64_t K, int32_t* labels,
                                   void* best, double* J) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!C || !labels) return fail(ctx, SYMNMF_EINVAL, "kmeans_assign: NULL argument");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, K, sc, kc);
    if (r != SYMNMF_OK) return r;
    void* Cs = sc.get(kc.factor_bytes());
    void* Pb = sc.get(kc.factor_bytes());
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "kmeans_assign: %s", hipGetErrorString(sc.err));
    if ((r = compute_norms(ctx, kc, sc)) != SYMNMF_OK) return r;
    if (kc.f64) {
        HIP_OK(ctx, launch_pack<double>(kc, C, Cs));
        HIP_OK(ctx, assign_step<double>(kc, Cs, Pb, labels, best, 0));
    } else {
        HIP_OK(ctx, launch_pack<float>(kc, C, Cs));
        HIP_OK(ctx, assign_step<float>(kc, Cs, Pb, labels, best, 0));
    }
    double sv[2];
    if ((r = read_scal(ctx, kc, sv)) != SYMNMF_OK) return r;
    if (J) *J = sv[0];
    if (!std::isfinite(sv[0])) return fail(ctx, SYMNMF_ENUMERIC, "kmeans_assign: non-finite objective");
    return SYMNMF_OK;
}

symnmf_status symnmf_kmeans_centroids(symnmf_ctx* ctx, const symnmf_S* S, const int32_t* labels, int64_t K,
                                      const void* C_prev, void* C) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!labels || !C) return fail(ctx, SYMNMF_EINVAL, "kmeans_centroids: NULL argument");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, K, sc, kc);
    if (r != SYMNMF_OK) return r;
    void* W = sc.get(kc.factor_bytes());
    void* M = sc.get(kc.factor_bytes());
    void* Cs = sc.get(kc.factor_bytes());
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "kmeans_centroids: %s", hipGetErrorString(sc.err));
    if ((r = compute_norms(ctx, kc, sc)) != SYMNMF_OK) return r;
    HIP_OK(ctx, launch_counts(kc, labels, -1));
    if ((r = check_bad(ctx, kc, "kmeans_centroids")) != SYMNMF_OK) return r;
    if (kc.f64) {
        if (C_prev) HIP_OK(ctx, launch_pack<double>(kc, C_prev, Cs));
        HIP_OK(ctx, centroid_step<double>(kc, labels, W, M, Cs, Cs));
        HIP_OK(ctx, launch_unpack<double>(kc, Cs, C));
    } else {
        if (C_prev) HIP_OK(ctx, launch_pack<float>(kc, C_prev, Cs));
        HIP_OK(ctx, centroid_step<float>(kc, labels, W, M, Cs, Cs));
        HIP_OK(ctx, launch_unpack<float>(kc, Cs, C));
    }
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    return SYMNMF_OK;
}

symnmf_status symnmf_kmeans(symnmf_ctx* ctx, const symnmf_S* S, int64_t K, uint64_t seed, const int64_t* init_rows,
                            double tol, int64_t max_iter, int32_t* labels, void* C, symnmf_kmeans_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return SYMNMF_EINVAL;
    if (!labels) return fail(ctx, SYMNMF_EINVAL, "kmeans: labels is NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol) || max_iter < 0)
        return fail(ctx, SYMNMF_EINVAL, "kmeans: need tol >= 0 and max_iter >= 0");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, K, sc, kc);
    if (r != SYMNMF_OK) return r;
    std::vector<int64_t> rows;
    if (init_rows) {
        rows.assign(init_rows, init_rows + K);
        std::vector<int64_t> sorted = rows;
        std::sort(sorted.begin(), sorted.end());
        for (int64_t i = 0; i < K; ++i) {
            if (sorted[(size_t)i] < 0 || sorted[(size_t)i] >= kc.n || (i > 0 && sorted[(size_t)i] == sorted[(size_t)i - 1]))
                return fail(ctx, SYMNMF_EINVAL, "kmeans: init_rows must be K distinct rows in [0, n)");
        }
    } else {
        rows = forgy_rows(seed, kc.n, K);
    }
    if (kc.f64) return kmeans_run<double>(ctx, kc, sc, rows, tol, max_iter, labels, C, stats, t0);
    return kmeans_run<float>(ctx, kc, sc, rows, tol, max_iter, labels, C, stats, t0);
}

symnmf_status symnmf_spectral(symnmf_ctx* ctx, const symnmf_S* S, int64_t max_iter, double tol, double* lambda1,
                              double* trace, double* r_eff, double* collapse, double* collapse_rows, int64_t* iters,
                              float* u1) {
    if (!ctx) return SYMNMF_EINVAL;
    if (max_iter < 1 || !(tol >= 0.0)) return fail(ctx, SYMNMF_EINVAL, "spectral: need max_iter >= 1, tol >= 0");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, 1, sc, kc);
    if (r != SYMNMF_OK) return r;
    if (kc.f64)
        return spectral_run<double>(ctx, kc, sc, max_iter, tol, lambda1, trace, r_eff, collapse, collapse_rows, iters,
                                    u1);
    return spectral_run<float>(ctx, kc, sc, max_iter, tol, lambda1, trace, r_eff, collapse, collapse_rows, iters, u1);
}

symnmf_status symnmf_silhouette(symnmf_ctx* ctx, const symnmf_S* S, const int32_t* labels, int64_t K, double* sil) {
    if (!ctx) return SYMNMF_EINVAL;
    if (!labels || !sil) return fail(ctx, SYMNMF_EINVAL, "silhouette: NULL argument");
    Scratch sc(ctx);
    KCall kc;
    symnmf_status r = kcall_setup(ctx, S, K, sc, kc);
    if (r != SYMNMF_OK) return r;
    void* W = sc.get(kc.factor_bytes());
    void* M = sc.get(kc.factor_bytes());
    void* Q = sc.get(kc.factor_bytes());
    double* spart = (double*)sc.get(kc.row_blocks() * 8);
    if (sc.err != hipSuccess) return fail(ctx, SYMNMF_ENOMEM, "silhouette: %s", hipGetErrorString(sc.err));
    if ((r = compute_norms(ctx, kc, sc)) != SYMNMF_OK) return r;
    HIP_OK(ctx, launch_counts(kc, labels, 0));
    if ((r = check_bad(ctx, kc, "silhouette")) != SYMNMF_OK) return r;
    std::vector<int32_t> counts((size_t)kc.ncol);
    HIP_OK(ctx, hipMemcpyAsync(counts.data(), kc.counts, kc.ncol * 4, hipMemcpyDeviceToHost, kc.sm));
    HIP_OK(ctx, hipStreamSynchronize(kc.sm));
    int64_t present = 0;
    for (int64_t c = 0; c < K; ++c) present += counts[(size_t)c] > 0 ? 1 : 0;
    if (present < 2) return fail(ctx, SYMNMF_EINVAL, "silhouette: needs at least two non-empty clusters");
    // M = S W (cluster sums of unit rows), Q = S M; s^_i . m_c = Q_ic / ||s_i||
    if (kc.f64) {
        HIP_OK(ctx, launch_weights_t<double>(kc, labels, W));
        HIP_OK(ctx, s_times(kc, W, M));
        HIP_OK(ctx, s_times(kc, M, Q));
        hipLaunchKernelGGL(silhouette_kernel<double>, dim3((unsigned)kc.row_blocks()), dim3(KT), 0, kc.sm,
                           (const double*)Q, kc.norms, labels, kc.counts, kc.n, kc.rows_pad, (int)kc.w, kc.K, spart);
    } else {
        HIP_OK(ctx, launch_weights_t<float>(kc, labels, W));
        HIP_OK(ctx, s_times(kc, W, M));
        HIP_OK(ctx, s_times(kc, M, Q));
        hipLaunchKernelGGL(silhouette_kernel<float>, dim3((unsigned)kc.row_blocks()), dim3(KT), 0, kc.sm,
                           (const float*)Q, kc.norms, labels, kc.counts, kc.n, kc.rows_pad, (int)kc.w, kc.K, spart);
    }
    HIP_OK(ctx, hipGetLastError());
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(KT), 0, kc.sm, spart, nullptr, kc.row_blocks(), kc.scal);
    HIP_OK(ctx, hipGetLastError());
    double sv[2];
    if ((r = read_scal(ctx, kc, sv)) != SYMNMF_OK) return r;
    *sil = sv[0] / (double)kc.n;
    if (!std::isfinite(*sil)) return fail(ctx, SYMNMF_ENUMERIC, "silhouette: non-finite value");
    return SYMNMF_OK;
}

}  // extern "C"
