// Order statistics on the device: MSB-first radix selection on IEEE bit
// patterns (for non-negative values the unsigned bit pattern orders like the
// value).  Used for median(g^2) of the Piecewise AdaGrad reset (appendix,
// Piecewise AdaGrad) and for the radial threshold of the TPDM exceedances.
//
// Pass d (8 bits per pass, from the top) histograms the digit of the keys that
// match the prefix fixed so far, then one thread walks the histogram to the
// bin holding the target rank, extends the prefix and rebases the rank.
#include "common.h"

namespace symnmf {

struct SelState {
    uint64_t prefix;
    uint64_t mask;
    uint64_t rank;
    uint64_t pad;
    uint32_t hist[256];
};

int64_t select_tmp_bytes() { return (int64_t)sizeof(SelState); }

template <typename T>
__device__ inline uint64_t sel_key(T v, int square);
template <>
__device__ inline uint64_t sel_key<float>(float v, int square) {
    const float x = square ? v * v : v;
    return (uint64_t)__builtin_bit_cast(uint32_t, x);
}
template <>
__device__ inline uint64_t sel_key<double>(double v, int square) {
    const double x = square ? v * v : v;
    return __builtin_bit_cast(uint64_t, x);
}

__global__ void sel_init(SelState* st, uint64_t rank) {
    const int t = threadIdx.x;
    st->hist[t] = 0;
    if (t == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->rank = rank;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void sel_hist(const T* __restrict__ x, int64_t m, int square, int shift,
                                                SelState* st) {
    __shared__ uint32_t lh[256];
    lh[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = sel_key<T>(x[i], square);
        if ((key & mask) == prefix) atomicAdd(&lh[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t v = lh[threadIdx.x];
    if (v) atomicAdd(&st->hist[threadIdx.x], v);
}

__global__ void sel_pick(SelState* st, int shift) {
    if (threadIdx.x == 0) {
        uint64_t cum = 0, rank = st->rank;
        int b = 0;
        for (; b < 255; ++b) {
            if (cum + st->hist[b] > rank) break;
            cum += st->hist[b];
        }
        st->prefix |= (uint64_t)b << shift;
        st->mask |= (uint64_t)255u << shift;
        st->rank = rank - cum;
    }
    __syncthreads();
    st->hist[threadIdx.x] = 0;
}

template <typename T>
__global__ void sel_out(const SelState* st, double* out) {
    if (sizeof(T) == 4) out[0] = (double)__builtin_bit_cast(float, (uint32_t)st->prefix);
    else out[0] = __builtin_bit_cast(double, st->prefix);
}

template <typename T>
static hipError_t run_select(const T* x, int square, int64_t m, int64_t rank, SelState* st, double* out,
                             hipStream_t stream) {
    hipLaunchKernelGGL(sel_init, dim3(1), dim3(256), 0, stream, st, (uint64_t)rank);
    int64_t blocks = (m + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    for (int shift = 8 * (int)sizeof(T) - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(sel_hist<T>, dim3(blocks), dim3(256), 0, stream, x, m, square, shift, st);
        hipLaunchKernelGGL(sel_pick, dim3(1), dim3(256), 0, stream, st, shift);
    }
    hipLaunchKernelGGL(sel_out<T>, dim3(1), dim3(1), 0, stream, st, out);
    return hipGetLastError();
}

hipError_t launch_select(const void* x, int x_f64, int square, int64_t m, int64_t rank, void* tmp,
                         double* out_dev, hipStream_t stream) {
    if (m < 1 || rank < 0 || rank >= m) return hipErrorInvalidValue;
    if (x_f64) return run_select<double>((const double*)x, square, m, rank, (SelState*)tmp, out_dev, stream);
    return run_select<float>((const float*)x, square, m, rank, (SelState*)tmp, out_dev, stream);
}

}  // namespace symnmf
