// Order statistics on the device: MSB-first radix selection on IEEE bit
// patterns (for non-negative values the unsigned bit pattern orders like the
// value).  Used for median(g^2) of the Piecewise AdaGrad reset (appendix,
// Piecewise AdaGrad) and for the radial threshold of the TPDM exceedances.
//
// Pass d (8 bits per pass, from the top) histograms the digit of the keys that
// match the prefix fixed so far, then one thread walks the histogram to the
// bin holding the target rank, extends the prefix and rebases the rank.
#include <mutex>

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
    if (m < 1 || m > SELECT_MAX_M || rank < 0 || rank >= m) return hipErrorInvalidValue;
    if (x_f64) return run_select<double>((const double*)x, square, m, rank, (SelState*)tmp, out_dev, stream);
    return run_select<float>((const float*)x, square, m, rank, (SelState*)tmp, out_dev, stream);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free median entry point (symnmf_median_sq_noalloc):
// a file-scope device array, one copy per GPU, kept until the process ends.
// In host code the symbol names a host-side stand-in, not device memory, so
// the host never passes it to a kernel: it uses the device address that
// hipGetSymbolAddress returns, fetched once per device (with that device
// current) when the first context on the device is created.
// ---------------------------------------------------------------------------
static_assert(sizeof(SelState) <= NOALLOC_SCRATCH_BYTES, "selection state must fit the scratch array");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[MAX_DEVICES] = {};
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_err[device];
}

void* noalloc_scratch(int device, hipError_t* err) {
    if (device < 0 || device >= MAX_DEVICES) {
        if (err) *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (err) *err = g_scratch_done[device] ? g_scratch_err[device] : hipErrorNotInitialized;
    return g_scratch_ptr[device];
}

}  // namespace symnmf
