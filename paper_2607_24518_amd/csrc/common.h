// Internal declarations shared by the HIP sources of the SymNMF library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <cstdlib>

#include "../../include/symnmf.h"

namespace symnmf {

// Row tile of S handled by one work unit / one update work-group, and the
// column chunk streamed per unit.  Storage pads rows and columns of S and the
// rows of H to multiples of these, so no kernel needs a bounds test on the
// streamed data.
constexpr int TR = 256;
constexpr int KC = 256;
constexpr int KMAX = 64;
// The update kernel works on row slices of SR = TR / SUBT rows (one
// work-group each); per-slice FP64 partials (Gram, trace, KKT) are indexed
// slice = SUBT * tile + sub.
constexpr int SUBT = 4;
constexpr int SR = TR / SUBT;
constexpr int64_t PAD = 256;

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Tiled storage of S (FP32, BF16, FP8).  S is cut into 256 x 256 tiles,
// stored tile after tile in (row tile, column chunk) order.  Inside a tile the
// elements appear in exactly the order the MFMA stream kernel consumes them:
// [wave wv 0..3][sub-step s][row group rg 0..3][lane l 0..63][E elements],
// where one lane holds E consecutive columns (16 bytes: E = 4 FP32, 8 BF16,
// 16 FP8) of row 64 wv + 16 rg + (l % 16), starting at column
// s (4E) + (l / 16) E.  Each wave instruction therefore reads 1 KB of
// contiguous memory and each wave streams 64 (FP32) / 32 / 16 KB sequentially
// per tile.  FP64 storage (parity runs) is plain row-major with leading
// dimension ld.
// ---------------------------------------------------------------------------
constexpr int64_t TILE_ELEMS = (int64_t)TR * KC;

__host__ __device__ inline int64_t tiled_offset(int64_t r, int64_t c, int64_t n_chunks, int E) {
    const int64_t R = r >> 8, C = c >> 8;
    const int rr = (int)(r & 255), cc = (int)(c & 255);
    const int wv = rr >> 6, rg = (rr >> 4) & 3, lr = rr & 15;
    const int W = 4 * E;
    const int NS = 256 / W;
    const int s = cc / W, lg = (cc % W) / E, e = cc % E;
    const int64_t in_tile = (((int64_t)(wv * NS + s) * 4 + rg) * 64 + (lg * 16 + lr)) * E + e;
    return (R * n_chunks + C) * TILE_ELEMS + in_tile;
}
inline int elems_per_16B(int32_t dtype) {
    return dtype == SYMNMF_S_FP32 ? 4 : (dtype == SYMNMF_S_BF16 ? 8 : 16);
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Storage conversions (round to nearest even)
// ---------------------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16_bits(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// OCP FP8 E4M3 (bias 7, no infinities, max 448, subnormal quantum 2^-9),
// saturating, round to nearest even.
__host__ __device__ inline uint8_t f32_to_fp8e4m3(float x) {
    uint8_t sign = (x < 0.0f || (x == 0.0f && __builtin_signbit(x))) ? 0x80 : 0;
    float a = __builtin_fabsf(x);
    if (!(a == a)) return 0x7f;                       // NaN
    if (a >= 448.0f) return sign | 0x7e;
    if (a < 0.015625f) {                              // below 2^-6: subnormal grid 2^-9
        float q = __builtin_rintf(a * 512.0f);        // 0..8 (8 = smallest normal, code 0x08)
        return sign | (uint8_t)q;
    }
    int e;
    float m = __builtin_frexpf(a, &e);                // a = m 2^e, m in [0.5, 1)
    float mant = __builtin_rintf((m * 2.0f - 1.0f) * 8.0f);   // 0..8
    int E = e - 1 + 7;
    if (mant >= 8.0f) { mant = 0.0f; E += 1; }
    uint32_t code = ((uint32_t)E << 3) | (uint32_t)mant;
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
}
__host__ __device__ inline float fp8e4m3_to_f32(uint8_t b) {
    int e = (b >> 3) & 15, m = b & 7;
    float v = e == 0 ? (float)m * (1.0f / 512.0f) : __builtin_ldexpf(1.0f + (float)m * 0.125f, e - 7);
    return (b & 0x80) ? -v : v;
}

template <typename T> __device__ inline double load_as_f64(const T* p);
template <> __device__ inline double load_as_f64<double>(const double* p) { return *p; }
template <> __device__ inline double load_as_f64<float>(const float* p) { return (double)*p; }
template <> __device__ inline double load_as_f64<uint16_t>(const uint16_t* p) { return (double)bf16_bits_to_f32(*p); }
template <> __device__ inline double load_as_f64<uint8_t>(const uint8_t* p) { return (double)fp8e4m3_to_f32(*p); }

// ---------------------------------------------------------------------------
// Work plan of one S.H pass.
//
// A pass covers "active" row tiles; active tile a streams the column-chunk
// list of its class (0..2), each chunk with weight 1 or 2 (the weight
// multiplies the H rows of that chunk, exactly).  Unit = (active tile, list
// position).  Units are numbered tile-major (active tile a owns units
// [unit_offset[a], unit_offset[a+1])) and split evenly over the Pe = min(P, U)
// persistent work-groups: WG w owns [w U / Pe, (w+1) U / Pe).  Every maximal
// run of one tile inside one WG's range writes one partial S.H tile at index
// (w + a) of the partial buffer; (w, a) -> w + a is one-to-one because the
// ranges are ordered, so the buffer needs at most (P + active tiles) tiles.
// The update kernel sums the partials of tile a in increasing w, so results
// do not depend on scheduling.
//
// The device-side plan lives in one int32 array (layout below) written by the
// plan kernel; a "full" pass (every tile, every chunk, weight 1) needs none of
// it.
// ---------------------------------------------------------------------------
struct PlanView {
    int32_t full;
    int32_t tall;             // full plans only: units are (pair of row tiles, chunk), see below
    int32_t n_tiles;          // row tiles of the stored panel
    int32_t n_chunks;         // column chunks (ld / KC)
    int32_t P;                // launched persistent work-groups
    // device arrays (unused when full)
    const int32_t* hdr;       // [0] n_active, [1] U lo, [2] U hi, [3] class_len[0..2] at 3..5
    const int32_t* active_tile;    // [n_tiles]
    const int32_t* active_class;   // [n_tiles]
    const int32_t* unit_offset;    // [n_tiles + 1]
    const int32_t* class_chunks;   // [3][n_chunks]
    const int32_t* class_weight;   // [3][n_chunks]
    const int32_t* tile_active;    // [n_tiles] active index or -1
};

// int32 words of the device plan for given sizes
inline int64_t plan_words(int64_t n_tiles, int64_t n_chunks) {
    return 8 + 3 * n_tiles + 1 + 6 * n_chunks + n_tiles;
}
inline PlanView plan_view(int32_t* base, int32_t full, int32_t n_tiles, int32_t n_chunks, int32_t P) {
    PlanView v;
    v.full = full; v.tall = 0; v.n_tiles = n_tiles; v.n_chunks = n_chunks; v.P = P;
    v.hdr = base;
    v.active_tile = base + 8;
    v.active_class = v.active_tile + n_tiles;
    v.unit_offset = v.active_class + n_tiles;
    v.class_chunks = v.unit_offset + n_tiles + 1;
    v.class_weight = v.class_chunks + 3 * n_chunks;
    v.tile_active = v.class_weight + 3 * n_chunks;
    return v;
}

// Tall full plans: a unit is (pair q of row tiles 2q and 2q+1, chunk), streamed
// by one 8-wave work-group whose two halves share the chunk image; the partial
// of tile 2q + h from work-group w goes to index 2 (w + q) + h (one-to-one for
// the same reason as above), so the buffer needs 2 (P + pairs) tiles.
__host__ __device__ inline int64_t tall_pairs(int64_t n_tiles) { return (n_tiles + 1) / 2; }

// Work-groups of a tall full pass: one per CU, except that when a whole
// number m of work-groups per tile pair fills at least 95 % of the CUs the
// pass uses exactly pairs * m.  The contiguous unit ranges then split every
// pair into the same m chunk segments, so all work-groups walk the same m
// chunk positions at the same time and the H images they stage are served
// from L2 / MALL instead of being fetched from HBM once per pair
// (SYMNMF_TALL_ALIGN=0 turns this off).
inline int32_t tall_wgs(int cus, int64_t n_tiles) {
    const int64_t pairs = tall_pairs(n_tiles);
    const char* e = std::getenv("SYMNMF_TALL_ALIGN");
    if (pairs <= cus && !(e && e[0] == '0')) {
        const int64_t m = cus / pairs;
        if (20 * pairs * m >= 19 * (int64_t)cus) return (int32_t)(pairs * m);
    }
    return cus;
}

__host__ __device__ inline int64_t wg_start(int64_t w, int64_t U, int64_t Pe) { return w * U / Pe; }
// the work-group whose range holds unit u
__host__ __device__ inline int64_t wg_owner(int64_t u, int64_t U, int64_t Pe) { return ((u + 1) * Pe - 1) / U; }

__device__ inline int64_t upd_unit_off(const PlanView& p, int32_t a) {
    return p.full ? (int64_t)a * p.n_chunks : (int64_t)p.unit_offset[a];
}

// The S.H partial tiles of active tile act: index (w + act), or 2 (w + pair) +
// half for tall full plans, over the work-groups w_lo..w_hi that streamed its
// units (none when act < 0).
__device__ inline void partial_slots(const PlanView& p, int32_t act, int64_t& w_lo, int64_t& w_hi,
                                     int64_t& slot_base, int64_t& slot_mul) {
    w_lo = 0;
    w_hi = -1;
    slot_base = act;
    slot_mul = 1;
    if (act < 0) return;
    int64_t U;
    if (p.full && p.tall) {
        const int64_t q = act >> 1;
        U = tall_pairs(p.n_tiles) * p.n_chunks;
        const int64_t Pe = U < p.P ? U : p.P;
        w_lo = wg_owner(q * p.n_chunks, U, Pe);
        w_hi = wg_owner((q + 1) * p.n_chunks - 1, U, Pe);
        slot_base = 2 * q + (act & 1);
        slot_mul = 2;
    } else {
        if (p.full) U = (int64_t)p.n_tiles * p.n_chunks;
        else U = (int64_t)(uint32_t)p.hdr[1] | ((int64_t)p.hdr[2] << 32);
        const int64_t Pe = U < p.P ? U : p.P;
        w_lo = wg_owner(upd_unit_off(p, act), U, Pe);
        w_hi = wg_owner(upd_unit_off(p, act + 1) - 1, U, Pe);
    }
}

// SplitMix64 (Steele, Lea & Flood 2014): output number c of the stream keyed s.
__host__ __device__ inline uint64_t splitmix64(uint64_t key, uint64_t c) {
    uint64_t z = key + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline double uniform24(uint64_t key, uint64_t c) {
    return (double)(splitmix64(key, c) >> 40) * (1.0 / 16777216.0);
}

// Index-set sampler of the stochastic variants: m distinct blocks of
// [0, nb) by a partial Fisher-Yates shuffle (Knuth, TAOCP 2, Algorithm P)
// driven by the SplitMix64 stream keyed by (seed, 2t + stream); flags[b] = 1
// for the chosen blocks.  perm: nb ints of scratch.
__host__ __device__ inline void sample_block_flags(uint64_t seed, int64_t t, int stream, int nb, int m,
                                                   int32_t* perm, uint8_t* flags) {
    const uint64_t key = splitmix64(seed, (uint64_t)(2 * t + stream));
    for (int i = 0; i < nb; ++i) perm[i] = i;
    for (int i = 0; i < m; ++i) {
        const double u = uniform24(key, (uint64_t)i);
        const int j = i + (int)(u * (double)(nb - i));
        const int32_t tmp = perm[i];
        perm[i] = perm[j];
        perm[j] = tmp;
    }
    for (int i = 0; i < nb; ++i) flags[i] = 0;
    for (int i = 0; i < m; ++i) flags[perm[i]] = 1;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// stream.hip: partial S.H of every active tile.  S: rows_pad x ld of stype;
// H: global rows, n_pad x k (h_f64: double); part: (P + n_tiles) * TR * k of
// the accumulation type (acc_f64: double).  Returns hipErrorInvalidValue for
// combinations without a kernel.
// MFMA kernels (stream_uses_mfma) read H through chunk images instead of H:
// img1 = images of H, img2 = images of 2H (block steps; may equal img1 otherwise).
hipError_t launch_stream(const void* S, int32_t stype, int64_t ld, const void* H, int h_f64, int64_t k,
                         void* part, int acc_f64, const PlanView& plan, hipStream_t stream,
                         const void* img1 = nullptr, const void* img2 = nullptr);
// 32-bit words of the H images of all n_chunks chunks for this storage type and rank
int64_t h_image_words(int32_t stype, int64_t k, int64_t n_chunks);
// Write the chunk images of wt * H (H: n_chunks * 256 rows x k, FP32).
hipError_t launch_h_image(const float* H, int32_t stype, int64_t k, int64_t n_chunks, float wt, uint32_t* img,
                          hipStream_t stream);
hipError_t launch_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t stream);
// plain read of bytes (multiple of 16); sink: sink_words words (>= 4), one per wave
hipError_t launch_read_probe(const void* src, int64_t bytes, uint32_t* sink, int64_t sink_words,
                             hipStream_t stream);
// Objective pass on the MFMA path: FP32 sums within each 256-column chunk,
// FP64 across chunks; FP64 partials.  img: chunk images of FP32 H.
int stream_acc64_supported(int32_t stype, int64_t k);
hipError_t launch_stream_acc64(const void* S, int32_t stype, int64_t k, const void* img, double* part,
                               const PlanView& p, hipStream_t stream);
int stream_uses_mfma(int32_t stype, int h_f64, int acc_f64, int64_t k);
// resident work-groups per CU of the stream kernel for this storage and rank
int stream_wgs_per_cu(int32_t stype, int64_t k);
// whether full steps of this storage and rank run the tall (8-wave) kernel
int stream_tall_supported(int32_t stype, int h_f64, int64_t k);

// plan.hip: build the device plan of a sub-sampled step.
struct PlanRequest {
    int32_t mode;            // 1 = row SVRG (I only), 2 = block SVRG
    int32_t n_tiles, n_chunks, tiles_per_block, chunks_per_block, n_blocks;
    int32_t m;               // sampled blocks per set
    int32_t independent;
    uint64_t seed;
    int64_t t;
};
hipError_t launch_plan(const PlanRequest& r, int32_t* plan_base, int32_t* tiles_I, int32_t* tiles_J,
                       int32_t* counts, hipStream_t stream);

struct UpdateArgs {
    int64_t rows, rows_pad, n, k;           // panel rows, padded rows, instruments, rank
    int64_t row0;                           // global row of panel row 0
    int32_t method, softplus;
    double eta, eps, alpha, mu;
    const void* H;        // H_t   (n_pad x k, global rows)
    void* Hn;             // H_{t+1}
    void* G;              // AdaGrad G / RMSprop v   (rows_pad x k, panel rows)
    void* M;              // RMSprop momentum
    void* Theta;          // softplus parameter
    void* Mu;             // snapshot gradient (SVRG), may be null
    void* Gout;           // gradient of this step, may be null
    const void* part;     // S.H partials
    const void* gram_eff; // [3][k][k] effective Gram per class (state precision)
    double cgrad;         // 4 (full / row steps) or 2 (block steps)
    int32_t store_mu;     // full SVRG step: mu <- g
    int32_t fp8;          // FP8 storage: scale partials, add the diagonal back
    int32_t block_step;   // Block-SVRG sampled step: the diagonal term S_ii h_i carries the
                          // weight of column i's chunk for the row's class (0, 0, 2)
    const float* panel_scale;
    const float* diag;    // FP8: S_ii of every panel row
    int64_t panel_rows;
    double* tile_gram;    // [tiles][k][k] Gram of H_{t+1} rows
    double* tile_tr;      // [tiles] sum H_t * SH_t
    double* tile_kkt;     // [tiles] sum proj(g)^2
    int32_t* tile_bad;    // [tiles] non-finite gradient count
    double rho;           // ADMM consensus penalty
    void* minv;           // ADMM: (2 W^T W + rho I)^-1, k x k (state precision)
    double beta1, beta2, beta3;   // Adam / NAdam / Adan decays
    double bc1, bc2, bc3;         // 1 - beta^(t+1): bias corrections of this step
    int32_t first;                // first step (Adan: zero gradient difference)
    void* D;              // Adan average of gradient differences
    void* Gp;             // Adan previous gradient
};
hipError_t launch_update(const UpdateArgs& a, int h_f64, const PlanView& plan, hipStream_t stream);
// ADMM step (full plans): the k x k inverse from the FP64 Gram of W_t, then the
// fused statistics + H / W / U update (a.M holds U).
hipError_t launch_admm(const UpdateArgs& a, const double* gram64, int h_f64, const PlanView& plan,
                       hipStream_t stream);

// Per-slice FP64 Gram partials (SUBT per tile) of rows [row0, row0 + tiles*TR) of H.
hipError_t launch_tile_gram(const void* H, int h_f64, int64_t row0, int64_t rows, int64_t tiles, int64_t k,
                            double* tile_gram, hipStream_t stream);
// FP64 Gram of the rows of [0, n) outside [skip_lo, skip_hi).
hipError_t launch_gram_rows(const void* H, int h_f64, int64_t n, int64_t skip_lo, int64_t skip_hi, int64_t k,
                            double* out, hipStream_t stream);

// Reduce tile partials: Gram_{t+1} (gram_next64, and gram_eff = 3 copies in
// state precision), and the statistics of H_t: stats[0] = tr(H^T S H),
// [1] = ||grad_proj||^2, [2] = non-finite count, [3] = ||Gram_t||_F^2.
hipError_t launch_finalize(int64_t tiles, int64_t k, const double* tile_gram, const double* tile_tr,
                           const double* tile_kkt, const int32_t* tile_bad, const double* gram_fixed,
                           const double* gram_cur64, double* gram_next64, void* gram_eff, int h_f64,
                           double* stats, hipStream_t stream);

// Effective Gram matrices of a block step: out[0] = Gram_J, out[1] = Gram_I,
// out[2] = Gram_I + Gram_J from per-tile Gram partials of H_t.
hipError_t launch_gram_select(int64_t k, const double* tile_gram, const int32_t* tiles_I,
                              const int32_t* tiles_J, const int32_t* counts, void* gram_eff, int h_f64,
                              hipStream_t stream);

hipError_t launch_init_H(float* H, int64_t n, int64_t k, uint64_t seed, float scale, hipStream_t stream);
hipError_t launch_copy_h(const void* src, int src_f64, void* dst, int dst_f64, int64_t count, hipStream_t stream);
// Zero `bytes` bytes at p on `stream` with a kernel (no memset node).
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream);
hipError_t launch_softplus_init(void* H, void* Theta, int h_f64, int64_t count, hipStream_t stream);
hipError_t launch_sum(const void* x, int x_f64, int64_t m, double* out, hipStream_t stream);
hipError_t launch_piecewise_apply(void* G, const void* g, int h_f64, int64_t m, double c, const double* med,
                                  hipStream_t stream);

// select.hip: element number ``rank`` (0-based, ascending) of the keys x_i^2
// (square = 1) or x_i (square = 0; x_i >= 0 required) over m values, by an
// MSB-first radix selection on the IEEE bit patterns (monotone for
// non-negative values).  The value goes to out_dev[0] (double).  tmp: device
// scratch of select_tmp_bytes().
int64_t select_tmp_bytes();
// the histogram counters are 32-bit: at most 2^32 - 1 values per selection
constexpr int64_t SELECT_MAX_M = 0xffffffffll;
hipError_t launch_select(const void* x, int x_f64, int square, int64_t m, int64_t rank, void* tmp,
                         double* out_dev, hipStream_t stream);

// Allocation-free entry points: the device address of the file-scope scratch
// array of select.hip on ``device``.  noalloc_scratch_init (device current)
// looks it up once per device; noalloc_scratch returns it (null and *err set
// when the lookup failed or was never made).
constexpr int64_t NOALLOC_SCRATCH_BYTES = 4096;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device, hipError_t* err);

// build_s.hip
struct BuildOut {
    void* data; float* scale; float* diag;
    int64_t rows, rows_pad, ld, n, row0; int32_t dtype; int64_t panel_rows;
};
// Flag bits set by the input checks of the S build: a non-finite X entry, a
// negative entry where raw TPDM marginals need X >= 0; the low bits count
// zero-variance columns.
constexpr int32_t BAD_NONFINITE = 1 << 30;
constexpr int32_t BAD_NEGATIVE = 1 << 29;
hipError_t launch_check_input(const float* X, int64_t count, float sign, int32_t* flag, hipStream_t stream);
hipError_t launch_standardise(const float* X, int64_t T, int64_t n, void* Z, int z_f64, int64_t ldz, int32_t* bad,
                              hipStream_t stream);
// TPDM: Omega (n_exc x ldz, FP32 or FP64) = column-normalised angular rows.
hipError_t launch_tpdm_omega(const float* X, int64_t T, int64_t n, int lower, int raw, void* Omega, int z_f64,
                             int64_t ldz, int64_t n_exc, void* work, hipStream_t stream);
int64_t tpdm_work_bytes(int64_t T, int64_t n, int raw);
// sums: device FP64 array of syrk_sum_words(o) words; [0..2] = sum S, sum S^2,
// sum S_stored^2 on return.  panel_max: FP8 only, zeroed, one word per panel.
int64_t syrk_sum_words(const BuildOut& o);
hipError_t launch_syrk_store(const void* Z, int z_f64, int64_t K, int64_t ldz, const BuildOut& o, double* sums,
                             uint32_t* panel_max, hipStream_t stream);
// The same product for BF16 / FP8 storage on the bf16 matrix cores with Z
// split into two bf16 planes; ws holds the planes (syrk_split_ws_bytes).
// Z: Kpad x ldz FP32 with K valid rows.
int64_t syrk_split_ws_bytes(int64_t K, int64_t ldz);
hipError_t launch_syrk_split_store(const float* Z, int64_t K, int64_t ldz, const BuildOut& o, double* sums,
                                   uint32_t* panel_max, void* ws, hipStream_t stream);
// sums: 4 + 3 * rows_pad words
hipError_t launch_store_dense(const void* src, int src_f64, const BuildOut& o, double* sums,
                              uint32_t* panel_max, hipStream_t stream);
hipError_t launch_fp8_decode_check(int32_t* bad, hipStream_t stream);
// objective pass: per-tile tr(H^T S H) partial and Gram of H (FP64 H).
hipError_t launch_objective_tiles(const UpdateArgs& a, const PlanView& plan, hipStream_t stream);

// warmstart.hip
hipError_t launch_omega(uint64_t seed, int64_t n, int64_t rows_alloc, int w, float* out, hipStream_t stream);
// dense FP32 S.H rows (rows x k) from the partials of a full FP32-accumulating stream pass
hipError_t launch_sh_dense(const float* part, int64_t rows, int64_t rows_pad, int64_t k, int32_t n_chunks, int32_t P,
                           const float* H, int64_t row0, const float* scale, const float* diag, int64_t panel_rows,
                           float* out, hipStream_t stream);
// C = alpha op(A) op(B) + bias with epilogue (0 none, 1 GELU, 2 softplus); Z: pre-epilogue copy
// or null.  split_ws (split_ws_floats floats, may be null) enables split-K for small outputs.
hipError_t launch_gemm(int ta, int tb, int b_bf16, int epi, const float* A, const void* B, const float* bias, float* C,
                       float* Z, int64_t M, int64_t N, int64_t K, float alpha, float* split_ws,
                       int64_t split_ws_floats, hipStream_t stream);
// dZ = dA * f'(Z): mode 1 GELU, mode 2 softplus
hipError_t launch_act_backward(const float* dA, const float* Z, float* dZ, int64_t m, int mode, hipStream_t stream);
hipError_t launch_colsum(const float* X, int64_t m, int64_t ncol, float* out, hipStream_t stream);
// residual output A = max(C + z, 0) (A holds z on entry; C = first k columns of X) and its backward
hipError_t launch_residual_relu(const float* X, int64_t ldx, float* A, int64_t rows, int64_t k, hipStream_t stream);
hipError_t launch_residual_relu_backward(const float* dA, const float* X, int64_t ldx, const float* Z, float* dZ,
                                         int64_t rows, int64_t k, hipStream_t stream);
hipError_t launch_adamw(float* P, const float* G, float* M, float* V, int64_t m, int64_t n_decay, float lr, float b1,
                        float b2, float eps, float wd, int64_t t, hipStream_t stream);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t m, hipStream_t stream);
// successive projection on R (m x k FP64, destroyed); pick: k device int64; bval/bidx: nb entries
hipError_t launch_spa(double* R, int64_t m, int64_t k, double* bval, int64_t* bidx, int nb, int64_t* pick,
                      hipStream_t stream);
int64_t xty_work_doubles(int64_t m, int64_t kx, int64_t ky);
hipError_t launch_xty(const float* X, int64_t ldx, int64_t kx, const float* Y, int64_t ldy, int64_t ky, int64_t m,
                      double* work, double* out, hipStream_t stream);
hipError_t launch_jacobi_topk(const double* G, int64_t w, int64_t k, double* V, double* M, double* lam,
                              int32_t* status, hipStream_t stream);
hipError_t launch_project_rows(const float* Y, int64_t m, int64_t w, const double* W, int64_t k, int64_t ldo,
                               int out_f64, void* out, hipStream_t stream);
hipError_t launch_anchor_solve(const float* Y, int64_t w, const double* M, int64_t k, const int64_t* anchors,
                               double* W, int32_t* status, hipStream_t stream);
hipError_t launch_gram_loss_grad(const float* A, const float* B, const double* AtA, const double* AtB, int64_t k,
                                 int64_t m, float ca, float cb, float* dA, hipStream_t stream);
hipError_t launch_clip_cols(const float* X, int64_t m, int64_t w, int64_t k, float* out, hipStream_t stream);
hipError_t launch_scale(float* x, int64_t m, float a, hipStream_t stream);
hipError_t launch_span_overlap(const double* MA, const double* AtB, const double* MB, int64_t k, double* out,
                               hipStream_t stream);

}  // namespace symnmf
