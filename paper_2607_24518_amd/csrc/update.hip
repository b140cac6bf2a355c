// Fused gradient + optimiser update of one iteration, and the FP64 reductions
// behind the objective and the stop rule.
//
// For every row tile of the panel the update kernel
//   * sums the S.H partials of the tile (stream kernel output) - or, for a
//     row the step did not sample, takes the snapshot gradient mu,
//   * forms g = c_g (H (Gram_eff) - S H) with the k x k Gram in LDS
//     (paper: grad f = 4 (H (H^T H) - S H), H (H^T H) formed right to left;
//     block steps: c_g = 2 with the block Gram, appendix Block-SVRG),
//   * applies the AdaGrad / RMSprop rule in projected or softplus form
//     (appendix family 3; eq. logspace_grad for softplus),
//   * writes H_{t+1} and accumulates in FP64 the per-tile partials of
//     tr(H_t^T S H_t), ||grad_proj||^2 (eq. proj_grad) and Gram(H_{t+1}).
// The finalize kernel reduces the tile partials in a fixed order.
#include "common.h"

namespace symnmf {

template <typename T> __device__ inline T dev_sqrt(T x);
template <> __device__ inline float dev_sqrt<float>(float x) { return __builtin_sqrtf(x); }
template <> __device__ inline double dev_sqrt<double>(double x) { return __builtin_sqrt(x); }

// softplus(x) = max(x, 0) + log1p(exp(-|x|)); sigmoid(x) = 1 / (1 + exp(-x))
__device__ inline float softplus_f(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ inline double softplus_f(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }
__device__ inline float sigmoid_f(float x) { return 0.5f * (1.0f + tanhf(0.5f * x)); }
__device__ inline double sigmoid_f(double x) { return 0.5 * (1.0 + tanh(0.5 * x)); }

__device__ inline double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;   // valid in thread 0
}

constexpr int UT = 256;   // threads of the update work-group (one row slice of SR rows)

template <typename HT, int KB>
__global__ __launch_bounds__(UT, sizeof(HT) == 4 ? 7 : 1) void update_kernel(UpdateArgs a, PlanView p) {
    __shared__ __align__(32) HT Hs[SR * KB];
    __shared__ __align__(32) HT Hns[SR * KB];
    __shared__ HT Gs[KB * KB];
    __shared__ double red[UT / 64];
    const int t = threadIdx.x;
    const int64_t slice = blockIdx.x;
    const int64_t tile = slice / SUBT;
    const int r0 = (int)(slice % SUBT) * SR;           // first tile row of the slice
    const int k = (int)a.k;
    const int32_t act = p.full ? (int32_t)tile : p.tile_active[tile];
    const int cls = (act >= 0 && !p.full) ? p.active_class[act] : 0;
    const HT* gram = (const HT*)a.gram_eff + (int64_t)cls * k * k;
    for (int e = t; e < k * k; e += UT) Gs[(e / k) * KB + e % k] = gram[e];
    const int64_t g0 = a.row0 + tile * TR + r0;       // global row of slice row 0
    const HT* Ht = (const HT*)a.H;
    for (int f = t; f < SR * k; f += UT) Hs[(f / k) * KB + f % k] = Ht[g0 * k + f];
    __syncthreads();

    int64_t w_lo, w_hi, slot_base, slot_mul;
    partial_slots(p, act, w_lo, w_hi, slot_base, slot_mul);
    const HT* part = (const HT*)a.part;
    HT* G = (HT*)a.G;
    HT* M = (HT*)a.M;
    HT* Th = (HT*)a.Theta;
    HT* Mu = (HT*)a.Mu;
    HT* Go = (HT*)a.Gout;
    HT* Hn = (HT*)a.Hn;
    const HT eta = (HT)a.eta, eps = (HT)a.eps, alpha = (HT)a.alpha, mom = (HT)a.mu, cg = (HT)a.cgrad;
    // H (H^T H) of this thread's elements.  With k == KB the elements
    // f = t + UT j of a thread share the column c = t % KB (UT is a multiple
    // of KB), so every Gram entry is read from LDS once for all of them and
    // the H rows in 4-wide vectors; the products are summed in the same order
    // as the per-element loop below.
    constexpr int NJ = SR * KB / UT;
    typedef HT hvec4 __attribute__((ext_vector_type(4)));
    const bool full_k = k == KB && act >= 0;
    HT hgv[NJ];
    if (full_k) {
        const int c = t % KB, rb = t / KB;
#pragma unroll
        for (int j = 0; j < NJ; ++j) hgv[j] = 0;
        for (int b = 0; b < KB; b += 4) {
            const HT g0 = Gs[b * KB + c], g1 = Gs[(b + 1) * KB + c], g2 = Gs[(b + 2) * KB + c],
                     g3 = Gs[(b + 3) * KB + c];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const hvec4 hv = *(const hvec4*)&Hs[(rb + j * (UT / KB)) * KB + b];
                HT v = hgv[j];
                v += hv[0] * g0;
                v += hv[1] * g1;
                v += hv[2] * g2;
                v += hv[3] * g3;
                hgv[j] = v;
            }
        }
    }
    // the S.H partials of this thread's elements, summed over the writing
    // work-groups in increasing order as below, but with the loads of all
    // elements of one work-group issued together (a row of the n = 10^6 share
    // has ten partials: one after another they are ten dependent load latencies
    // per element)
    HT shv[NJ];
    if (full_k) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) shv[j] = 0;
        for (int64_t w = w_lo; w <= w_hi; ++w) {
            // element f = r k + c of the slice: its partial entry is f past the
            // slot's first row of this slice
            const HT* pw = part + ((slot_mul * w + slot_base) * TR + r0) * (int64_t)k;
#pragma unroll
            for (int j = 0; j < NJ; ++j) shv[j] += pw[t + UT * j];
        }
    }
    double tr = 0.0, kkt = 0.0;
    int bad = 0;
    // one element f = r k + c of the slice; with full_k its S.H sum and
    // H (H^T H) entry come in precomputed (sh_in, hg_in)
    auto element = [&](int f, HT sh_in, HT hg_in) {
        const int r = f / k, c = f - r * k;             // slice row, column
        const int64_t prow = tile * TR + r0 + r;
        HT hn = 0;
        if (prow < a.rows) {
            const HT h = Hs[r * KB + c];
            const int64_t idx = prow * k + c;
            HT g, sh = 0, hg = 0;
            if (act >= 0) {
                if (full_k) {
                    sh = sh_in;
                } else {
                    for (int64_t w = w_lo; w <= w_hi; ++w)
                        sh += part[((slot_mul * w + slot_base) * TR + r0 + r) * (int64_t)k + c];
                }
                if (a.fp8) {   // codes carry S * scale off the diagonal; S_ii is kept exactly
                    // and enters with the weight the plan gives column i of this row:
                    // 1 on full and row-sampled steps; on a block step 0 for rows in I
                    // only or J only (their own block is not among the streamed
                    // chunks) and 2 for rows in both sets
                    const HT dw = (p.full || !a.block_step) ? (HT)1 : (cls == 2 ? (HT)2 : (HT)0);
                    sh = sh / (HT)a.panel_scale[prow / a.panel_rows] + dw * (HT)a.diag[prow] * h;
                }
                if (full_k) {
                    hg = hg_in;
                } else {
                    for (int b = 0; b < k; ++b) hg += Hs[r * KB + b] * Gs[b * KB + c];
                }
                g = cg * (hg - sh);
                tr += (double)h * (double)sh;
            } else {
                g = Mu[idx];
            }
            const HT pg = a.softplus ? g : (h > (HT)0 ? g : (g < (HT)0 ? g : (HT)0));
            kkt += (double)pg * (double)pg;
            if (!(g == g) || g - g != (HT)0) ++bad;
            if (a.store_mu) Mu[idx] = g;
            if (Go) Go[idx] = g;
            if (a.method == SYMNMF_ADAM || a.method == SYMNMF_NADAM || a.method == SYMNMF_ADAN) {
                // family 3, Adam-type rules on x = Theta (softplus) or H (projected)
                const HT x = a.softplus ? Th[idx] : h;
                const HT gx = a.softplus ? g * sigmoid_f(x) : g;
                const HT b1 = (HT)a.beta1, b2 = (HT)a.beta2;
                const HT m = b1 * M[idx] + ((HT)1 - b1) * gx;
                M[idx] = m;
                HT step;
                if (a.method == SYMNMF_ADAN) {
                    const HT b3 = (HT)a.beta3;
                    HT* D = (HT*)a.D;
                    HT* Gp = (HT*)a.Gp;
                    const HT diff = a.first ? (HT)0 : gx - Gp[idx];
                    const HT d = b2 * D[idx] + ((HT)1 - b2) * diff;
                    const HT u = gx + b2 * diff;
                    const HT nv = b3 * G[idx] + ((HT)1 - b3) * u * u;
                    D[idx] = d;
                    G[idx] = nv;
                    Gp[idx] = gx;
                    step = (m / (HT)a.bc1 + b2 * d / (HT)a.bc2) / (dev_sqrt(nv / (HT)a.bc3) + eps);
                } else {
                    const HT v = b2 * G[idx] + ((HT)1 - b2) * gx * gx;
                    G[idx] = v;
                    HT mh = m / (HT)a.bc1;
                    if (a.method == SYMNMF_NADAM) mh = b1 * mh + ((HT)1 - b1) * gx / (HT)a.bc1;
                    step = mh / (dev_sqrt(v / (HT)a.bc2) + eps);
                }
                const HT xn = x - eta * step;
                if (a.softplus) {
                    Th[idx] = xn;
                    hn = softplus_f(xn);
                } else {
                    hn = xn > (HT)0 ? xn : (HT)0;
                }
            } else if (a.method == SYMNMF_MU) {
                // family 1: dampened multiplicative update, H stays >= 0
                hn = (HT)0.5 * h * ((HT)1 + sh / (hg + eps));
            } else if (a.softplus) {
                HT th = Th[idx];
                const HT gt = g * sigmoid_f(th);
                if (a.method == SYMNMF_RMSPROP) {
                    const HT v = alpha * G[idx] + ((HT)1 - alpha) * gt * gt;
                    const HT m = mom * M[idx] + eta * gt / (dev_sqrt(v) + eps);
                    G[idx] = v;
                    M[idx] = m;
                    th -= m;
                } else {
                    const HT acc = G[idx] + gt * gt;
                    G[idx] = acc;
                    th -= eta * gt / (dev_sqrt(acc) + eps);
                }
                Th[idx] = th;
                hn = softplus_f(th);
            } else if (a.method == SYMNMF_RMSPROP) {
                const HT v = alpha * G[idx] + ((HT)1 - alpha) * g * g;
                const HT m = mom * M[idx] + eta * g / (dev_sqrt(v) + eps);
                G[idx] = v;
                M[idx] = m;
                hn = h - m;
                hn = hn > (HT)0 ? hn : (HT)0;
            } else {
                const HT acc = G[idx] + g * g;
                G[idx] = acc;
                hn = h - eta * g / (dev_sqrt(acc) + eps);
                hn = hn > (HT)0 ? hn : (HT)0;
            }
            Hn[(g0 + r) * k + c] = hn;
        }
        Hns[r * KB + c] = hn;
    };
    if (full_k) {
        // the thread's elements f = t + UT j with compile-time j, so the
        // precomputed sums stay in registers
#pragma unroll
        for (int j = 0; j < NJ; ++j) element(t + UT * j, shv[j], hgv[j]);
    } else {
        for (int f = t; f < SR * k; f += UT) element(f, (HT)0, (HT)0);
    }
    __syncthreads();
    double* tg = a.tile_gram + slice * (int64_t)k * k;
    if (KB >= 32 && k == KB) {
        // each thread: entries (ia0 + q, ib), q < NQ (a multiple of 4, ia0 too),
        // consecutive ia read as aligned 4-wide vectors; the same FP64 sums
        // over the slice rows
        constexpr int NQ = KB >= 32 ? (KB * KB) / UT : 4;
        static_assert(NQ % 4 == 0, "4-wide Gram reads need NQ % 4 == 0");
        const int ib = t % KB, ia0 = (t / KB) * NQ;
        double sq[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sq[q] = 0.0;
        for (int r = 0; r < SR; ++r) {
            const double hb = (double)Hns[r * KB + ib];
#pragma unroll
            for (int q = 0; q < NQ; q += 4) {
                const hvec4 hv = *(const hvec4*)&Hns[r * KB + ia0 + q];
#pragma unroll
                for (int e = 0; e < 4; ++e) sq[q + e] += (double)hv[e] * hb;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) tg[(ia0 + q) * k + ib] = sq[q];
    } else {
        for (int e = t; e < k * k; e += UT) {
            const int ia = e / k, ib = e - ia * k;
            double s = 0.0;
            for (int r = 0; r < SR; ++r) s += (double)Hns[r * KB + ia] * (double)Hns[r * KB + ib];
            tg[e] = s;
        }
    }
    const double str = block_sum(tr, red);
    const double skk = block_sum(kkt, red);
    const double sbad = block_sum((double)bad, red);
    if (t == 0) {
        a.tile_tr[slice] = str;
        a.tile_kkt[slice] = skk;
        a.tile_bad[slice] = (int32_t)sbad;
    }
}

hipError_t launch_update(const UpdateArgs& a, int h_f64, const PlanView& p, hipStream_t stream) {
    const int64_t tiles = a.rows_pad / TR;
    dim3 grid(tiles * SUBT), block(UT);
    if (h_f64) {
        if (a.k <= 8) hipLaunchKernelGGL((update_kernel<double, 8>), grid, block, 0, stream, a, p);
        else if (a.k <= 16) hipLaunchKernelGGL((update_kernel<double, 16>), grid, block, 0, stream, a, p);
        else if (a.k <= 32) hipLaunchKernelGGL((update_kernel<double, 32>), grid, block, 0, stream, a, p);
        else return hipErrorInvalidValue;
    } else {
        if (a.k <= 8) hipLaunchKernelGGL((update_kernel<float, 8>), grid, block, 0, stream, a, p);
        else if (a.k <= 16) hipLaunchKernelGGL((update_kernel<float, 16>), grid, block, 0, stream, a, p);
        else if (a.k <= 32) hipLaunchKernelGGL((update_kernel<float, 32>), grid, block, 0, stream, a, p);
        else hipLaunchKernelGGL((update_kernel<float, 64>), grid, block, 0, stream, a, p);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ADMM (appendix family 6).  Per step: the inverse of M = 2 W^T W + rho I (k x k,
// FP64 Gauss-Jordan in one work-group; M is symmetric positive definite, so
// no pivoting), then one fused pass over the rows of the panel that sums the
// S.W partials and, per row,
//   * records the statistics of W_t: tr partial W . SW, the projected gradient
//     of g = 4 (W (W^T W) - S W) (the stop rule is taken on W),
//   * a = 2 SW + rho (W - U) and H = a M^-1 (eq. admm_H),
//   * W_{t+1} = [H + U]_+ (eq. admm_W), U <- U + H - W_{t+1} (eq. admm_U),
//   * the FP64 Gram partials of W_{t+1}.
// ---------------------------------------------------------------------------
template <typename HT>
__global__ __launch_bounds__(256) void admm_minv_kernel(const double* __restrict__ gram, int k, double rho,
                                                        HT* __restrict__ minv) {
    __shared__ double A[KMAX * 2 * KMAX];
    __shared__ double fac[KMAX];
    const int t = threadIdx.x, w2 = 2 * k;
    for (int e = t; e < k * w2; e += 256) {
        const int i = e / w2, j = e - i * w2;
        A[e] = j < k ? 2.0 * gram[i * k + j] + (i == j ? rho : 0.0) : (j - k == i ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int piv = 0; piv < k; ++piv) {
        const double d = A[piv * w2 + piv];
        __syncthreads();
        for (int j = t; j < w2; j += 256) A[piv * w2 + j] /= d;
        __syncthreads();
        for (int i = t; i < k; i += 256) fac[i] = A[i * w2 + piv];
        __syncthreads();
        for (int e = t; e < k * w2; e += 256) {
            const int i = e / w2, j = e - i * w2;
            if (i != piv) A[e] -= fac[i] * A[piv * w2 + j];
        }
        __syncthreads();
    }
    for (int e = t; e < k * k; e += 256) minv[e] = (HT)A[(e / k) * w2 + k + e % k];
}

template <typename HT, int KB>
__global__ __launch_bounds__(UT) void admm_update_kernel(UpdateArgs a, PlanView p) {
    __shared__ __align__(32) HT Ws[SR * KB];
    __shared__ __align__(32) HT Wns[SR * KB];
    __shared__ __align__(32) HT As[SR * KB];
    __shared__ HT Gs[KB * KB];
    __shared__ HT Ms[KB * KB];
    __shared__ double red[UT / 64];
    const int t = threadIdx.x;
    const int64_t slice = blockIdx.x;
    const int64_t tile = slice / SUBT;
    const int r0 = (int)(slice % SUBT) * SR;
    const int k = (int)a.k;
    const int32_t act = (int32_t)tile;                  // full steps only
    const HT* gram = (const HT*)a.gram_eff;
    const HT* minv = (const HT*)a.minv;
    for (int e = t; e < k * k; e += UT) {
        Gs[(e / k) * KB + e % k] = gram[e];
        Ms[(e / k) * KB + e % k] = minv[e];
    }
    const int64_t g0 = a.row0 + tile * TR + r0;
    const HT* Wt = (const HT*)a.H;
    for (int f = t; f < SR * k; f += UT) Ws[(f / k) * KB + f % k] = Wt[g0 * k + f];
    __syncthreads();
    int64_t w_lo, w_hi, slot_base, slot_mul;
    partial_slots(p, act, w_lo, w_hi, slot_base, slot_mul);
    const HT* part = (const HT*)a.part;
    HT* Ud = (HT*)a.M;
    HT* Go = (HT*)a.Gout;
    HT* Wn = (HT*)a.Hn;
    const HT rho = (HT)a.rho;
    // With k == KB the elements f = t + UT j of a thread share the column
    // c = t % KB: the S.W partials are loaded writer by writer for all of them
    // at once, and the Gram and M^-1 entries of the column are read from LDS
    // once for all rows (rows in 4-wide vectors); every sum keeps the order
    // of the per-element loops below.
    constexpr int NJ = SR * KB / UT;
    typedef HT hvec4 __attribute__((ext_vector_type(4)));
    const bool full_k = k == KB;
    const int cc = t % KB, rb = t / KB;
    HT swv[NJ], wgv[NJ];
    if (full_k) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) swv[j] = wgv[j] = 0;
        for (int64_t w = w_lo; w <= w_hi; ++w) {
            const HT* pw = part + ((slot_mul * w + slot_base) * TR + r0) * (int64_t)k;
#pragma unroll
            for (int j = 0; j < NJ; ++j) swv[j] += pw[t + UT * j];
        }
        for (int b = 0; b < KB; b += 4) {
            const HT g0 = Gs[b * KB + cc], g1 = Gs[(b + 1) * KB + cc], g2 = Gs[(b + 2) * KB + cc],
                     g3 = Gs[(b + 3) * KB + cc];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const hvec4 wv = *(const hvec4*)&Ws[(rb + j * (UT / KB)) * KB + b];
                HT v = wgv[j];
                v += wv[0] * g0;
                v += wv[1] * g1;
                v += wv[2] * g2;
                v += wv[3] * g3;
                wgv[j] = v;
            }
        }
    }
    double tr = 0.0, kkt = 0.0;
    int bad = 0;
    int jj = 0;
    for (int f = t; f < SR * k; f += UT, ++jj) {
        const int r = f / k, c = f - r * k;
        const int64_t prow = tile * TR + r0 + r;
        HT av = 0;
        if (prow < a.rows) {
            const HT w = Ws[r * KB + c];
            const int64_t idx = prow * k + c;
            HT sw = 0;
            if (full_k) {
                sw = swv[jj < NJ ? jj : 0];
            } else {
                for (int64_t wg = w_lo; wg <= w_hi; ++wg)
                    sw += part[((slot_mul * wg + slot_base) * TR + r0 + r) * (int64_t)k + c];
            }
            if (a.fp8) sw = sw / (HT)a.panel_scale[prow / a.panel_rows] + (HT)a.diag[prow] * w;
            HT wg = 0;
            if (full_k) {
                wg = wgv[jj < NJ ? jj : 0];
            } else {
                for (int b = 0; b < k; ++b) wg += Ws[r * KB + b] * Gs[b * KB + c];
            }
            const HT g = (HT)4 * (wg - sw);
            tr += (double)w * (double)sw;
            const HT pg = w > (HT)0 ? g : (g < (HT)0 ? g : (HT)0);
            kkt += (double)pg * (double)pg;
            if (!(g == g) || g - g != (HT)0) ++bad;
            if (Go) Go[idx] = g;
            av = (HT)2 * sw + rho * (w - Ud[idx]);
        }
        As[r * KB + c] = av;
    }
    __syncthreads();
    HT hv[NJ];
    if (full_k) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) hv[j] = 0;
        for (int b = 0; b < KB; b += 4) {
            const HT m0 = Ms[b * KB + cc], m1 = Ms[(b + 1) * KB + cc], m2 = Ms[(b + 2) * KB + cc],
                     m3 = Ms[(b + 3) * KB + cc];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const hvec4 av4 = *(const hvec4*)&As[(rb + j * (UT / KB)) * KB + b];
                HT v = hv[j];
                v += av4[0] * m0;
                v += av4[1] * m1;
                v += av4[2] * m2;
                v += av4[3] * m3;
                hv[j] = v;
            }
        }
    }
    jj = 0;
    for (int f = t; f < SR * k; f += UT, ++jj) {
        const int r = f / k, c = f - r * k;
        const int64_t prow = tile * TR + r0 + r;
        HT wn = 0;
        if (prow < a.rows) {
            const int64_t idx = prow * k + c;
            HT h = 0;
            if (full_k) {
                h = hv[jj < NJ ? jj : 0];
            } else {
                for (int j = 0; j < k; ++j) h += As[r * KB + j] * Ms[j * KB + c];
            }
            const HT u = Ud[idx];
            wn = h + u > (HT)0 ? h + u : (HT)0;
            Ud[idx] = u + h - wn;
            Wn[(g0 + r) * k + c] = wn;
        }
        Wns[r * KB + c] = wn;
    }
    __syncthreads();
    double* tg = a.tile_gram + slice * (int64_t)k * k;
    if (KB >= 32 && k == KB) {
        // entries (ia0 + q, ib), q < NQ, as in the update kernel: the same FP64
        // sums over the slice rows, consecutive ia read as 4-wide vectors
        constexpr int NQ = KB >= 32 ? (KB * KB) / UT : 4;
        static_assert(NQ % 4 == 0, "4-wide Gram reads need NQ % 4 == 0");
        const int ib = t % KB, ia0 = (t / KB) * NQ;
        double sq[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sq[q] = 0.0;
        for (int r = 0; r < SR; ++r) {
            const double hb = (double)Wns[r * KB + ib];
#pragma unroll
            for (int q = 0; q < NQ; q += 4) {
                const hvec4 wv = *(const hvec4*)&Wns[r * KB + ia0 + q];
#pragma unroll
                for (int e = 0; e < 4; ++e) sq[q + e] += (double)wv[e] * hb;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) tg[(ia0 + q) * k + ib] = sq[q];
    } else {
        for (int e = t; e < k * k; e += UT) {
            const int ia = e / k, ib = e - ia * k;
            double s = 0.0;
            for (int r = 0; r < SR; ++r) s += (double)Wns[r * KB + ia] * (double)Wns[r * KB + ib];
            tg[e] = s;
        }
    }
    const double str = block_sum(tr, red);
    const double skk = block_sum(kkt, red);
    const double sbad = block_sum((double)bad, red);
    if (t == 0) {
        a.tile_tr[slice] = str;
        a.tile_kkt[slice] = skk;
        a.tile_bad[slice] = (int32_t)sbad;
    }
}

hipError_t launch_admm(const UpdateArgs& a, const double* gram64, int h_f64, const PlanView& p, hipStream_t stream) {
    if (!p.full || a.k > KMAX || (h_f64 && a.k > 32)) return hipErrorInvalidValue;
    if (h_f64)
        hipLaunchKernelGGL(admm_minv_kernel<double>, dim3(1), dim3(256), 0, stream, gram64, (int)a.k, a.rho,
                           (double*)a.minv);
    else
        hipLaunchKernelGGL(admm_minv_kernel<float>, dim3(1), dim3(256), 0, stream, gram64, (int)a.k, a.rho,
                           (float*)a.minv);
    const int64_t tiles = a.rows_pad / TR;
    dim3 grid(tiles * SUBT), block(UT);
    if (h_f64) {
        if (a.k <= 8) hipLaunchKernelGGL((admm_update_kernel<double, 8>), grid, block, 0, stream, a, p);
        else if (a.k <= 16) hipLaunchKernelGGL((admm_update_kernel<double, 16>), grid, block, 0, stream, a, p);
        else hipLaunchKernelGGL((admm_update_kernel<double, 32>), grid, block, 0, stream, a, p);
    } else {
        if (a.k <= 8) hipLaunchKernelGGL((admm_update_kernel<float, 8>), grid, block, 0, stream, a, p);
        else if (a.k <= 16) hipLaunchKernelGGL((admm_update_kernel<float, 16>), grid, block, 0, stream, a, p);
        else if (a.k <= 32) hipLaunchKernelGGL((admm_update_kernel<float, 32>), grid, block, 0, stream, a, p);
        else hipLaunchKernelGGL((admm_update_kernel<float, 64>), grid, block, 0, stream, a, p);
    }
    return hipGetLastError();
}

// Per-tile FP64 Gram partials of H rows [row0 + tile*TR, +TR) (rows >= row0+rows are zero).
template <typename HT>
__global__ __launch_bounds__(256) void tile_gram_kernel(const HT* __restrict__ H, int64_t row0, int64_t rows,
                                                        int k, double* __restrict__ out) {
    const int64_t slice = blockIdx.x;
    const int t = threadIdx.x;
    double* dst = out + slice * (int64_t)k * k;
    for (int e = t; e < k * k; e += 256) {
        const int ia = e / k, ib = e - ia * k;
        double s = 0.0;
        for (int r = 0; r < SR; ++r) {
            const int64_t prow = slice * SR + r;
            if (prow < rows) s += (double)H[(row0 + prow) * k + ia] * (double)H[(row0 + prow) * k + ib];
        }
        dst[e] = s;
    }
}

hipError_t launch_tile_gram(const void* H, int h_f64, int64_t row0, int64_t rows, int64_t tiles, int64_t k,
                            double* tile_gram, hipStream_t stream) {
    if (h_f64)
        hipLaunchKernelGGL(tile_gram_kernel<double>, dim3(tiles * SUBT), dim3(256), 0, stream, (const double*)H,
                           row0, rows, (int)k, tile_gram);
    else
        hipLaunchKernelGGL(tile_gram_kernel<float>, dim3(tiles * SUBT), dim3(256), 0, stream, (const float*)H,
                           row0, rows, (int)k, tile_gram);
    return hipGetLastError();
}

// FP64 Gram of the rows of [0, n) outside [skip_lo, skip_hi): one work-group per
// entry, fixed order.  (For a row panel: the rows that stay fixed.)
template <typename HT>
__global__ __launch_bounds__(256) void gram_rows_kernel(const HT* __restrict__ H, int64_t n, int64_t skip_lo,
                                                        int64_t skip_hi, int k, double* __restrict__ out) {
    __shared__ double red[8];
    const int e = blockIdx.x;
    const int ia = e / k, ib = e - ia * k;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256)
        if (r < skip_lo || r >= skip_hi) s += (double)H[r * k + ia] * (double)H[r * k + ib];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[e] = s;
}

hipError_t launch_gram_rows(const void* H, int h_f64, int64_t n, int64_t skip_lo, int64_t skip_hi, int64_t k,
                            double* out, hipStream_t stream) {
    if (h_f64)
        hipLaunchKernelGGL(gram_rows_kernel<double>, dim3(k * k), dim3(256), 0, stream, (const double*)H, n, skip_lo,
                           skip_hi, (int)k, out);
    else
        hipLaunchKernelGGL(gram_rows_kernel<float>, dim3(k * k), dim3(256), 0, stream, (const float*)H, n, skip_lo,
                           skip_hi, (int)k, out);
    return hipGetLastError();
}

template <typename HT>
__global__ __launch_bounds__(256) void finalize_kernel(int64_t tiles, int k, const double* __restrict__ tile_gram,
                                                       const double* __restrict__ tile_tr,
                                                       const double* __restrict__ tile_kkt,
                                                       const int32_t* __restrict__ tile_bad,
                                                       const double* __restrict__ gram_fixed,
                                                       const double* __restrict__ gram_cur,
                                                       double* __restrict__ gram_next, HT* __restrict__ gram_eff,
                                                       double* __restrict__ stats) {
    __shared__ double red[8];
    const int kk = k * k;
    const int ngram = (kk + 3) / 4;          // one wave per Gram entry
    const int t = threadIdx.x;
    if ((int)blockIdx.x < ngram) {
        const int e = blockIdx.x * 4 + (t >> 6);
        const int lane = t & 63;
        if (e >= kk) return;
        // lane l sums tiles l, l+64, ...; then a fixed-order butterfly
        double s = 0.0;
        for (int64_t i = lane; i < tiles; i += 64) s += tile_gram[i * kk + e];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) {
            if (gram_fixed) s += gram_fixed[e];
            gram_next[e] = s;
            gram_eff[e] = (HT)s;
            gram_eff[kk + e] = (HT)s;
            gram_eff[2 * kk + e] = (HT)s;
        }
        return;
    }
    double tr = 0.0, kkt = 0.0, bad = 0.0, gn = 0.0;
    for (int64_t i = t; i < tiles; i += 256) {
        tr += tile_tr[i];
        kkt += tile_kkt[i];
        bad += (double)tile_bad[i];
    }
    if (gram_cur)
        for (int e = t; e < kk; e += 256) gn += gram_cur[e] * gram_cur[e];
    tr = block_sum(tr, red);
    kkt = block_sum(kkt, red);
    bad = block_sum(bad, red);
    gn = block_sum(gn, red);
    if (t == 0) {
        stats[0] = tr;
        stats[1] = kkt;
        stats[2] = bad;
        stats[3] = gn;
    }
}

hipError_t launch_finalize(int64_t tiles, int64_t k, const double* tile_gram, const double* tile_tr,
                           const double* tile_kkt, const int32_t* tile_bad, const double* gram_fixed,
                           const double* gram_cur64, double* gram_next64, void* gram_eff, int h_f64,
                           double* stats, hipStream_t stream) {
    const int ngram = (int)((k * k + 3) / 4);
    dim3 grid(ngram + 1), block(256);
    if (h_f64)
        hipLaunchKernelGGL(finalize_kernel<double>, grid, block, 0, stream, tiles, (int)k, tile_gram, tile_tr,
                           tile_kkt, tile_bad, gram_fixed, gram_cur64, gram_next64, (double*)gram_eff, stats);
    else
        hipLaunchKernelGGL(finalize_kernel<float>, grid, block, 0, stream, tiles, (int)k, tile_gram, tile_tr,
                           tile_kkt, tile_bad, gram_fixed, gram_cur64, gram_next64, (float*)gram_eff, stats);
    return hipGetLastError();
}

// Block step: Gram_J, Gram_I and their sum from the slice partials of H_t.
template <typename HT>
__global__ __launch_bounds__(256) void gram_select_kernel(int k, const double* __restrict__ tile_gram,
                                                          const int32_t* __restrict__ tI,
                                                          const int32_t* __restrict__ tJ,
                                                          const int32_t* __restrict__ counts,
                                                          HT* __restrict__ out) {
    const int kk = k * k;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kk) return;
    double gi = 0.0, gj = 0.0;
    for (int i = 0; i < counts[0]; ++i)
        for (int sub = 0; sub < SUBT; ++sub) gi += tile_gram[((int64_t)tI[i] * SUBT + sub) * kk + e];
    for (int i = 0; i < counts[1]; ++i)
        for (int sub = 0; sub < SUBT; ++sub) gj += tile_gram[((int64_t)tJ[i] * SUBT + sub) * kk + e];
    out[e] = (HT)gj;
    out[kk + e] = (HT)gi;
    out[2 * kk + e] = (HT)(gi + gj);
}

hipError_t launch_gram_select(int64_t k, const double* tile_gram, const int32_t* tiles_I, const int32_t* tiles_J,
                              const int32_t* counts, void* gram_eff, int h_f64, hipStream_t stream) {
    dim3 grid((k * k + 255) / 256), block(256);
    if (h_f64)
        hipLaunchKernelGGL(gram_select_kernel<double>, grid, block, 0, stream, (int)k, tile_gram, tiles_I, tiles_J,
                           counts, (double*)gram_eff);
    else
        hipLaunchKernelGGL(gram_select_kernel<float>, grid, block, 0, stream, (int)k, tile_gram, tiles_I, tiles_J,
                           counts, (float*)gram_eff);
    return hipGetLastError();
}

// H0_ij = u_ij * scale, u_ij the 24-bit uniform of counter i*k + j.
__global__ void init_h_kernel(float* __restrict__ H, int64_t count, uint64_t seed, float scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        H[i] = (float)uniform24(seed, (uint64_t)i) * scale;
}

hipError_t launch_init_H(float* H, int64_t n, int64_t k, uint64_t seed, float scale, hipStream_t stream) {
    const int64_t count = n * k;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(init_h_kernel, dim3(blocks), dim3(256), 0, stream, H, count, seed, scale);
    return hipGetLastError();
}

// Zero fill of `bytes` bytes at any alignment: 16-byte vector stores over the
// aligned middle, single bytes for the unaligned ends.  Used instead of a
// memset node so that work a caller records into a HIP graph replays the
// clear as a kernel.
__global__ void zero_kernel(unsigned char* __restrict__ p, int64_t bytes) {
    const int64_t mis = (int64_t)((16 - ((uintptr_t)p & 15)) & 15);
    const int64_t head = mis < bytes ? mis : bytes;
    const int64_t nvec = (bytes - head) / 16;
    const int64_t tail0 = head + nvec * 16;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    u32x4* v = (u32x4*)(p + head);
    for (int64_t i = i0; i < nvec; i += stride) v[i] = u32x4{0u, 0u, 0u, 0u};
    if (i0 < head) p[i0] = 0;
    if (i0 < bytes - tail0) p[tail0 + i0] = 0;
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    if (!p) return hipErrorInvalidValue;
    int64_t blocks = (bytes / 16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, stream, (unsigned char*)p, bytes);
    return hipGetLastError();
}

template <typename A, typename B>
__global__ void copy_kernel(const A* __restrict__ s, B* __restrict__ d, int64_t m) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (B)s[i];
}

hipError_t launch_copy_h(const void* src, int src_f64, void* dst, int dst_f64, int64_t count, hipStream_t stream) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return hipSuccess;
    if (src_f64 && dst_f64)
        hipLaunchKernelGGL((copy_kernel<double, double>), dim3(blocks), dim3(256), 0, stream, (const double*)src, (double*)dst, count);
    else if (src_f64)
        hipLaunchKernelGGL((copy_kernel<double, float>), dim3(blocks), dim3(256), 0, stream, (const double*)src, (float*)dst, count);
    else if (dst_f64)
        hipLaunchKernelGGL((copy_kernel<float, double>), dim3(blocks), dim3(256), 0, stream, (const float*)src, (double*)dst, count);
    else
        hipLaunchKernelGGL((copy_kernel<float, float>), dim3(blocks), dim3(256), 0, stream, (const float*)src, (float*)dst, count);
    return hipGetLastError();
}

// Theta0 = softplus^-1(max(H0, 1e-12)); H0 <- softplus(Theta0).
template <typename HT>
__global__ void softplus_init_kernel(HT* __restrict__ H, HT* __restrict__ Th, int64_t m) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        double h = (double)H[i];
        h = h > 1e-12 ? h : 1e-12;
        const double th = h > 20.0 ? h + log(-expm1(-h)) : log(expm1(h));
        Th[i] = (HT)th;
        H[i] = softplus_f((HT)th);
    }
}

hipError_t launch_softplus_init(void* H, void* Theta, int h_f64, int64_t count, hipStream_t stream) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return hipSuccess;
    if (h_f64)
        hipLaunchKernelGGL(softplus_init_kernel<double>, dim3(blocks), dim3(256), 0, stream, (double*)H, (double*)Theta, count);
    else
        hipLaunchKernelGGL(softplus_init_kernel<float>, dim3(blocks), dim3(256), 0, stream, (float*)H, (float*)Theta, count);
    return hipGetLastError();
}

// FP64 sum of m values (single work-group, fixed order).
template <typename T>
__global__ __launch_bounds__(1024) void sum_kernel(const T* __restrict__ x, int64_t m, double* out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 1024) s += (double)x[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int i = 0; i < 16; ++i) r += red[i];
        *out = r;
    }
}

hipError_t launch_sum(const void* x, int x_f64, int64_t m, double* out, hipStream_t stream) {
    if (x_f64) hipLaunchKernelGGL(sum_kernel<double>, dim3(1), dim3(1024), 0, stream, (const double*)x, m, out);
    else hipLaunchKernelGGL(sum_kernel<float>, dim3(1), dim3(1024), 0, stream, (const float*)x, m, out);
    return hipGetLastError();
}

// Piecewise reset: G_i <- max(c g_i^2, c median(g^2)).
template <typename HT>
__global__ void piecewise_kernel(HT* __restrict__ G, const HT* __restrict__ g, int64_t m, double c,
                                 const double* __restrict__ med) {
    const HT floor_v = (HT)(c * (double)med[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const HT v = (HT)c * g[i] * g[i];
        G[i] = v > floor_v ? v : floor_v;
    }
}

// Objective pass (FP64 H, FP64 S.H partials of a full plan): per tile
// tr partial sum_r h_r . (S H)_r and the FP64 Gram of the tile's H rows.
__global__ __launch_bounds__(256) void objective_tiles_kernel(UpdateArgs a, PlanView p) {
    __shared__ double red[8];
    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int k = (int)a.k;
    const int64_t g0 = a.row0 + tile * TR;
    const double* H = (const double*)a.H;
    const double* part = (const double*)a.part;
    const int64_t U = (int64_t)p.n_tiles * p.n_chunks;
    const int64_t Pe = U < p.P ? U : p.P;
    const int64_t w_lo = wg_owner(tile * p.n_chunks, U, Pe);
    const int64_t w_hi = wg_owner((tile + 1) * p.n_chunks - 1, U, Pe);
    double tr = 0.0;
    for (int f = t; f < TR * k; f += 256) {
        const int r = f / k, c = f - r * k;
        const int64_t prow = tile * TR + r;
        if (prow >= a.rows) continue;
        double sh = 0.0;
        for (int64_t w = w_lo; w <= w_hi; ++w) sh += part[((w + tile) * TR + r) * (int64_t)k + c];
        const double h = H[(g0 + r) * k + c];
        if (a.fp8) sh = sh / (double)a.panel_scale[prow / a.panel_rows] + (double)a.diag[prow] * h;
        tr += h * sh;
    }
    double* tg = a.tile_gram + tile * (int64_t)k * k;
    for (int e = t; e < k * k; e += 256) {
        const int ia = e / k, ib = e - ia * k;
        double s = 0.0;
        for (int r = 0; r < TR; ++r)
            if (tile * TR + r < a.rows) s += H[(g0 + r) * k + ia] * H[(g0 + r) * k + ib];
        tg[e] = s;
    }
    const double str = block_sum(tr, red);
    if (t == 0) {
        a.tile_tr[tile] = str;
        a.tile_kkt[tile] = 0.0;
        a.tile_bad[tile] = 0;
    }
}

hipError_t launch_objective_tiles(const UpdateArgs& a, const PlanView& p, hipStream_t stream) {
    hipLaunchKernelGGL(objective_tiles_kernel, dim3(a.rows_pad / TR), dim3(256), 0, stream, a, p);
    return hipGetLastError();
}

hipError_t launch_piecewise_apply(void* G, const void* g, int h_f64, int64_t m, double c, const double* med,
                                  hipStream_t stream) {
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (h_f64)
        hipLaunchKernelGGL(piecewise_kernel<double>, dim3(blocks), dim3(256), 0, stream, (double*)G, (const double*)g, m, c, med);
    else
        hipLaunchKernelGGL(piecewise_kernel<float>, dim3(blocks), dim3(256), 0, stream, (float*)G, (const float*)g, m, c, med);
    return hipGetLastError();
}

}  // namespace symnmf
