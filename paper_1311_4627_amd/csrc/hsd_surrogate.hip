// Learned surrogate of the emissivity solve: an MLP 33 -> 256 -> 256 -> 256 -> L
// (GELU after the hidden layers) mapping the field's energy in 32 wavelength
// bands and the grain radius to log10(j_lambda / A), A the absorbed power.  It
// is trained here on spectra of the plain solve, on the GPU (BF16 matrix-core
// products with FP32 accumulation, FP32 master weights, Adam), and evaluated
// with its energy balance checked per pair.  The paper's introduction names
// precomputed emissivity tables as the cheap alternative to the full solve;
// this is a learned table of that kind with the plain solve as its fallback.
//
// Layouts.  Parameters are one FP32 vector, layer by layer: W_l row-major
// [out][in], then b_l.  Raw inputs X are [n][33]: log10 of the band energies
// int u dlambda (trapezoid over grid nodes floor(b (L-1) / 32) ..
// floor((b+1) (L-1) / 32)), then log10 of the radius in cm.  Raw targets Y are
// [n][L]: log10(max(j, 1e-6 max j) / A) (the floor keeps wavelengths that carry
// no power from dominating the fit).  Inputs are z-scored per column; targets
// have their column means removed and are divided by one pooled standard
// deviation, so the loss weighs an error in dex the same at every wavelength.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "hsd_internal.h"

namespace hsd {
namespace {

constexpr int kBands = 32;
constexpr int kLossBlocks = 1024;   // blocks of the loss reduction (one FP64 partial each)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16, round to nearest even (the hardware conversion).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned short to_bf16(float f) {
    return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}
// two values, lo in the low half
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }

// erfc from the Chebyshev-fitted form of Numerical Recipes (Press et al.,
// "erfcc"): erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + |x|/2), P of degree 9,
// fractional error below 1.2e-7 for x >= 0; erfc(-x) = 2 - erfc(x).  Branch
// free: one reciprocal, one exp and ten FMAs.
__device__ __forceinline__ float erfc_fast(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, ax, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    const float r = t * __expf(fmaf(-ax, ax, p));
    return x >= 0.f ? r : 2.0f - r;
}
__device__ __forceinline__ float phi_cdf(float z) { return 0.5f * erfc_fast(-z * 0.70710678118654752f); }

// GELU of the inference kernels, x Phi(x) with Phi from the erf approximation
// of Abramowitz & Stegun, formula 7.1.26: with s = |x| / sqrt(2) and
// t = 1 / (1 + p s), 1 - erf(s) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-s^2),
// |error| <= 1.5e-7 in erf, so <= 7.5e-8 in Phi.  The inference kernels store
// activations as BF16 (relative spacing 2^-8), far coarser than that; this
// form takes 15 instructions where erfc_fast's takes 23.
__device__ __forceinline__ float gelu_infer(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, ax, 1.0f));
    // half the polynomial: q = (1 - erf(s)) / 2 = Phi(-|x|)
    float p = 0.5f * 1.061405429f;
    p = fmaf(p, t, 0.5f * -1.453152027f);
    p = fmaf(p, t, 0.5f * 1.421413741f);
    p = fmaf(p, t, 0.5f * -0.284496736f);
    p = fmaf(p, t, 0.5f * 0.254829592f);
    const float q = p * t * __builtin_amdgcn_exp2f((x * x) * -0.72134752044448170f);   // e^(-x^2/2)
    return x * (x >= 0.f ? 1.0f - q : q);
}
__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z); }
__device__ __forceinline__ float gelu_grad(float z) {
    return phi_cdf(z) + z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---- per-cell band energies --------------------------------------------------
// One 64-lane wave per cell; lane b < 32 integrates band b in FP64.
__global__ void __launch_bounds__(256) k_bands(const double* u, const double* lam, int n_cells, int L,
                                               float* bands) {
    const int lane = threadIdx.x & 63;
    const int cell = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (cell >= n_cells || lane >= kBands) return;
    const int e0 = (lane * (L - 1)) / kBands, e1 = ((lane + 1) * (L - 1)) / kBands;
    const double* uc = u + static_cast<size_t>(cell) * L;
    double s = 0.0;
    for (int j = e0; j < e1; ++j) s += 0.5 * (uc[j] + uc[j + 1]) * (lam[j + 1] - lam[j]);
    bands[static_cast<size_t>(cell) * kBands + lane] = static_cast<float>(log10(fmax(s, 1e-300)));
}

// Absorption weights of the selected grains, transposed: wcT[j][s] =
// c C_abs,s(lambda_j) w_j with w_j the trapezoid weight of node j, so the
// absorbed power of a pair is A = sum_j u_j wcT[j][s].
__global__ void __launch_bounds__(256) k_wc(const double* const* cabs, const double* lam, int n_sel, int L,
                                            double* wcT) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_sel * L) return;
    const int j = i / n_sel, s = i - j * n_sel;
    const double lo = j > 0 ? lam[j - 1] : lam[0];
    const double hi = j + 1 < L ? lam[j + 1] : lam[L - 1];
    wcT[i] = kLight * cabs[s][j] * 0.5 * (hi - lo);
}

// Pair rows R = cell * n_sel + s (s indexes the selected grains) in
// [row0, row0 + n_rows), written at R - row0: the absorbed power A (FP64), and
// the inputs either raw (X, 33 floats) or normalised as the first layer reads
// them (xb, 96 BF16: hi terms of the 33 inputs, their lo terms, zeros).
// A[cell][s] = sum_j u[cell][j] wcT[j][s] is a small FP64 matrix product: a
// block takes S selected grains (64, or 32 or 16 for smaller selections) and
// 512 / S cells, and stages 64-wavelength slices of both operands in LDS;
// each thread sums two cells of one grain in wavelength order (the same order
// for every S).
struct PairArgs {
    const double* u;
    const float* bands;        // [n_cells][32]
    const double* wcT;         // [L][n_sel]
    const float* loga;         // [n_sel] log10 radius (cm)
    long long row0, n_rows;
    long long cell0, n_cells;  // cells touched by the rows
    int n_sel, L;
    float* X;                  // [n_rows][33] or null
    double* A;                 // [n_rows] or null
    unsigned short* xb;        // [n_rows][96] or null
    const float* xm; const float* xs;   // input statistics (xb)
};

constexpr int kPairLam = 64;

template <int kPairSlots>
__global__ void __launch_bounds__(256) k_pairs(PairArgs a) {
    constexpr int kPairCells = 512 / kPairSlots;     // two per thread
    __shared__ double us[kPairCells][kPairLam];
    __shared__ double ws[kPairLam][kPairSlots];
    const int tid = threadIdx.x;
    const int sl = tid % kPairSlots, cg = tid / kPairSlots;
    const long long c0 = a.cell0 + static_cast<long long>(blockIdx.x) * kPairCells;
    const int s0 = blockIdx.y * kPairSlots;
    const int ns = min(kPairSlots, a.n_sel - s0);
    const int nc = static_cast<int>(min(static_cast<long long>(kPairCells), a.cell0 + a.n_cells - c0));
    if (a.A) {
        double p0 = 0.0, p1 = 0.0;
        for (int j0 = 0; j0 < a.L; j0 += kPairLam) {
            const int nl = min(kPairLam, a.L - j0);
            for (int e = tid; e < kPairCells * kPairLam; e += 256) {
                const int cc = e / kPairLam, l = e % kPairLam;
                us[cc][l] = cc < nc && l < nl ? a.u[(c0 + cc) * a.L + j0 + l] : 0.0;
            }
            for (int e = tid; e < kPairLam * kPairSlots; e += 256) {
                const int l = e / kPairSlots, ss = e % kPairSlots;
                ws[l][ss] = l < nl && ss < ns ? a.wcT[static_cast<long long>(j0 + l) * a.n_sel + s0 + ss] : 0.0;
            }
            __syncthreads();
            for (int l = 0; l < nl; ++l) {
                const double w = ws[l][sl];
                p0 = fma(us[2 * cg][l], w, p0);
                p1 = fma(us[2 * cg + 1][l], w, p1);
            }
            __syncthreads();
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cc = 2 * cg + h;
            const long long rr = (c0 + cc) * a.n_sel + s0 + sl - a.row0;
            if (cc < nc && sl < ns && rr >= 0 && rr < a.n_rows) a.A[rr] = h ? p1 : p0;
        }
    }
    // inputs: staged once in LDS (raw, and normalised as hi and lo terms), so
    // that the write loops below issue stores only (a load between stores
    // would wait for all of them: the memory counter is in order)
    __shared__ float braw[kPairCells][kBands], araw[kPairSlots];
    __shared__ unsigned short bnorm[kPairCells][2][kBands], anorm[kPairSlots][2];
    {
        for (int e = tid; e < kPairCells * kBands; e += 256) {
            const int cc = e / kBands, k = e % kBands;
            if (cc < nc) {
                const float v = a.bands[(c0 + cc) * kBands + k];
                braw[cc][k] = v;
                if (a.xb) {
                    const float x = (v - a.xm[k]) / a.xs[k];
                    const unsigned short hi = to_bf16(x);
                    bnorm[cc][0][k] = hi;
                    bnorm[cc][1][k] = to_bf16(x - from_bf16(hi));
                }
            }
        }
        if (tid < ns) {
            const float v = a.loga[s0 + tid];
            araw[tid] = v;
            if (a.xb) {
                const float x = (v - a.xm[kBands]) / a.xs[kBands];
                const unsigned short hi = to_bf16(x);
                anorm[tid][0] = hi;
                anorm[tid][1] = to_bf16(x - from_bf16(hi));
            }
        }
    }
    __syncthreads();
    // the rows of one cell and this slot group are contiguous
    for (int cc = 0; cc < nc; ++cc) {
        const long long rbase = (c0 + cc) * a.n_sel + s0 - a.row0;
        if (a.X) {
            for (int e = tid; e < ns * 33; e += 256) {
                const int ss = e / 33, k = e % 33;
                const long long rr = rbase + ss;
                if (rr >= 0 && rr < a.n_rows) a.X[rr * 33 + k] = k < kBands ? braw[cc][k] : araw[ss];
            }
        }
        if (a.xb) {
            // row layout: hi of the 33 inputs, lo of the 33 inputs, 30 zeros;
            // two columns per 32-bit store
            for (int e = tid; e < ns * 48; e += 256) {
                const int ss = e / 48, k2 = 2 * (e % 48);
                const long long rr = rbase + ss;
                if (rr < 0 || rr >= a.n_rows) continue;
                unsigned v = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int col = k2 + h;
                    unsigned b = 0;
                    if (col < 66) {
                        const int term = col < 33 ? 0 : 1, k = col - 33 * term;
                        b = k < kBands ? bnorm[cc][term][k] : anorm[ss][term];
                    }
                    v |= b << (16 * h);
                }
                reinterpret_cast<unsigned*>(a.xb + rr * 96)[k2 / 2] = v;
            }
        }
    }
}

// Raw targets from spectra, one wave per row: Y[r][k] = log10(max(j, 1e-6
// max j) / A) for the L wavelengths, Y[r][L] = log10(4 pi int j dlambda / A)
// (trapezoid, FP64 sums).
__global__ void __launch_bounds__(256) k_targets(const float* j, const double* A, const double* lam, long long n,
                                                 int L, float* Y) {
    const int lane = threadIdx.x & 63;
    const long long r = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const float* jr = j + r * L;
    float mx = 0.f;
    double em = 0.0;
    for (int k = lane; k < L; k += 64) {
        mx = fmaxf(mx, jr[k]);
        if (k + 1 < L) em += 0.5 * (lam[k + 1] - lam[k]) * (static_cast<double>(jr[k]) + jr[k + 1]);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, m, 64));
        em += __shfl_xor(em, m, 64);
    }
    const double fl = 1e-6 * static_cast<double>(mx);
    const double a = A[r];
    float* yr = Y + r * (L + 1);
    for (int k = lane; k < L; k += 64) yr[k] = static_cast<float>(log10(fmax(static_cast<double>(jr[k]), fl) / a));
    if (lane == 0) yr[L] = static_cast<float>(log10(4.0 * kPi * em / a));
}

// Column sums and sums of squares in FP64, first stage: one thread per
// column and block of rows, each block's partial written to its own slot
// (part[block][2 w]: sums, then squares); k_colstats_sum adds the blocks in
// order, so the statistics do not depend on scheduling.
__global__ void __launch_bounds__(256) k_colstats(const float* Xm, long long n, int w, long long rows_per_block,
                                                  double* part) {
    const int col = blockIdx.y * 256 + threadIdx.x;
    if (col >= w) return;
    const long long r0 = static_cast<long long>(blockIdx.x) * rows_per_block;
    const long long r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
    double s = 0.0, q = 0.0;
    for (long long r = r0; r < r1; ++r) {
        const double v = Xm[r * w + col];
        s += v;
        q += v * v;
    }
    double* p = part + static_cast<long long>(blockIdx.x) * 2 * w;
    p[col] = s;
    p[w + col] = q;
}

// Second stage: out[c] = sum over blocks b = 0, 1, ... of part[b][c], c < 2 w.
__global__ void __launch_bounds__(256) k_colstats_sum(const double* part, int n_blocks, int w2, double* out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= w2) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += part[static_cast<long long>(b) * w2 + c];
    out[c] = s;
}

// Gather a minibatch and z-score it: rows idx[b] of X (33 wide) and Y (L wide).
__global__ void __launch_bounds__(256) k_gather(const float* X, const float* Y, const long long* idx, int B, int L,
                                                const float* xm, const float* xs, const float* ym, const float* ys,
                                                float* Xb, float* Yb) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const long long r = idx[b];
    for (int k = threadIdx.x; k < 33; k += blockDim.x) Xb[b * 33 + k] = (X[r * 33 + k] - xm[k]) / xs[k];
    if (Y)
        for (int k = threadIdx.x; k < L; k += blockDim.x)
            Yb[static_cast<long long>(b) * L + k] = (Y[r * L + k] - ym[k]) / ys[k];
}

// Band-weighted loss: per-element weights of each minibatch row from its raw
// targets y_k = log10(j_k / A).  The accuracy that matters is that of the
// spectrum integrated over the 32 bands (band b: grid nodes e_b .. e_(b+1),
// trapezoid rule) that hold at least 1e-3 of the row's emitted power; an
// error d_k in log10 j_k moves band b by ln 10 sum_k d_k j_k q_kb / J_b, so
// the loss weights element k by rho_k = sum over such bands b of
// j_k q_kb / J_b / n_bands (q_kb: node k's trapezoid weight inside band b;
// sum_k rho_k = 1):  W_k = (1 - bw) + bw L rho_k, and 1 for the ratio output.
// One block per row; the band sums run in a fixed order.
__global__ void __launch_bounds__(256) k_loss_weights(const float* Y, const long long* idx, int L, int n_out,
                                                      const float* wl, const float* wr, const int* segband,
                                                      const int* bedge, float bw, float* W) {
    __shared__ float f[kMaxLambda];
    __shared__ float seg[kMaxLambda];
    __shared__ double J[kBands];
    __shared__ float red[4];
    __shared__ float inv_n;
    const int b = blockIdx.x;
    const float* y = Y + idx[b] * n_out;
    float mx = -INFINITY;
    for (int k = threadIdx.x; k < L; k += 256) mx = fmaxf(mx, y[k]);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    for (int k = threadIdx.x; k < L; k += 256) f[k] = exp2f((y[k] - mx) * 3.32192809488736234787f);
    __syncthreads();
    for (int k = threadIdx.x; k + 1 < L; k += 256) seg[k] = wr[k] * f[k] + wl[k + 1] * f[k + 1];
    __syncthreads();
    if (threadIdx.x < kBands) {
        double t = 0.0;
        for (int k = bedge[threadIdx.x]; k < bedge[threadIdx.x + 1]; ++k) t += seg[k];
        J[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int q = 0; q < kBands; ++q) tot += J[q];
        int nc = 0;
        for (int q = 0; q < kBands; ++q) {
            const bool on = J[q] >= 1e-3 * tot && J[q] > 0.0;
            nc += on ? 1 : 0;
            if (!on) J[q] = 0.0;          // 0 marks a band outside the metric
        }
        inv_n = nc > 0 ? 1.f / static_cast<float>(nc) : 0.f;
    }
    __syncthreads();
    float* w = W + static_cast<long long>(b) * n_out;
    for (int k = threadIdx.x; k < n_out; k += 256) {
        float wk = 1.f;
        if (k < L) {
            double rho = 0.0;
            if (k + 1 < L && J[segband[k]] > 0.0) rho += wr[k] * f[k] / J[segband[k]];
            if (k > 0 && J[segband[k - 1]] > 0.0) rho += wl[k] * f[k] / J[segband[k - 1]];
            wk = (1.f - bw) + bw * static_cast<float>(L) * static_cast<float>(rho) * inv_n;
        }
        w[k] = wk;
    }
}

// Minibatch indices from a counter-based generator (SplitMix64 of seed and
// position; uniform enough for sampling with replacement).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// The step comes from `ctr` (device memory) when given: a training step
// replayed from a graph reads its counter there.
__global__ void k_batch_idx(unsigned long long seed, long long step, const long long* ctr, int B, long long n,
                            long long* idx) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (ctr) step = *ctr;
    const unsigned long long h = splitmix64(seed ^ splitmix64(static_cast<unsigned long long>(step) * B + b));
    idx[b] = static_cast<long long>(h % static_cast<unsigned long long>(n));
}

// Loss and its gradient with respect to the network output:
// L = mean W (yhat - y)^2 (W = 1 without band weighting),
// dL/dyhat = 2 W (yhat - y) / (B L).  A fixed grid walks
// the elements; each block writes its FP64 partial sum of squares to its own
// slot, and k_loss_sum adds the slots in order.
__global__ void __launch_bounds__(256) k_loss(const float* yhat, const float* y, const float* wt, long long n,
                                              float scale, float* dy, double* part) {
    __shared__ double red[4];
    double l = 0.0;
    for (long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * 256) {
        const float r = yhat[i] - y[i];
        const float wr = wt ? wt[i] * r : r;
        dy[i] = scale * wr;
        l += static_cast<double>(wr) * r;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) l += __shfl_xor(l, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_loss_sum(const double* part, int n, double* loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += part[b];
    *loss = s;
}

// Bias gradient, first stage: column sums of dZ [B][N] over chunks of 32
// rows (blockIdx.y), written per chunk; k_split_sum adds the chunks in order.
__global__ void __launch_bounds__(256) k_colsum(const float* dz, int B, int N, float* part) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const int b0 = blockIdx.y * 32, b1 = min(B, b0 + 32);
    float s = 0.f;
    for (int b = b0; b < b1; ++b) s += dz[static_cast<long long>(b) * N + j];
    part[static_cast<long long>(blockIdx.y) * N + j] = s;
}

// Adam (Kingma & Ba) with bias correction folded into the step size.
// One Adam step; we (if given) follows the iterates as a moving average,
// we = ed we + (1 - ed) w.
// With `sched`, the step sizes of step *ctr come from sched[*ctr - t0]
// (computed on the host, as for the by-value form).
__global__ void __launch_bounds__(256) k_adam(float* w, const float* g, float* m, float* v, long long n, float lr_t,
                                              float b1, float b2, float eps_t, float* we, float ed,
                                              const float2* sched, const long long* ctr, long long t0) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    if (sched) {
        const float2 p = sched[*ctr - t0];
        lr_t = p.x;
        eps_t = p.y;
    }
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr_t * mi / (sqrtf(vi) + eps_t);
    w[i] = wi;
    if (we) we[i] = fmaf(ed, we[i] - wi, wi);
}

// End of a graph-replayed training step: the minibatch loss into the trace
// (if any), then the step counter advances.
__global__ void k_step_end(long long* ctr, long long t0, const double* loss, double* trace) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const long long t = *ctr;
    if (trace) trace[t - t0] = *loss;
    *ctr = t + 1;
}

// ---- BF16 matrix-core GEMM ----------------------------------------------------------
// C[i][j] = epilogue(sum_k A[i][k] B[k][j]) with arbitrary strides: A[i][k] at
// A[i*sai + k*sak], B[k][j] at B[k*sbk + j*sbj].  Operands are FP32 in memory
// and rounded to BF16 as they are staged in LDS; the v_mfma_f32_16x16x16_bf16
// products accumulate in FP32.  Operand layout of that instruction: lane l
// supplies A[l % 16][4 (l / 16) + 0..3] and B[4 (l / 16) + 0..3][l % 16];
// accumulator register i of lane l is D[4 (l / 16) + i][l % 16].  One
// 256-thread block computes a 64 x 64 tile, each wave a 32 x 32 quarter.
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

struct GemmArgs {
    const float* A; long long sai, sak;
    const float* B; long long sbk, sbj;
    float* C; long long ldc;           // EPI_BIAS_GELU: pre-activations (may be null)
    float* C2; long long ldc2;         // EPI_BIAS_GELU: activations
    const float* bias;                 // [N]
    const float* aux; long long ldaux; // EPI_GELU_BWD: pre-activations
    int M, N, K;
    int kchunk;                        // split K: block z sums k in [z kchunk, (z+1) kchunk) (EPI_STORE only)
    long long split_stride;            //   and writes its partial at C + z split_stride
    int asplit;                        // A as two BF16 terms: k in [K, 2K) stages A[i][k-K] - bf16(A[i][k-K])
                                       //   against B[k-K][j] (not with split K)
};

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    constexpr int BM = 64, BN = 64, BK = 32, LK = BK + 8;
    __shared__ __align__(16) unsigned short As[BM][LK];
    __shared__ __align__(16) unsigned short Bs[BN][LK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long m0 = static_cast<long long>(blockIdx.y) * BM;
    const int n0 = blockIdx.x * BN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool a_kfast = g.sak == 1;
    const bool b_kfast = g.sbk == 1;
    const int Kr = g.K;
    int kbeg = 0, kend = g.asplit ? 2 * Kr : Kr;
    float* Cz = g.C;
    if constexpr (EPI == EPI_STORE) {
        if (g.kchunk > 0) {
            kbeg = blockIdx.z * g.kchunk;
            kend = min(g.K, kbeg + g.kchunk);
            Cz = g.C + blockIdx.z * g.split_stride;
        }
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int e = 0; e < (BM * BK) / 256; ++e) {
            const int idx = tid + 256 * e;
            const int i = a_kfast ? idx / BK : idx % BM;
            const int k = a_kfast ? idx % BK : idx / BM;
            const long long gi = m0 + i;
            const int gk = k0 + k;
            float v = 0.f;
            if (gi < g.M && gk < kend) {
                const bool lo = gk >= Kr;
                v = g.A[gi * g.sai + (lo ? gk - Kr : gk) * g.sak];
                if (lo) v -= from_bf16(to_bf16(v));
            }
            As[i][k] = to_bf16(v);
        }
#pragma unroll
        for (int e = 0; e < (BN * BK) / 256; ++e) {
            const int idx = tid + 256 * e;
            const int j = b_kfast ? idx / BK : idx % BN;
            const int k = b_kfast ? idx % BK : idx / BN;
            const int gj = n0 + j, gk = k0 + k;
            float v = 0.f;
            if (gj < g.N && gk < kend) {
                const int kr = gk >= Kr ? gk - Kr : gk;
                v = g.B[static_cast<long long>(kr) * g.sbk + static_cast<long long>(gj) * g.sbj];
            }
            Bs[j][k] = to_bf16(v);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x4 af[2], bf[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                af[t] = *reinterpret_cast<const bf16x4*>(&As[wm + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
                bf[t] = *reinterpret_cast<const bf16x4*>(&Bs[wn + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long i = m0 + wm + a * 16 + 4 * (lane >> 4) + r;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int j = n0 + wn + b * 16 + (lane & 15);
                if (i >= g.M || j >= g.N) continue;
                const float v = acc[a][b][r];
                if constexpr (EPI == EPI_STORE) {
                    Cz[i * g.ldc + j] = v;
                } else if constexpr (EPI == EPI_BIAS) {
                    g.C[i * g.ldc + j] = v + g.bias[j];
                } else if constexpr (EPI == EPI_BIAS_GELU) {
                    const float z = v + g.bias[j];
                    if (g.C) g.C[i * g.ldc + j] = z;
                    g.C2[i * g.ldc2 + j] = gelu(z);
                } else {
                    g.C[i * g.ldc + j] = v * gelu_grad(g.aux[i * g.ldaux + j]);
                }
            }
        }
    }
}

template <int EPI>
hipError_t gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const dim3 grid((g.N + 63) / 64, static_cast<unsigned>((g.M + 63) / 64));
    hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// Sum of the split-K partials: out[e] = sum_z part[z * stride + e], z in order.
__global__ void __launch_bounds__(256) k_split_sum(const float* part, int nz, long long stride, long long n,
                                                   float* out) {
    const long long e = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= n) return;
    float acc = 0.f;
    for (int z = 0; z < nz; ++z) acc += part[z * stride + e];
    out[e] = acc;
}

// C[M][N] = A . B with K split over `nz` blocks along z into a workspace of
// nz * M * N floats, then summed in a fixed order (deterministic).
hipError_t gemm_splitk(GemmArgs g, int nz, float* work, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    float* out = g.C;
    const long long mn = static_cast<long long>(g.M) * g.N;
    g.kchunk = ((g.K + nz - 1) / nz + 31) / 32 * 32;
    nz = (g.K + g.kchunk - 1) / g.kchunk;
    g.C = work;
    g.ldc = g.N;
    g.split_stride = mn;
    const dim3 grid((g.N + 63) / 64, static_cast<unsigned>((g.M + 63) / 64), static_cast<unsigned>(nz));
    hipLaunchKernelGGL((k_gemm<EPI_STORE>), grid, dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_sum, dim3(static_cast<unsigned>((mn + 255) / 256)), dim3(256), 0, s, work, nz, mn, mn,
                       out);
    return hipGetLastError();
}

// Per-pair diagnostics of surrogate rows and the energy-balance check: diag =
// (A, 4 pi int j dlambda, R, flags) with R = A, or R = rho A when the
// predicted energy ratios rho are given, flags bit 3 (value from the
// surrogate) and bit 4 (|emitted / R - 1| > tol: the pair goes to the plain
// solve); cnt[slot] and cnt[n_slots] count the flagged pairs, and the first
// list_cap flagged pairs (in no particular order) are appended to list.  The
// emitted power is the sum of the n_parts column-slice partials emit[x][r],
// in slice order (a fixed order, so the check decides the same way on every
// run).  Row r of the chunk is selection entry off0 + r of cells from cell0 on
// (n + n_sel < 2^31).
// The reference power of the check: A (rho and bud null), rho A (the
// network's predicted ratio), or the table's budget: A times the slot's node
// ratios bud[row][k] interpolated linearly at the cell's node coordinate t.
__global__ void __launch_bounds__(256) k_sur_diag(const double* A, const float* emit, int n_parts, const float* rho,
                                                  const double* bud, const int* bud_row, int bud_K,
                                                  const double* cell_t, long long cell0, int off0, int n, int n_sel,
                                                  int n_slots, const int* sel, float tol, float* diag, unsigned* cnt,
                                                  long long* list, long long list_cap) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const unsigned rs = static_cast<unsigned>(off0 + r);
    const long long cell = cell0 + rs / static_cast<unsigned>(n_sel);
    const int slot = sel[rs % static_cast<unsigned>(n_sel)];
    const double a = A[r];
    double ref = rho ? a * static_cast<double>(rho[r]) : a;
    if (bud) {
        const double t = cell_t[cell];
        const int k = min(static_cast<int>(t), bud_K - 2);
        const double w = t - k;
        const double* br = bud + static_cast<long long>(bud_row[slot]) * bud_K;
        ref = a * ((1.0 - w) * br[k] + w * br[k + 1]);
    }
    float e = 0.f;
    for (int x = 0; x < n_parts; ++x) e += emit[static_cast<long long>(x) * n + r];
    const bool bad = !(fabs(static_cast<double>(e) / ref - 1.0) <= tol);
    const long long pair = cell * n_slots + slot;
    float* d = diag + pair * 4;
    const float4 v = make_float4(static_cast<float>(a), e, static_cast<float>(ref), bad ? 24.f : 8.f);
    if ((reinterpret_cast<size_t>(diag) & 15) == 0) {
        *reinterpret_cast<float4*>(d) = v;
    } else {
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
    }
    if (bad) {
        atomicAdd(cnt + slot, 1u);
        const unsigned pos = atomicAdd(cnt + n_slots, 1u);
        if (pos < list_cap) list[pos] = pair;
    }
}

// Lists of the flagged pairs per slot (order within a slot is arbitrary; each
// pair's result does not depend on it).
// The same per-slot lists from the check's list of flagged pairs.
__global__ void __launch_bounds__(256) k_fb_scatter_list(const long long* list, long long n, int n_slots,
                                                         const int* seg_off, unsigned* cursor, int* cellmap,
                                                         long long* pairs) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const long long p = list[i];
    const int slot = static_cast<int>(p % n_slots);
    const unsigned pos = atomicAdd(cursor + slot, 1u);
    const long long k = seg_off[slot] + static_cast<long long>(pos);
    cellmap[k] = static_cast<int>(p / n_slots);
    pairs[k] = p;
}

__global__ void __launch_bounds__(256) k_fb_scatter(const float* diag, long long n_pairs, int n_slots,
                                                    const int* seg_off, unsigned* cursor, int* cellmap,
                                                    long long* pairs) {
    const long long p = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= n_pairs) return;
    if (!(static_cast<int>(diag[p * 4 + 3]) & 16)) return;
    const int slot = static_cast<int>(p % n_slots);
    const unsigned pos = atomicAdd(cursor + slot, 1u);
    const long long k = seg_off[slot] + static_cast<long long>(pos);
    cellmap[k] = static_cast<int>(p / n_slots);
    pairs[k] = p;
}


// ---- inference: weight-stationary dense layers on BF16 activations --------------
// A layer out[r][n] = epi(sum_k in[r][k] W[n][k] + b[n]) over many rows r.  A
// block keeps a slice of 128 output columns of W (BF16, all K) in LDS and runs
// row tiles of 64 through it, so the weights are read from memory once per
// block instead of once per row tile.  Each wave owns 16 rows; lane l holds
// row l % 16 and the K/4 contiguous inputs starting at (K/4)(l / 16), which is
// how it feeds v_mfma_f32_16x16x16_bf16: in step s its 4 inputs are
// k = (K/4) q + 4 s + 0..3 (q = l / 16), and the weight fragment it reads
// from LDS uses the same k, so each product still sums over every k once.

// Weights for inference, BF16: W1 padded to K = 64, then W2, W3, W4.
__global__ void __launch_bounds__(256) k_pack_bf16(const float* w, long long oW1, long long oW2, long long oW3,
                                                   long long oW4, int L, unsigned short* wb) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    const long long n1 = 256 * 96, n2 = 256 * 256, n4 = static_cast<long long>(L) * 256;
    if (i < n1) {
        // first layer against [hi | lo | 0] inputs: the 33 weights twice, then zeros
        const int r = static_cast<int>(i / 96), k = static_cast<int>(i % 96);
        wb[i] = k < 66 ? to_bf16(w[oW1 + r * 33 + (k < 33 ? k : k - 33)]) : 0;
    } else if (i < n1 + n2) {
        wb[i] = to_bf16(w[oW2 + (i - n1)]);
    } else if (i < n1 + 2 * n2) {
        wb[i] = to_bf16(w[oW3 + (i - n1 - n2)]);
    } else if (i < n1 + 2 * n2 + n4) {
        wb[i] = to_bf16(w[oW4 + (i - n1 - 2 * n2)]);
    }
}

struct DenseArgs {
    const unsigned short* in;   // [M][K] bf16
    const unsigned short* W;    // [N][K] bf16
    const float* bias;          // [N]
    int M, N;
    unsigned short* out;        // hidden: [M][N] bf16
    // spectrum epilogue
    float* j; int L;            // spectrum rows of L; output column L is the energy ratio
    const float* ym; const float* ys;
    const double* Arow; const float* wq; float* emit;
    float* rho;                 // [M] predicted energy ratio 10^y_L
    long long cell0; int off0;  // row r is selection entry (off0 + r) of cells from cell0 on
    int n_sel, n_slots; const int* sel;
    int sel_shift;              // log2(n_sel) when n_sel is a power of two, else -1
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 128 output columns per block (LDS slice), 128 rows per tile: each wave owns
// 32 rows as two groups of 16, so every weight fragment read from LDS feeds
// two matrix-core products.  v_mfma_f32_16x16x32_bf16 takes 8 inputs per lane;
// step s uses k = (K/4) q + 8 s + 0..7 for lane l (q = l / 16) in both operands.
// SPLIT, hidden layer: each activation is also written as its low BF16 term,
// out rows of 2N (hi, then lo).  SPLIT, output layer: input rows of 2K (hi,
// then lo), both terms multiplied by the same weight fragment.
template <int K, bool SPECTRUM, bool SPLIT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_dense(DenseArgs a) {
    // rows per wave: 2 groups of 16 (hidden layers), 1 group (output layer,
    // whose epilogue needs the registers)
    constexpr int G = SPECTRUM ? 1 : 2;
    constexpr int NB = 128, TM = 64 * G, LDK = K + 8, S = K / 32;
    constexpr int NT = SPECTRUM && SPLIT ? 2 : 1;       // input terms per row
    constexpr int RIN = K * NT;                          // input row length
    __shared__ __align__(16) unsigned short Ws[NB][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // 1-D grid of nsplit column slices x ngrp row-tile groups (ngrp a multiple
    // of 8).  Workgroups go to the 8 XCDs round robin by index, so block L
    // runs on XCD L % 8; the mapping below puts every column slice of a group
    // on the same XCD, where the group's input rows are fetched into L2 once
    const int nsplit = (a.N + NB - 1) / NB;
    const int ngrp = static_cast<int>(gridDim.x) / nsplit;
    const int kk = static_cast<int>(blockIdx.x) >> 3;
    const int slice = kk % nsplit;
    const int grp = (kk / nsplit) * 8 + static_cast<int>(blockIdx.x & 7);
    const int n0 = slice * NB;
    const bool has_ratio = SPECTRUM && n0 <= a.L && a.L < n0 + NB;   // wave-uniform
    // LDS row 16 c + m holds output column colof(c, m) of the slice, m the
    // MFMA column (lane l % 16) of subtile c = 0..7.  Hidden layers: column
    // 8 m + c, so a lane's 8 BF16 results are one 16-byte store and the 16
    // lanes of a row write 256 contiguous bytes.  Output layer (FP32): columns
    // 4 m + c for c < 4 and 64 + 4 m + (c - 4) for c >= 4, so each of the two
    // 16-byte stores per lane and row also covers 256 contiguous bytes.
    auto colof = [](int c, int m) { return SPECTRUM ? (c < 4 ? 4 * m + c : 64 + 4 * m + (c - 4)) : 8 * m + c; };
    for (int e = tid; e < NB * (K / 8); e += 256) {
        const int rr = e / (K / 8), k8 = (e % (K / 8)) * 8;
        const int col = colof(rr >> 4, rr & 15);
        u32x4 v = {0u, 0u, 0u, 0u};
        if (n0 + col < a.N) v = *reinterpret_cast<const u32x4*>(a.W + static_cast<long long>(n0 + col) * K + k8);
        *reinterpret_cast<u32x4*>(&Ws[rr][k8]) = v;
    }
    __syncthreads();
    const int q = lane >> 4, rl = lane & 15;
    const int nc = n0 + 8 * rl;                    // hidden layers: first of this lane's 8 output columns
    const int n_tiles = (a.M + TM - 1) / TM;
    auto load = [&](int t, auto& f) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const long long row = static_cast<long long>(t) * TM + wave * 16 * G + g * 16 + rl;
#pragma unroll
            for (int h = 0; h < NT; ++h) {
                if (t < n_tiles && row < a.M) {
                    const u32x4* src = reinterpret_cast<const u32x4*>(a.in + row * RIN + h * K + (K / 4) * q);
#pragma unroll
                    for (int v = 0; v < S; ++v) f[g][h][v] = src[v];
                } else {
#pragma unroll
                    for (int v = 0; v < S; ++v) f[g][h][v] = u32x4{0u, 0u, 0u, 0u};
                }
            }
        }
    };
    // epilogue constants of this lane's 8 columns, held in registers so that
    // no load sits between the epilogue's stores (the memory counter is in
    // order: a wait for such a load would also wait for every store before it)
    // hidden layers: the biases; output layer: j = A 2^(acc e_c + f_c),
    // e_c = s_c log2(10), f_c = (b_c s_c + m_c) log2(10), and the quadrature weights
    float b8[SPECTRUM ? 1 : 8];
    if constexpr (!SPECTRUM) {
#pragma unroll
        for (int c = 0; c < 8; ++c) b8[c] = a.bias[nc + c < a.N ? nc + c : a.N - 1];
    }
    float e8[SPECTRUM ? 8 : 1], f8[SPECTRUM ? 8 : 1], w8[SPECTRUM ? 8 : 1];
    if constexpr (SPECTRUM) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int nn = n0 + colof(c, rl);
            const int n = nn < a.N ? nn : a.N - 1;
            e8[c] = a.ys[n] * 3.32192809488736235f;
            f8[c] = (a.bias[n] * a.ys[n] + a.ym[n]) * 3.32192809488736235f;
            w8[c] = nn < a.N ? a.wq[n] : 0.f;
        }
    }
    // the next tile's inputs are loaded while this tile computes
    // one tile: computes from cur while the next tile's inputs load into nxt;
    // the two buffers alternate roles (no register copies between tiles)
    using Frag = u32x4[G][NT][S];
    auto tile = [&](const int t, Frag& cur, Frag& nxt) {
        // output layer: destination slot and absorbed power of this lane's 4
        // rows, loaded before the prefetch so the epilogue waits only for them
        int slot4[SPECTRUM ? 4 : 1];
        float A4[SPECTRUM ? 4 : 1];
        if constexpr (SPECTRUM) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = t * TM + wave * 16 + 4 * q + i;
                const unsigned rc = static_cast<unsigned>(a.off0 + (r < a.M ? r : a.M - 1));
                slot4[i] = a.sel[a.sel_shift >= 0 ? (rc & ((1u << a.sel_shift) - 1u))
                                                  : rc % static_cast<unsigned>(a.n_sel)];
                A4[i] = static_cast<float>(a.Arow[r < a.M ? r : a.M - 1]);
            }
        }
        load(t + ngrp, nxt);
        f32x4 acc[G][8];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[g][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < S; ++st) {
            // two subtiles at a time, so that the products into one accumulator
            // are not issued back to back
#pragma unroll
            for (int c = 0; c < 8; c += 2) {
                bf16x8 b[2];
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    b[e] = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const u32x4*>(&Ws[16 * (c + e) + rl][(K / 4) * q + 8 * st]));
#pragma unroll
                for (int h = 0; h < NT; ++h)
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int e = 0; e < 2; ++e)
                            acc[g][c + e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, cur[g][h][st]), b[e], acc[g][c + e], 0, 0, 0);
            }
            // keep each step's weight fragments within the step (bounds register use)
            __builtin_amdgcn_sched_barrier(0);
        }
        // accumulator register i of lane l, subtile c: row 4 q + i of its group
        // of 16, output column nc + c
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long r = static_cast<long long>(t) * TM + wave * 16 * G + g * 16 + 4 * q + i;
                if constexpr (!SPECTRUM) {
                    constexpr int NO = SPLIT ? 2 : 1;             // output terms per activation
                    if (r < a.M) {
                        // BF16 pairs: hi terms, and the lo terms bf16(x - hi)
                        unsigned ph[4], pl[4];
#pragma unroll
                        for (int c = 0; c < 8; c += 2) {
                            const float x0 = gelu_infer(acc[g][c][i] + b8[c]);
                            const float x1 = gelu_infer(acc[g][c + 1][i] + b8[c + 1]);
                            ph[c / 2] = pack_bf16(x0, x1);
                            pl[c / 2] = SPLIT ? pack_bf16(x0 - __uint_as_float(ph[c / 2] << 16),
                                                          x1 - __uint_as_float(ph[c / 2] & 0xFFFF0000u))
                                              : 0u;
                        }
                        unsigned short* orow = a.out + r * (NO * a.N);
                        if (nc + 8 <= a.N) {
                            *reinterpret_cast<u32x4*>(orow + nc) = u32x4{ph[0], ph[1], ph[2], ph[3]};
                            if constexpr (SPLIT)
                                *reinterpret_cast<u32x4*>(orow + a.N + nc) = u32x4{pl[0], pl[1], pl[2], pl[3]};
                        } else {
#pragma unroll
                            for (int c = 0; c < 8; ++c)
                                if (nc + c < a.N) {
                                    orow[nc + c] = static_cast<unsigned short>(ph[c / 2] >> (16 * (c & 1)));
                                    if constexpr (SPLIT)
                                        orow[a.N + nc + c] = static_cast<unsigned short>(pl[c / 2] >> (16 * (c & 1)));
                                }
                        }
                    }
                } else {
                    float part = 0.f;
                    if (r < a.M) {
                        const unsigned rc = static_cast<unsigned>(a.off0 + static_cast<int>(r));
                        const long long cell =
                            a.cell0 + (a.sel_shift >= 0 ? rc >> a.sel_shift : rc / static_cast<unsigned>(a.n_sel));
                        float* jrow = a.j + (cell * a.n_slots + slot4[i]) * a.L;
                        const float Ar = A4[i];
                        float jv[8];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            jv[c] = Ar * __builtin_amdgcn_exp2f(fmaf(acc[g][c][i], e8[c], f8[c]));
                            part += jv[c] * w8[c];
                        }
                        // columns n0 + 4 rl + 0..3 and n0 + 64 + 4 rl + 0..3: the
                        // spectrum below L, the energy ratio at L
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const int cb = n0 + 64 * hh + 4 * rl;
                            if (has_ratio) {        // only the slice that holds column L
#pragma unroll
                                for (int c = 0; c < 4; ++c)
                                    if (cb + c == a.L)
                                        a.rho[r] = __builtin_amdgcn_exp2f(
                                            fmaf(acc[g][4 * hh + c][i], e8[4 * hh + c], f8[4 * hh + c]));
                            }
                            if (cb + 4 <= a.L) {
                                float* dst = jrow + cb;
                                if ((reinterpret_cast<size_t>(dst) & 15) == 0) {
                                    *reinterpret_cast<float4*>(dst) =
                                        make_float4(jv[4 * hh], jv[4 * hh + 1], jv[4 * hh + 2], jv[4 * hh + 3]);
                                } else {
#pragma unroll
                                    for (int c = 0; c < 4; ++c) dst[c] = jv[4 * hh + c];
                                }
                            } else {
#pragma unroll
                                for (int c = 0; c < 4; ++c)
                                    if (cb + c < a.L) jrow[cb + c] = jv[4 * hh + c];
                            }
                        }
                    }
#pragma unroll
                    for (int m = 1; m < 16; m <<= 1) part += __shfl_xor(part, m, 16);
                    if (rl == 0 && r < a.M) a.emit[static_cast<long long>(slice) * a.M + r] = part;
                }
            }
        }
    };
    Frag b0, b1;
    int t = grp;
    load(t, b0);
    for (; t < n_tiles; t += 2 * ngrp) {
        tile(t, b0, b1);
        if (t + ngrp >= n_tiles) break;
        tile(t + ngrp, b1, b0);
    }
}

}  // namespace

// ---- host side ------------------------------------------------------------------------

namespace {

void sur_layout(Sur& s) {
    long long o = 0;
    for (int l = 0; l < 4; ++l) {
        s.off_W[l] = o;
        o += static_cast<long long>(s.widths[l + 1]) * s.widths[l];
        s.off_b[l] = o;
        o += s.widths[l + 1];
    }
    s.n_params = o;
}

}  // namespace

hipError_t sur_alloc(Sur& s) {
    sur_layout(s);
    hipError_t e = hipSuccess;
    auto al = [&](auto*& p, size_t n) {
        if (e == hipSuccess) e = hipMalloc(&p, n * sizeof(*p));
    };
    al(s.w, s.n_params); al(s.g, s.n_params); al(s.m, s.n_params); al(s.v, s.n_params); al(s.we, s.n_params);
    al(s.xm, 33); al(s.xs, 33); al(s.ym, s.n_out); al(s.ys, s.n_out); al(s.wq, s.n_out); al(s.loss, 1 + kLossBlocks);
    if (e == hipSuccess) e = hipMemset(s.m, 0, sizeof(float) * s.n_params);
    if (e == hipSuccess) e = hipMemset(s.v, 0, sizeof(float) * s.n_params);
    if (e == hipSuccess) {
        std::vector<float> wq(s.n_out, 0.f);   // the ratio output carries no weight
        const std::vector<double>& lam = s.c->lam_host;
        for (int j = 0; j + 1 < s.L; ++j) {
            const double h = 0.5 * (lam[j + 1] - lam[j]) * 4.0 * kPi;
            wq[j] += static_cast<float>(h);
            wq[j + 1] += static_cast<float>(h);
        }
        e = hipMemcpy(s.wq, wq.data(), sizeof(float) * s.n_out, hipMemcpyHostToDevice);
    }
    // trapezoid half-segments of every node (to its left and right) and the
    // band of every segment, for the band-weighted loss
    al(s.bw_l, s.L); al(s.bw_r, s.L); al(s.segband, std::max(s.L - 1, 1)); al(s.bedge, kBands + 1);
    if (e == hipSuccess) {
        const std::vector<double>& lam = s.c->lam_host;
        const int L = s.L;
        std::vector<float> l(L, 0.f), r(L, 0.f);
        std::vector<int> sb(std::max(L - 1, 1), 0), be(kBands + 1);
        for (int k = 0; k < L; ++k) {
            if (k > 0) l[k] = static_cast<float>(0.5 * (lam[k] - lam[k - 1]));
            if (k + 1 < L) r[k] = static_cast<float>(0.5 * (lam[k + 1] - lam[k]));
        }
        for (int q = 0; q <= kBands; ++q) be[q] = static_cast<int>((static_cast<long long>(q) * (L - 1)) / kBands);
        for (int q = 0; q < kBands; ++q)
            for (int k = be[q]; k < be[q + 1]; ++k) sb[k] = q;
        e = hipMemcpy(s.bw_l, l.data(), sizeof(float) * L, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.bw_r, r.data(), sizeof(float) * L, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.segband, sb.data(), sizeof(int) * sb.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.bedge, be.data(), sizeof(int) * be.size(), hipMemcpyHostToDevice);
    }
    return e;
}

void sur_free(Sur& s) {
    for (float* p : {s.w, s.g, s.m, s.v, s.we, s.xm, s.xs, s.ym, s.ys, s.wq, s.Xb, s.Yb, s.Yh, s.dY, s.Wb, s.bw_l,
                     s.bw_r})
        (void)hipFree(p);
    (void)hipFree(s.segband);
    (void)hipFree(s.bedge);
    for (int i = 0; i < 3; ++i) {
        (void)hipFree(s.Z[i]);
        (void)hipFree(s.H[i]);
    }
    for (int i = 0; i < 2; ++i) (void)hipFree(s.dZ[i]);
    (void)hipFree(s.idx);
    (void)hipFree(s.loss);
    (void)hipFree(s.split_work);
    (void)hipFree(s.wb);
}

hipError_t sur_grow(Sur& s, int B) {
    if (B <= s.cap_B) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    for (float* p : {s.Xb, s.Yb, s.Yh, s.dY, s.Wb}) (void)hipFree(p);
    for (int i = 0; i < 3; ++i) {
        (void)hipFree(s.Z[i]);
        (void)hipFree(s.H[i]);
        s.Z[i] = s.H[i] = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(s.dZ[i]);
        s.dZ[i] = nullptr;
    }
    (void)hipFree(s.idx);
    s.Xb = s.Yb = s.Yh = s.dY = s.Wb = nullptr;
    s.idx = nullptr;
    s.cap_B = 0;
    auto al = [&](auto*& p, size_t n) {
        if (e == hipSuccess) e = hipMalloc(&p, n * sizeof(*p));
    };
    const size_t b = static_cast<size_t>(B);
    al(s.Xb, b * 33); al(s.Yb, b * s.n_out); al(s.Yh, b * s.n_out); al(s.dY, b * s.n_out); al(s.Wb, b * s.n_out);
    for (int i = 0; i < 3; ++i) {
        al(s.Z[i], b * 256);
        al(s.H[i], b * 256);
    }
    al(s.dZ[0], b * 256); al(s.dZ[1], b * 256);
    al(s.idx, b);
    // split K so that the weight-gradient products (at most 500 x 256 outputs,
    // K = batch) spread over a few hundred blocks
    s.splits = std::max(1, std::min(32, B / 256));
    (void)hipFree(s.split_work);
    s.split_work = nullptr;
    al(s.split_work, static_cast<size_t>(s.splits) * std::max(s.n_out, 256) * 256 +
                         static_cast<size_t>((B + 31) / 32) * std::max(s.n_out, 256));
    if (e == hipSuccess) s.cap_B = B;
    return e;
}

hipError_t sur_bands(const Ctx& c, const double* u, int n_cells, float* bands, hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bands, dim3((n_cells + 3) / 4), dim3(256), 0, st, u, c.lam, n_cells, c.L, bands);
    return hipGetLastError();
}

hipError_t sur_wc(const Ctx& c, const double* const* cabs, int n_sel, double* wcT, hipStream_t st) {
    const int n = n_sel * c.L;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wc, dim3((n + 255) / 256), dim3(256), 0, st, cabs, c.lam, n_sel, c.L, wcT);
    return hipGetLastError();
}

hipError_t sur_pairs(const Ctx& c, const double* u, const float* bands, const double* wcT, const float* loga,
                     long long row0, long long n_rows, int n_sel, float* X, double* A, unsigned short* xb,
                     const float* xm, const float* xs, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const long long cell0 = row0 / n_sel;
    const long long cell1 = (row0 + n_rows - 1) / n_sel;
    PairArgs p{u, bands, wcT, loga, row0, n_rows, cell0, cell1 - cell0 + 1, n_sel, c.L, X, A, xb, xm, xs};
    // grain slots per block: the smallest of 16 / 32 / 64 that holds the
    // selection (64 and several blocks across it beyond that)
    const int S = n_sel <= 16 ? 16 : n_sel <= 32 ? 32 : 64;
    const int C = 512 / S;
    const dim3 grid(static_cast<unsigned>((p.n_cells + C - 1) / C), static_cast<unsigned>((n_sel + S - 1) / S));
    if (S == 16) hipLaunchKernelGGL(k_pairs<16>, grid, dim3(256), 0, st, p);
    else if (S == 32) hipLaunchKernelGGL(k_pairs<32>, grid, dim3(256), 0, st, p);
    else hipLaunchKernelGGL(k_pairs<64>, grid, dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t sur_targets(const float* j, const double* A, const double* lam, long long n, int L, float* Y,
                       hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_targets, dim3(static_cast<unsigned>((n + 3) / 4)), dim3(256), 0, st, j, A, lam, n, L, Y);
    return hipGetLastError();
}

// Column means and standard deviations of a [n][w] FP32 matrix (FP64 sums in
// a fixed order: the same bits on every run).
hipError_t sur_colstats(const float* Xm, long long n, int w, std::vector<double>& mean, std::vector<double>& sd) {
    const long long rpb = 1024;
    const int nblk = static_cast<int>((n + rpb - 1) / rpb);
    double* d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(double) * 2 * w * (static_cast<size_t>(nblk) + 1));
    double* tot = d + static_cast<size_t>(nblk) * 2 * w;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colstats, dim3(static_cast<unsigned>(nblk), (w + 255) / 256), dim3(256), 0, nullptr, Xm,
                           n, w, rpb, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colstats_sum, dim3((2 * w + 255) / 256), dim3(256), 0, nullptr, d, nblk, 2 * w, tot);
        e = hipGetLastError();
    }
    std::vector<double> h(2 * w);
    if (e == hipSuccess) e = hipMemcpy(h.data(), tot, sizeof(double) * 2 * w, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return e;
    mean.resize(w);
    sd.resize(w);
    for (int k = 0; k < w; ++k) {
        mean[k] = h[k] / n;
        const double var = h[w + k] / n - mean[k] * mean[k];
        sd[k] = var > 0.0 ? std::sqrt(var) : 1.0;
    }
    return hipSuccess;
}

namespace {

GemmArgs nt(const float* A, int lda, const float* W, int ldw, float* C, int ldc, int M, int N, int K) {
    // C[M][N] = A[M][K] . W[N][K]^T
    GemmArgs g{};
    g.A = A; g.sai = lda; g.sak = 1;
    g.B = W; g.sbk = 1; g.sbj = ldw;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    return g;
}

}  // namespace

// Forward pass of a batch of B normalised rows Xb [B][33]; keeps the
// pre-activations Z and activations H (training) and writes the output Yh.
// The inputs of the first and the last layer enter as two BF16 terms each.
hipError_t sur_forward(Sur& s, int B, const float* Xb, hipStream_t st, bool keep_z) {
    hipError_t e = hipSuccess;
    const float* h = Xb;
    int in = 33;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        GemmArgs g = nt(h, in, s.w + s.off_W[l], in, keep_z ? s.Z[l] : nullptr, 256, B, 256, in);
        g.asplit = kSplitIn[l];
        g.C2 = s.H[l];
        g.ldc2 = 256;
        g.bias = s.w + s.off_b[l];
        e = gemm<EPI_BIAS_GELU>(g, st);
        h = s.H[l];
        in = 256;
    }
    if (e != hipSuccess) return e;
    GemmArgs g = nt(h, 256, s.w + s.off_W[3], 256, s.Yh, s.n_out, B, s.n_out, 256);
    g.asplit = kSplitIn[3];
    g.bias = s.w + s.off_b[3];
    return gemm<EPI_BIAS>(g, st);
}

// Backward pass from dY (= dL/dYh) into s.g (weights and biases).
hipError_t sur_backward(Sur& s, int B, const float* Xb, hipStream_t st) {
    hipError_t e = hipSuccess;
    const float* dz = s.dY;
    int nout = s.n_out;
    for (int l = 3; l >= 0 && e == hipSuccess; --l) {
        const int nin = s.widths[l];
        const float* hin = l > 0 ? s.H[l - 1] : Xb;
        // dW[nout][nin] = dz^T [nout][B] . hin [B][nin]
        GemmArgs g{};
        g.A = dz; g.sai = 1; g.sak = nout;
        g.B = hin; g.sbk = nin; g.sbj = 1;
        g.C = s.g + s.off_W[l]; g.ldc = nin;
        g.M = nout; g.N = nin; g.K = B;
        e = gemm_splitk(g, s.splits, s.split_work, st);
        if (e != hipSuccess) break;
        const int nchunk = (B + 31) / 32;
        hipLaunchKernelGGL(k_colsum, dim3((nout + 255) / 256, nchunk), dim3(256), 0, st, dz, B, nout, s.split_work);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_split_sum, dim3((nout + 255) / 256), dim3(256), 0, st, s.split_work, nchunk,
                               static_cast<long long>(nout), static_cast<long long>(nout), s.g + s.off_b[l]);
            e = hipGetLastError();
        }
        if (e != hipSuccess || l == 0) break;
        // dz_prev[B][nin] = (dz [B][nout] . W [nout][nin]) * gelu'(Z[l-1])
        float* dzp = s.dZ[l % 2];
        GemmArgs h{};
        h.A = dz; h.sai = nout; h.sak = 1;
        h.B = s.w + s.off_W[l]; h.sbk = nin; h.sbj = 1;
        h.C = dzp; h.ldc = nin;
        h.aux = s.Z[l - 1]; h.ldaux = 256;
        h.M = B; h.N = nin; h.K = nout;
        e = gemm<EPI_GELU_BWD>(h, st);
        dz = dzp;
        nout = nin;
    }
    return e;
}

hipError_t sur_loss(Sur& s, int B, hipStream_t st) {
    const long long n = static_cast<long long>(B) * s.n_out;
    const int blocks = static_cast<int>(std::min<long long>(kLossBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(k_loss, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, s.Yh, s.Yb,
                       s.band_weight > 0.f ? s.Wb : nullptr, n, 2.0f / static_cast<float>(n), s.dY, s.loss + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(64), 0, st, s.loss + 1, blocks, s.loss);
    return hipGetLastError();
}

hipError_t sur_gather(Sur& s, const float* X, const float* Y, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(B), dim3(256), 0, st, X, Y, s.idx, B, s.n_out, s.xm, s.xs, s.ym, s.ys, s.Xb, s.Yb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && Y && s.band_weight > 0.f) {
        hipLaunchKernelGGL(k_loss_weights, dim3(B), dim3(256), 0, st, Y, s.idx, s.L, s.n_out, s.bw_l, s.bw_r,
                           s.segband, s.bedge, s.band_weight, s.Wb);
        e = hipGetLastError();
    }
    return e;
}

hipError_t sur_batch_idx(Sur& s, unsigned long long seed, long long step, int B, long long n, hipStream_t st,
                         const long long* ctr) {
    hipLaunchKernelGGL(k_batch_idx, dim3((B + 255) / 256), dim3(256), 0, st, seed, step, ctr, B, n, s.idx);
    return hipGetLastError();
}

hipError_t sur_seq_idx(Sur& s, long long first, int B, hipStream_t st) {
    std::vector<long long> h(B);
    for (int b = 0; b < B; ++b) h[b] = first + b;
    hipError_t e = hipMemcpyAsync(s.idx, h.data(), sizeof(long long) * B, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

float2 adam_step_sizes(float lr, long long t) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - std::pow(b1, static_cast<double>(t));
    const double c2 = 1.0 - std::pow(b2, static_cast<double>(t));
    // w -= lr (m / c1) / (sqrt(v / c2) + eps) = lr sqrt(c2) / c1 * m / (sqrt(v) + eps sqrt(c2))
    return make_float2(static_cast<float>(lr * std::sqrt(c2) / c1), static_cast<float>(eps * std::sqrt(c2)));
}

hipError_t sur_adam(Sur& s, float lr, hipStream_t st, bool ema, float ema_decay) {
    ++s.t;
    s.wb_fresh = false;
    const float2 p = adam_step_sizes(lr, s.t);
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((s.n_params + 255) / 256)), dim3(256), 0, st, s.w, s.g,
                       s.m, s.v, s.n_params, p.x, 0.9f, 0.999f, p.y, ema ? s.we : nullptr, ema_decay,
                       static_cast<const float2*>(nullptr), static_cast<const long long*>(nullptr), 0LL);
    return hipGetLastError();
}

hipError_t sur_adam_sched(Sur& s, const float2* sched, const long long* ctr, long long t0, hipStream_t st, bool ema,
                          float ema_decay) {
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((s.n_params + 255) / 256)), dim3(256), 0, st, s.w, s.g,
                       s.m, s.v, s.n_params, 0.f, 0.9f, 0.999f, 0.f, ema ? s.we : nullptr, ema_decay, sched, ctr, t0);
    return hipGetLastError();
}

hipError_t sur_step_end(long long* ctr, long long t0, const double* loss, double* trace, hipStream_t st) {
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, ctr, t0, loss, trace);
    return hipGetLastError();
}

// Weights in BF16 for inference (packed once per parameter change).
hipError_t sur_pack(Sur& s, hipStream_t st) {
    if (s.wb_fresh) return hipSuccess;
    const long long n = 256LL * 96 + 2LL * 256 * 256 + static_cast<long long>(s.n_out) * 256;
    if (!s.wb) {
        const hipError_t e = hipMalloc(&s.wb, sizeof(unsigned short) * n);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_pack_bf16, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, s.w, s.off_W[0],
                       s.off_W[1], s.off_W[2], s.off_W[3], s.n_out, s.wb);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) s.wb_fresh = true;
    return e;
}

namespace {

template <int K, bool SPEC, bool SPLIT>
hipError_t dense(const DenseArgs& a, hipStream_t st) {
    const int nsplit = (a.N + 127) / 128;
    const int n_tiles = (a.M + (SPEC ? 63 : 127)) / (SPEC ? 64 : 128);
    // two blocks per CU fit (LDS): about 512 blocks over the column slices;
    // row-tile groups in multiples of 8 (one per XCD, see the kernel)
    const int ngrp = (std::max(1, std::min(n_tiles, 512 / nsplit)) + 7) / 8 * 8;
    hipLaunchKernelGGL((k_dense<K, SPEC, SPLIT>), dim3(nsplit * ngrp), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

// Inference of rows [row0, row0 + M) of a selection from the normalised
// inputs xb [M][96] (hi and lo terms, as sur_pairs writes them): spectra
// scattered to j (pair rows); emit[x][r] = 4 pi int j dlambda over the
// wavelengths of column slice x (sur_emit_parts(n_out) slices of 128);
// rho[r] = the predicted energy ratio.  Workspaces: h0 [M][512], h1 [M][256]
// BF16.
hipError_t sur_infer_rows(Sur& s, int M, const unsigned short* xb, const double* A, long long row0, int n_sel,
                          int n_slots, const int* sel, float* j, float* emit, float* rho, unsigned short* h0,
                          unsigned short* h1, hipStream_t st) {
    if (M <= 0) return hipSuccess;
    if (static_cast<long long>(M) + n_sel >= (1LL << 31)) return hipErrorInvalidValue;
    hipError_t e = sur_pack(s, st);
    if (e != hipSuccess) return e;
    const unsigned short* W1 = s.wb;
    const unsigned short* W2 = W1 + 256 * 96;
    const unsigned short* W3 = W2 + 256 * 256;
    const unsigned short* W4 = W3 + 256 * 256;
    DenseArgs d{};
    d.M = M;
    d.N = 256;
    d.in = xb; d.W = W1; d.bias = s.w + s.off_b[0]; d.out = h0;
    e = dense<96, false, false>(d, st);
    if (e != hipSuccess) return e;
    d.in = h0; d.W = W2; d.bias = s.w + s.off_b[1]; d.out = h1;
    e = dense<256, false, false>(d, st);
    if (e != hipSuccess) return e;
    // last hidden layer: hi and lo terms for the output layer
    d.in = h1; d.W = W3; d.bias = s.w + s.off_b[2]; d.out = h0;
    e = dense<256, false, true>(d, st);
    if (e != hipSuccess) return e;
    DenseArgs o{};
    o.in = h0; o.W = W4; o.bias = s.w + s.off_b[3]; o.M = M; o.N = s.n_out;
    o.j = j; o.L = s.L; o.ym = s.ym; o.ys = s.ys; o.Arow = A; o.wq = s.wq; o.emit = emit; o.rho = rho;
    // M + n_sel < 2^31 (one chunk), so the row arithmetic fits 32 bits
    o.cell0 = row0 / n_sel; o.off0 = static_cast<int>(row0 - o.cell0 * n_sel);
    o.n_sel = n_sel; o.n_slots = n_slots; o.sel = sel;
    o.sel_shift = -1;
    for (int b = 0; b < 31; ++b)
        if (n_sel == (1 << b)) o.sel_shift = b;
    return dense<256, true, true>(o, st);
}

int sur_emit_parts(int n_out) { return (n_out + 127) / 128; }

hipError_t sur_diag(const double* A, const float* emit, int n_parts, const float* rho, const double* bud,
                    const int* bud_row, int bud_K, const double* cell_t, long long row0, long long n, int n_sel,
                    int n_slots, const int* sel, float tol, float* diag, unsigned* cnt, long long* list,
                    long long list_cap, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n + n_sel >= (1LL << 31)) return hipErrorInvalidValue;
    const long long cell0 = row0 / n_sel;
    const int off0 = static_cast<int>(row0 - cell0 * n_sel);
    hipLaunchKernelGGL(k_sur_diag, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, A, emit, n_parts,
                       rho, bud, bud_row, bud_K, cell_t, cell0, off0, static_cast<int>(n), n_sel, n_slots, sel, tol,
                       diag, cnt, list, list_cap);
    return hipGetLastError();
}

hipError_t sur_fb_scatter_list(const long long* list, long long n, int n_slots, const int* seg_off, unsigned* cursor,
                               int* cellmap, long long* pairs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fb_scatter_list, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, list, n,
                       n_slots, seg_off, cursor, cellmap, pairs);
    return hipGetLastError();
}

hipError_t sur_fb_scatter(const float* diag, long long n_pairs, int n_slots, const int* seg_off, unsigned* cursor,
                          int* cellmap, long long* pairs, hipStream_t st) {
    if (n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fb_scatter, dim3(static_cast<unsigned>((n_pairs + 255) / 256)), dim3(256), 0, st, diag,
                       n_pairs, n_slots, seg_off, cursor, cellmap, pairs);
    return hipGetLastError();
}

}  // namespace hsd
