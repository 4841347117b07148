// Emission contraction and the emitted-power diagnostic.
//
// j[c, g, lambda] = C_abs(lambda) sum_i P_i B_lambda(T_i) [E_i >= hc/lambda]
// (Sec. 2.3, eq:emission with eq:emission-lambda) is, for one grain g and all
// cells, a dense product (cells x bins) . (bins x wavelengths).  The solver
// stores P~ = P / max P in single precision and the grain table holds
// B~ = C_abs B_lambda(T_i) [..] / s_lambda with s_lambda its column maximum, so
// both operands lie in [0, 1]; the product runs on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32) with FP32 accumulation and the epilogue restores
// j = (P~ B~) * maxP * s_lambda.
#include <cmath>

#include "hsd_internal.h"

namespace hsd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int APAD = 1, BPAD = 4;
constexpr int BK3 = 64, LK3 = BK3 + 8;      // split-BF16 kernel: k per step, LDS row length (ushorts)

// One 256-thread block computes a 64 (cells) x 64 (wavelengths) tile; each of
// its four waves owns a 32 x 32 quarter as 2 x 2 MFMA 16x16 blocks.
// Operand layout of v_mfma_f32_16x16x4_f32: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator register i of lane l is
// D[4 (l / 16) + i][l % 16].
__global__ void __launch_bounds__(256) k_contract(ContractLaunch a) {
    __shared__ float As[BM][BK + APAD];
    __shared__ float Bs[BK][BN + BPAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // Workgroup b runs on XCD b % 8; each XCD takes whole row tiles with all
    // their wavelength tiles in a row, so a tile's P~ rows are read from HBM
    // once and then served by that XCD's L2.
    const int nlt = a.Lp / BN;
    const int b = blockIdx.x;
    const int m = b / 8;
    const int rt = 8 * (m / nlt) + (b % 8);
    if (rt * BM >= a.n_cells) return;          // padding tile: the whole block leaves before any barrier
    const int row0 = rt * BM;                  // first cell of the tile
    const int col0 = (m % nlt) * BN;           // first wavelength of the tile
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int ar = tid >> 2, ak = (tid & 3) * 4;      // A tile loader: row, k offset
    const int bk = tid >> 4, bc = (tid & 15) * 4;     // B tile loader: k row, column offset
    const bool arow_ok = (row0 + ar) < a.n_cells;
    const float* Arow = a.Pt + static_cast<size_t>(row0 + ar) * a.nb;

    for (int k0 = 0; k0 < a.nb; k0 += BK) {
        float4 av = make_float4(0.f, 0.f, 0.f, 0.f);
        if (arow_ok) av = *reinterpret_cast<const float4*>(Arow + k0 + ak);
        const float4 bv = *reinterpret_cast<const float4*>(a.Bt + static_cast<size_t>(k0 + bk) * a.Lp + col0 + bc);
        As[ar][ak + 0] = av.x;
        As[ar][ak + 1] = av.y;
        As[ar][ak + 2] = av.z;
        As[ar][ak + 3] = av.w;
        *reinterpret_cast<float4*>(&Bs[bk][bc]) = bv;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float af[2], bf[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) af[bi] = As[wr + bi * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) bf[bj] = Bs[kk + (lane >> 4)][wc + bj * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[bi], bf[bj], acc[bi][bj], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + wr + bi * 16 + 4 * (lane >> 4) + i;
            if (row >= a.n_cells) continue;
            const size_t cell = a.rowmap ? static_cast<size_t>(a.rowmap[row]) : static_cast<size_t>(row);
            const float ps = a.pscale[cell * a.n_gslots + a.gslot];
            float* jrow = a.j + (cell * a.n_gslots + a.gslot) * a.L;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int col = col0 + wc + bj * 16 + (lane & 15);
                if (col < a.L) jrow[col] = acc[bi][bj][i] * ps * a.bscale[col];
            }
        }
    }
}

// The same product with each operand split into two BF16 terms, x = hi + lo
// (hi = bf16(x), lo = bf16(x - hi)), and hi hi + hi lo + lo hi accumulated in
// FP32 on v_mfma_f32_16x16x32_bf16 (16 times the FP32 matrix-core rate; the
// dropped lo lo term and the split's remainders keep every product within
// 3 2^-16 of exact).  P~ is split as it is staged in LDS; the grain's table
// comes pre-split and transposed (Bh, Bl: [Lp][nbp], nbp a multiple of 64).  Same tiles, XCD order
// and epilogue as k_contract; in step s lane l supplies row l % 16 of its A
// block with k = 8 (l / 16) + 0..7 and column l % 16 of its B block with the
// same k, so every product still sums over each k once.
typedef unsigned int u32x4c __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned pack_hi2(float x0, float x1, unsigned& lo) {
    const __bf16 h0 = static_cast<__bf16>(x0), h1 = static_cast<__bf16>(x1);
    const __bf16 l0 = static_cast<__bf16>(x0 - static_cast<float>(h0));
    const __bf16 l1 = static_cast<__bf16>(x1 - static_cast<float>(h1));
    lo = __builtin_bit_cast(unsigned short, l0) | (static_cast<unsigned>(__builtin_bit_cast(unsigned short, l1)) << 16);
    return __builtin_bit_cast(unsigned short, h0) | (static_cast<unsigned>(__builtin_bit_cast(unsigned short, h1)) << 16);
}

__global__ void __launch_bounds__(256) k_contract3(ContractLaunch a) {
    __shared__ __align__(16) unsigned short Ah[BM][LK3];
    __shared__ __align__(16) unsigned short Al[BM][LK3];
    __shared__ __align__(16) unsigned short Bhs[BN][LK3];
    __shared__ __align__(16) unsigned short Bls[BN][LK3];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nlt = a.Lp / BN;
    const int b = blockIdx.x;
    const int m = b / 8;
    const int rt = 8 * (m / nlt) + (b % 8);
    if (rt * BM >= a.n_cells) return;          // padding tile: the whole block leaves before any barrier
    const int row0 = rt * BM;
    const int col0 = (m % nlt) * BN;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    // loaders: thread t stages row (or column) t / 4, k = 16 (t % 4) + 0..15
    const int lr = tid >> 2, lk = (tid & 3) * 16;
    const bool arow_ok = (row0 + lr) < a.n_cells;
    const float* Arow = a.Pt + static_cast<size_t>(row0 + lr) * a.nb;
    const size_t boff = static_cast<size_t>(col0 + lr) * a.nbp + lk;
    const int rl = lane & 15, q = lane >> 4;
    // the next step's operands are loaded into registers while this step's
    // products run
    float4 v[4];
    u32x4c bh[2], bl[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k0 < a.nbp) {
            if (arow_ok && k0 + lk < a.nb) {      // nb is a multiple of 16: a chunk is wholly inside or outside
#pragma unroll
                for (int c = 0; c < 4; ++c) v[c] = *reinterpret_cast<const float4*>(Arow + k0 + lk + 4 * c);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                bh[c] = *reinterpret_cast<const u32x4c*>(a.Bh + boff + k0 + 8 * c);
                bl[c] = *reinterpret_cast<const u32x4c*>(a.Bl + boff + k0 + 8 * c);
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < a.nbp; k0 += BK3) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            unsigned l0, l1, l2, l3;
            const unsigned h0 = pack_hi2(v[2 * c].x, v[2 * c].y, l0), h1 = pack_hi2(v[2 * c].z, v[2 * c].w, l1);
            const unsigned h2 = pack_hi2(v[2 * c + 1].x, v[2 * c + 1].y, l2);
            const unsigned h3 = pack_hi2(v[2 * c + 1].z, v[2 * c + 1].w, l3);
            const u32x4c ahv = {h0, h1, h2, h3}, alv = {l0, l1, l2, l3};
            *reinterpret_cast<u32x4c*>(&Ah[lr][lk + 8 * c]) = ahv;
            *reinterpret_cast<u32x4c*>(&Al[lr][lk + 8 * c]) = alv;
            *reinterpret_cast<u32x4c*>(&Bhs[lr][lk + 8 * c]) = bh[c];
            *reinterpret_cast<u32x4c*>(&Bls[lr][lk + 8 * c]) = bl[c];
        }
        __syncthreads();
        fetch(k0 + BK3);
#pragma unroll
        for (int ks = 0; ks < BK3; ks += 32) {
            bf16x8c ah[2], al[2], bhf[2], blf[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ah[t] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&Ah[wr + 16 * t + rl][ks + 8 * q]));
                al[t] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&Al[wr + 16 * t + rl][ks + 8 * q]));
                bhf[t] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&Bhs[wc + 16 * t + rl][ks + 8 * q]));
                blf[t] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&Bls[wc + 16 * t + rl][ks + 8 * q]));
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bhf[bj], acc[bi][bj], 0, 0, 0);
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], blf[bj], acc[bi][bj], 0, 0, 0);
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[bi], bhf[bj], acc[bi][bj], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + wr + bi * 16 + 4 * (lane >> 4) + i;
            if (row >= a.n_cells) continue;
            const size_t cell = a.rowmap ? static_cast<size_t>(a.rowmap[row]) : static_cast<size_t>(row);
            const float ps = a.pscale[cell * a.n_gslots + a.gslot];
            float* jrow = a.j + (cell * a.n_gslots + a.gslot) * a.L;
            for (int bj = 0; bj < 2; ++bj) {
                const int col = col0 + wc + bj * 16 + (lane & 15);
                if (col < a.L) jrow[col] = acc[bi][bj][i] * ps * a.bscale[col];
            }
        }
    }
}

// Emitted power of each pair, 4 pi int j dlambda (trapezoid, FP64 sum), one
// 16-lane segment per pair; the other diagnostics come from the solver.
__global__ void __launch_bounds__(256) k_diag(DiagLaunch a) {
    const int lane = threadIdx.x & 15;
    const size_t k = static_cast<size_t>(blockIdx.x) * 16 + (threadIdx.x >> 4);
    const size_t n_k = a.pairs ? static_cast<size_t>(a.n_list) : static_cast<size_t>(a.n_cells) * a.n_gslots;
    const bool valid = k < n_k;
    const size_t pair = !valid ? 0 : (a.pairs ? static_cast<size_t>(a.pairs[k]) : k);
    const float* jr = a.j + (valid ? pair : 0) * a.L;
    double em = 0.0;
    for (int j = lane; j + 1 < a.L; j += 16)
        em += 0.5 * (static_cast<double>(jr[j]) + jr[j + 1]) * (a.lam[j + 1] - a.lam[j]);
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) em += __shfl_xor(em, m, 16);
    if (lane == 0 && valid) a.diag[pair * 4 + 1] = static_cast<float>(4.0 * kPi * em);
}

// Size-distribution convolution (Sec. 2.3, eq:convolution on the size grid):
// out[c][l] = (lambda_l if lw) * sum_g w_g j[c][g][l], FP64 sums; one thread
// per (cell, wavelength), consecutive threads on consecutive wavelengths.
__global__ void __launch_bounds__(256) k_sizedist(const float* j, const double* w, const double* lam, int n_cells,
                                                  int G, int L, int lw, double* out) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= static_cast<long long>(n_cells) * L) return;
    const long long c = i / L;
    const int l = static_cast<int>(i - c * L);
    const float* jc = j + c * G * L + l;
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc = fma(w[g], static_cast<double>(jc[static_cast<long long>(g) * L]), acc);
    out[i] = lw ? acc * lam[l] : acc;
}

}  // namespace

hipError_t launch_contract(const ContractLaunch& a, hipStream_t s) {
    if (a.n_cells <= 0) return hipSuccess;
    const int nrt8 = ((a.n_cells + BM - 1) / BM + 7) / 8 * 8;
    if (a.mode == 1) {
        if (!a.Bh || !a.Bl || a.nbp < a.nb || a.nbp % BK3 != 0 || a.nb % 16 != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_contract3, dim3(nrt8 * (a.Lp / BN)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_contract, dim3(nrt8 * (a.Lp / BN)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_diag(const DiagLaunch& a, hipStream_t s) {
    const size_t n_pairs = a.pairs ? static_cast<size_t>(a.n_list) : static_cast<size_t>(a.n_cells) * a.n_gslots;
    if (n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag, dim3(static_cast<unsigned>((n_pairs + 15) / 16)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sizedist(const float* j, const double* w, const double* lam, int n_cells, int G, int L, int lw,
                           double* out, hipStream_t s) {
    const long long n = static_cast<long long>(n_cells) * L;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sizedist, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, j, w, lam, n_cells, G,
                       L, lw, out);
    return hipGetLastError();
}

}  // namespace hsd
