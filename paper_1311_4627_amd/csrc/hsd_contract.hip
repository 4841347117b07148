// Emission contraction and per-pair energy diagnostics.
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
    const int row0 = blockIdx.y * BM;          // first cell of the tile
    const int col0 = blockIdx.x * BN;          // first wavelength of the tile
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
            const float ps = a.pscale[static_cast<size_t>(row) * a.n_gslots + a.gslot];
            float* jrow = a.j + (static_cast<size_t>(row) * a.n_gslots + a.gslot) * a.L;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int col = col0 + wc + bj * 16 + (lane & 15);
                if (col < a.L) jrow[col] = acc[bi][bj][i] * ps * a.bscale[col];
            }
        }
    }
}

// Energy bookkeeping of one pair per wavefront: emitted power 4 pi int j dlambda
// and the representable absorbed power A_rep = sum_i P_i Cum_(jrep(i)), with
// Cum_j = int_{lambda_j} c u C_abs dlambda (trapezoid), all in FP64.
__global__ void __launch_bounds__(256) k_diag(DiagLaunch a) {
    extern __shared__ double cum_s[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cell_raw = blockIdx.x * 4 + wave;
    const bool valid = cell_raw < a.n_cells;
    const int cell = valid ? cell_raw : a.n_cells - 1;   // dead waves still reach the barriers
    const int L = a.L;
    double* cum = cum_s + wave * (L + 1);
    const size_t pair = static_cast<size_t>(cell) * a.n_gslots + a.gslot;
    const float* jr = a.j + pair * L;
    double em = 0.0;
    for (int j = lane; j + 1 < L; j += 64) em += 0.5 * (static_cast<double>(jr[j]) + jr[j + 1]) * (a.lam[j + 1] - a.lam[j]);
    const double* uc = a.u + static_cast<size_t>(cell) * L;
    // segment integrals, then a serial suffix sum per 64-entry chunk and chunk carries
    for (int j = lane; j < L; j += 64) {
        double s = 0.0;
        if (j + 1 < L) {
            const double u0 = uc[j] >= 0.0 && uc[j] < INFINITY ? uc[j] : 0.0;
            const double u1 = uc[j + 1] >= 0.0 && uc[j + 1] < INFINITY ? uc[j + 1] : 0.0;
            s = 0.5 * kLight * (u0 * a.cabs[j] + u1 * a.cabs[j + 1]) * (a.lam[j + 1] - a.lam[j]);
        }
        cum[j] = s;
    }
    __syncthreads();
    if (lane == 0) {
        double run = 0.0;
        cum[L] = 0.0;
        for (int j = L - 1; j >= 0; --j) {
            run += cum[j];
            cum[j] = run;
        }
    }
    __syncthreads();
    const float* prow = a.Pt + static_cast<size_t>(cell) * a.nb;
    const double ps = a.pscale[pair];
    double ar = 0.0;
    for (int i = lane; i < a.nb; i += 64) {
        const int jr_i = a.jrep[i];
        ar += static_cast<double>(prow[i]) * ps * cum[jr_i < L ? jr_i : L];
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        em += __shfl_xor(em, m, 64);
        ar += __shfl_xor(ar, m, 64);
    }
    if (lane == 0 && valid) {
        a.diag[pair * 4 + 1] = static_cast<float>(4.0 * kPi * em);
        a.diag[pair * 4 + 2] = static_cast<float>(ar);
    }
}

}  // namespace

hipError_t launch_contract(const ContractLaunch& a, hipStream_t s) {
    if (a.n_cells <= 0) return hipSuccess;
    dim3 grid(a.Lp / BN, (a.n_cells + BM - 1) / BM);
    hipLaunchKernelGGL(k_contract, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_diag(const DiagLaunch& a, hipStream_t s) {
    if (a.n_cells <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 4 * (a.L + 1);
    hipLaunchKernelGGL(k_diag, dim3((a.n_cells + 3) / 4), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace hsd
