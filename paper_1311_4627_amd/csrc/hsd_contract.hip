// Emission contraction and the emitted-power diagnostic.
//
// j[c, g, lambda] = C_abs(lambda) sum_i P_i B_lambda(T_i) [E_i >= hc/lambda]
// (Sec. 2.3, eq:emission with eq:emission-lambda) is, for one grain g and all
// cells, a dense product (cells x bins) . (bins x wavelengths).  The solver
// stores P~ = P / max P in single precision and the grain table holds
// B~ = C_abs B_lambda(T_i) [..] / s_lambda with s_lambda its column maximum, so
// both operands lie in [0, 1]; the product runs on the matrix cores with FP32
// accumulation and the epilogue restores j = (P~ B~) * maxP * s_lambda.  All
// grains of a batch run as one launch (a workgroup per grain slot and 64-row
// tile, each walking every wavelength tile), and the epilogue also integrates
// the emitted power 4 pi int j dlambda of every pair it completes, so j is
// written once and never read back.
#include <cmath>
#include <vector>

#include "hsd_internal.h"

namespace hsd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4c __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));

// 16-byte loads through global (not flat) addressing
typedef const __attribute__((address_space(1))) u32x4c* GlobalU32x4;
__device__ __forceinline__ u32x4c load16(const unsigned short* p) { return *(GlobalU32x4)(p); }

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int APAD = 1, BPAD = 4;

// The workgroup's slot: the last slot whose first workgroup is <= b (the
// same on every lane).
__device__ __forceinline__ int find_slot(const ContractSlot* sl, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sl[mid].tile0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// The eight rows a lane's accumulators belong to (each wave a 32 x 32
// quarter of the 64 x 64 tile as 2 x 2 blocks of 16 x 16; accumulator
// register i of lane l lies in row 4 (l / 16) + i of its block): their j rows
// (null beyond the slot's rows), their max P, and their pair index.
struct RowInfo {
    float* jrow[2][4];
    float ps[2][4];
    long long pair[2][4];
};

__device__ __forceinline__ RowInfo row_info(const ContractLaunch& a, const ContractSlot& sl, int row0, int wr,
                                            int lane) {
    RowInfo ri;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + wr + bi * 16 + 4 * (lane >> 4) + i;
            ri.jrow[bi][i] = nullptr;
            ri.ps[bi][i] = 0.f;
            ri.pair[bi][i] = -1;
            if (row < sl.rows) {
                const long long cell = sl.rowmap_off >= 0 ? a.rowmap[sl.rowmap_off + row] : row;
                const long long pair = cell * a.n_gslots + sl.gslot;
                ri.pair[bi][i] = pair;
                ri.ps[bi][i] = a.pscale[pair];
                ri.jrow[bi][i] = a.j + pair * a.L;
            }
        }
    }
    return ri;
}

// Epilogue of one 64 x 64 tile: j = acc * maxP * s_lambda, and the tile's
// share of each row's emitted power added to em in FP64 (columns in order).
__device__ __forceinline__ void tile_epilogue(const ContractLaunch& a, const ContractSlot& sl, const RowInfo& ri,
                                              const f32x4 (&acc)[2][2], int col0, int wc, int lane,
                                              double (&em)[2][4]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float* jrow = ri.jrow[bi][i];
            if (!jrow) continue;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int col = col0 + wc + bj * 16 + (lane & 15);
                if (col < a.L) {
                    const float v = acc[bi][bj][i] * ri.ps[bi][i] * sl.bscale[col];
                    jrow[col] = v;
                    em[bi][i] = fma(a.wtrap[col], static_cast<double>(v), em[bi][i]);
                }
            }
        }
    }
}

// After the last tile: each row's emitted power summed over the 16 lanes that
// hold its columns (a fixed tree), then over the two waves that share its
// rows (through LDS), written to diag entry 1.
__device__ __forceinline__ void finish_emitted(const ContractLaunch& a, const RowInfo& ri, double (&em)[2][4],
                                               int wave, int lane, double (*red)[32]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) em[bi][i] += __shfl_xor(em[bi][i], m, 16);
    if ((lane & 15) == 0 && (wave & 1)) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave >> 1][bi * 16 + 4 * (lane >> 4) + i] = em[bi][i];
    }
    __syncthreads();
    if ((lane & 15) == 0 && !(wave & 1) && a.diag) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (ri.pair[bi][i] >= 0)
                    a.diag[ri.pair[bi][i] * 4 + 1] =
                        static_cast<float>(em[bi][i] + red[wave >> 1][bi * 16 + 4 * (lane >> 4) + i]);
    }
}

// FP32 products (v_mfma_f32_16x16x4_f32; lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]).  One 256-thread workgroup per (slot, 64-row tile)
// walks every 64-wavelength tile; its P~ rows stay in the L2 of the XCD that
// runs it between tiles.
__global__ void __launch_bounds__(256) k_contract(ContractLaunch a) {
    __shared__ float As[BM][BK + APAD];
    __shared__ float Bs[BK][BN + BPAD];
    __shared__ double red[2][32];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int b = static_cast<int>(blockIdx.x);
    const ContractSlot sl = a.slots[find_slot(a.slots, a.n_slots, b)];
    const int row0 = (b - sl.tile0) * BM;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int ar = tid >> 2, ak = (tid & 3) * 4;      // A tile loader: row, k offset
    const int bk = tid >> 4, bc = (tid & 15) * 4;     // B tile loader: k row, column offset
    const bool arow_ok = (row0 + ar) < sl.rows;
    const float* Arow = a.Pt + sl.pt_off + static_cast<size_t>(row0 + ar) * sl.nb;
    const RowInfo ri = row_info(a, sl, row0, wr, lane);
    double em[2][4] = {};
    for (int col0 = 0; col0 < a.Lp; col0 += BN) {
        f32x4 acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < sl.nb; k0 += BK) {
            float4 av = make_float4(0.f, 0.f, 0.f, 0.f);
            if (arow_ok) av = *reinterpret_cast<const float4*>(Arow + k0 + ak);
            const float4 bv = *reinterpret_cast<const float4*>(sl.Bt + static_cast<size_t>(k0 + bk) * a.Lp + col0 + bc);
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
        tile_epilogue(a, sl, ri, acc, col0, wc, lane, em);
    }
    finish_emitted(a, ri, em, wave, lane, red);
}

// The same product with each operand split into two BF16 terms, x = hi + lo
// (hi = bf16(x), lo = bf16(x - hi)), and hi hi + hi lo + lo hi accumulated in
// FP32 on v_mfma_f32_16x16x32_bf16 (16 times the FP32 matrix-core rate; the
// dropped lo lo term and the split's remainders keep every product within
// 3 2^-16 of exact).  The solver writes P~ already split (each row: nb hi
// values, then nb lo values, in the row's nb floats of space) and the grain's
// table comes split and transposed (Bh, Bl: [Lp][nbp], zero beyond nb), so the
// loop holds no conversions.
//
// A workgroup of W waves (4 or 8, a tuning choice) takes 64 rows of one slot
// and walks the wavelengths in panels of 64 W; each wave owns 64 x 64 of a
// panel as 4 x 4 blocks of 16 x 16.  The P~ rows go through LDS (double
// buffered, one barrier per step of 32 bins), since every wave uses them;
// each wave reads its own columns of the table straight from global memory
// (L2: one grain's table serves every row tile), each block's next step as
// soon as its products of this step have issued; the P~ rows are fetched two
// steps ahead (they come from HBM), and the register budget is held to three
// waves per SIMD (measured: one step ahead at three waves 1.58 ms per batched
// step, two steps ahead at two waves 1.64 ms, two ahead at three 1.52 ms).
// Eight waves cover the whole padded grid of up to 512 wavelengths in one
// panel, so the P~ rows are read once (four waves read them once per panel)
// at the price of one workgroup per CU.  In a step, lane l supplies row
// (column) l % 16 of a block with bins 8 (l / 16) + 0..7 of the step.
constexpr int KS = 32, LKA = KS + 8;        // bins per step; LDS row length of each P~ plane (ushorts)

template <int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3, 3))) k_contract3(ContractLaunch a) {
    constexpr int NT = 64 * W, PW = 64 * W;
    constexpr int NPL = W >= 8 ? 1 : 2;         // P~ planes staged per loader thread
    __shared__ __align__(16) unsigned short As[2][2][BM][LKA];     // [plane][buffer][row][bin]
    __shared__ double emsh[W][BM];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int b = static_cast<int>(blockIdx.x);
    const ContractSlot sl = a.slots[find_slot(a.slots, a.n_slots, b)];
    const int row0 = (b - sl.tile0) * BM;
    const int rl = lane & 15, q = lane >> 4;
    const int kend = (sl.nb + KS - 1) / KS * KS;
    // P~ loader: thread t stages row (t % 256) / 4, bins 8 (t % 4) + 0..7 of a
    // step, of both planes (four waves) or of plane t / 256 (eight waves).
    // Rows past the slot's last, and bins past nb, load an in-range chunk and
    // zero it (nb is a multiple of 16, so a chunk of 8 is wholly inside or outside).
    const int lt = tid & 255, pl0 = NPL == 1 ? (tid >> 8) : 0;
    const int lr = lt >> 2, lk = (lt & 3) * 8;
    const bool arow_ok = (row0 + lr) < sl.rows;
    const unsigned short* Arow = reinterpret_cast<const unsigned short*>(
        a.Pt + sl.pt_off + static_cast<size_t>(min(row0 + lr, sl.rows - 1)) * sl.nb);
    auto fetch_a = [&](int k0, u32x4c (&v)[NPL]) {
        const bool ok = arow_ok && k0 + lk < sl.nb;
        const int k = ok ? k0 + lk : 0;
        const u32x4c z = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            v[p] = load16(Arow + (pl0 + p) * sl.nb + k);
            v[p] = ok ? v[p] : z;
        }
    };
    auto stage_a = [&](int buf, const u32x4c (&v)[NPL]) {
#pragma unroll
        for (int p = 0; p < NPL; ++p) *reinterpret_cast<u32x4c*>(&As[pl0 + p][buf][lr][lk]) = v[p];
    };
    for (int r = tid; r < W * BM; r += NT) emsh[r / BM][r % BM] = 0.0;
    for (int p0 = 0; p0 < a.Lp; p0 += PW) {
        const int wc = p0 + wave * 64;           // the wave's first column
        const bool wact = wc < a.Lp;             // wave-uniform
        // the wave's table columns: column wc + 16 cb + rl, bins from 8 q
        const size_t bo = static_cast<size_t>(min(wc, a.Lp - 64) + rl) * sl.nbp + 8 * q;
        auto fetch_b = [&](int k0, int cb, u32x4c& h, u32x4c& l) {
            h = load16(sl.Bh + bo + static_cast<size_t>(16 * cb) * sl.nbp + k0);
            l = load16(sl.Bl + bo + static_cast<size_t>(16 * cb) * sl.nbp + k0);
        };
        f32x4 acc[4][4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[bi][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        u32x4c av[NPL], an[NPL], bh[4], bl[4];
        fetch_a(0, av);
        fetch_a(min(KS, kend - KS), an);         // the next step's rows, two steps ahead from here on
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) fetch_b(0, cb, bh[cb], bl[cb]);
        __syncthreads();                         // the previous panel's readers are done with buffer 0
        stage_a(0, av);
        __syncthreads();
        // Straight-line steps: a wave past the last column computes on an
        // in-range column and writes nothing; the last step fetches its own
        // operands again instead of the (absent) next ones.
        for (int k0 = 0, cur = 0; k0 < kend; k0 += KS, cur ^= 1) {
            const int kn = min(k0 + KS, kend - KS);
            fetch_a(min(k0 + 2 * KS, kend - KS), av);
            bf16x8c fh[4], fl[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                fh[bi] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&As[0][cur][16 * bi + rl][8 * q]));
                fl[bi] = __builtin_bit_cast(bf16x8c, *reinterpret_cast<const u32x4c*>(&As[1][cur][16 * bi + rl][8 * q]));
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const bf16x8c gh = __builtin_bit_cast(bf16x8c, bh[cb]), gl = __builtin_bit_cast(bf16x8c, bl[cb]);
#pragma unroll
                for (int bi = 0; bi < 4; ++bi) {
                    acc[bi][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[bi], gh, acc[bi][cb], 0, 0, 0);
                    acc[bi][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[bi], gl, acc[bi][cb], 0, 0, 0);
                    acc[bi][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[bi], gh, acc[bi][cb], 0, 0, 0);
                }
                fetch_b(kn, cb, bh[cb], bl[cb]);     // in flight during the other blocks' products
            }
            // buffer cur ^ 1 was last read before the previous step's barrier
            stage_a(cur ^ 1, an);
#pragma unroll
            for (int p = 0; p < NPL; ++p) an[p] = av[p];
            __syncthreads();
        }
        if (!wact) continue;
        // epilogue: j = acc * maxP * s_lambda; each row's share of the emitted
        // power over the wave's 64 columns (lanes of one quarter hold one
        // row's columns: a fixed tree over them), added to the row's running
        // sum for this wave
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rt = 16 * bi + 4 * q + i;          // row in the tile
                const int row = row0 + rt;
                double em = 0.0;
                if (row < sl.rows) {
                    const long long cell = sl.rowmap_off >= 0 ? a.rowmap[sl.rowmap_off + row] : row;
                    const long long pair = cell * a.n_gslots + sl.gslot;
                    const float ps = a.pscale[pair];
                    float* jrow = a.j + pair * a.L;
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        const int col = wc + 16 * cb + rl;
                        if (col < a.L) {
                            const float v = acc[bi][cb][i] * ps * sl.bscale[col];
                            jrow[col] = v;
                            em = fma(a.wtrap[col], static_cast<double>(v), em);
                        }
                    }
                }
#pragma unroll
                for (int m = 1; m < 16; m <<= 1) em += __shfl_xor(em, m, 16);
                if (rl == 0) emsh[wave][rt] += em;
            }
        }
    }
    __syncthreads();
    if (tid < BM && a.diag && row0 + tid < sl.rows) {
        const int row = row0 + tid;
        const long long cell = sl.rowmap_off >= 0 ? a.rowmap[sl.rowmap_off + row] : row;
        const long long pair = cell * a.n_gslots + sl.gslot;
        // the waves' sums in a fixed pairwise order
        double e[W];
#pragma unroll
        for (int w = 0; w < W; ++w) e[w] = emsh[w][tid];
#pragma unroll
        for (int h = 1; h < W; h <<= 1)
#pragma unroll
            for (int w = 0; w + h < W; w += 2 * h) e[w] += e[w + h];
        a.diag[pair * 4 + 1] = static_cast<float>(e[0]);
    }
}

// Size-distribution convolution (Sec. 2.3, eq:convolution on the size grid):
// out[c][l] = (lambda_l if lw) * sum_g w_g j[c][g][l], FP64 sums; one thread
// per (cell, wavelength), consecutive threads on consecutive wavelengths.
// flags: bit 0 weights by lambda, bit 1 divides by 1 eV in erg (the paper's units).
__global__ void __launch_bounds__(256) k_sizedist(const float* j, const double* w, const double* lam, int n_cells,
                                                  int G, int L, int flags, double* out) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= static_cast<long long>(n_cells) * L) return;
    const long long c = i / L;
    const int l = static_cast<int>(i - c * L);
    const float* jc = j + c * G * L + l;
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc = fma(w[g], static_cast<double>(jc[static_cast<long long>(g) * L]), acc);
    if (flags & 1) acc *= lam[l];
    out[i] = (flags & 2) ? acc / 1.602176634e-12 : acc;
}

}  // namespace

int contract_blocks(std::vector<ContractSlot>& slots) {
    int t = 0;
    for (ContractSlot& s : slots) {
        s.tile0 = t;
        t += (s.rows + BM - 1) / BM;
    }
    return t;
}

hipError_t launch_contract(const ContractLaunch& a, hipStream_t s) {
    if (a.n_blocks <= 0 || a.n_slots <= 0) return hipSuccess;
    if (a.Lp % BN != 0) return hipErrorInvalidValue;
    if (a.mode == 1 && a.waves == 8) hipLaunchKernelGGL(k_contract3<8>, dim3(a.n_blocks), dim3(512), 0, s, a);
    else if (a.mode == 1) hipLaunchKernelGGL(k_contract3<4>, dim3(a.n_blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_contract, dim3(a.n_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sizedist(const float* j, const double* w, const double* lam, int n_cells, int G, int L, int flags,
                           double* out, hipStream_t s) {
    const long long n = static_cast<long long>(n_cells) * L;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sizedist, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, j, w, lam, n_cells, G,
                       L, flags, out);
    return hipGetLastError();
}

}  // namespace hsd
