// The fused per-pair solve: heating rates -> cumulative sums -> X recursion ->
// normalised P, for a batch of (cell, grain) pairs.
//
// Layout.  A pair is served by a segment of P consecutive lanes of one
// wavefront (P = 8, 16, 32 or 64, so a wave serves 64/P pairs of the same grain
// and different cells).  Lane q of the segment owns the enthalpy rows
// k = r * P + q, r = 0..R-1, and keeps for each of them, in registers, the
// inflow G(k) = sum_{j<f} A_kj X_j from the columns already processed; once the
// recursion passes row k the same register holds X_k.
//
// Recursion.  With B_fj = sum_{k>=f} A_kj (eq:bmatrix) the flux that feeds bin
// f is sum_{j<f} B_fj X_j = sum_{k>=f} G(k), so step f of eq:xf is
//     X_f = [ sum_{k>=f} G(k) ] / T_(f-1)f,   then   G(k) += A_kf X_f  for k > f.
// This is the B-matrix recursion with its double sum taken column by column
// instead of row by row: every term is the same non-negative product A_kj X_j,
// nothing is ever subtracted (the direct solve's cancellation that the paper's
// Sec. 2.1 warns about cannot occur), and B is never stored.  The suffix sum
// over k is a segmented wavefront reduction in FP64 (DPP within rows of 16
// lanes, lane-swap instructions across rows).
//
// Rates.  Column f's rates A_kf are produced in the update itself: on
// log-uniform grids the transition's wavelength-grid coordinate is
// a_f - b_(k-f) (see hsd_index.h); the log-log interpolation of
// Omega = u_lambda C_abs (eq:interpolation) and the factor lambda^3 dE_k / (h^2 c)
// of eq:heating give A_kf = 2^(tab[jlo] + w (tab[jlo+1] - tab[jlo])) 2^gamma_k
// with tab_j = log2(u_j C_abs_j) + 3 j dlog2(lambda) (per pair, in LDS) and
// gamma_k = log2(dE_k) + 3 log2(lambda_0) - log2(h^2 c).  The upper bin's width
// dE_k grows by r per bin, so 2^gamma_k = c0 r^k depends on the row alone and
// stays out of the per-rate arithmetic: the register of a row above the
// diagonal holds H(k) = G(k) / (c0 r^k), updated by H(k) += 2^(...) X_f, and the
// lane's share of the suffix sum, sum over its slots s of c0 r^(s P + q - s0) H,
// is evaluated by Horner's rule in r^-P from the lowest slot up and scaled once
// by the lane's factor c0 r^((R-1) P + q - s0).  The exponent and exp2 are
// single precision; the product with X_f and every sum are double precision.
// Row slots are processed in groups of KG (2 or 4, chosen per bin class by the
// autotuner) with straight-line bodies, so the LDS reads of a group overlap; a
// group wholly outside the column's grid-resident rows kb..ke skips its rates.
//
// Continuous (intrabin) heating of row f+1 from column f adds
// X_f Cum(jstar_f) / (E_(f+1) - E_f), Cum_j being the absorbed power of photons at
// wavelengths >= lambda_j; each lane keeps the value for its own rows.
//
// Rescaling.  When a new X_f exceeds 2^500 the pair's whole state (X_0..X_f and
// every pending G) is multiplied by 2^-500, exactly (the appendix on precision
// control rescales by 1e-30 above 1e30 in single precision).
#include <atomic>
#include <cmath>
#include <utility>

#include "hsd_index.h"
#include "hsd_internal.h"

namespace hsd {
namespace {

constexpr double kBig = 0x1p500;
constexpr double kShrink = 0x1p-500;
constexpr float kNoField = -1.0e30f;   // log2 table entry of a non-positive Omega
// The pair's log2 table is shifted to a largest entry of kBias (and c0 down by
// 2^-kBias), so single-precision exp2 keeps that much headroom below its
// underflow for the rates of the faint parts of the field.
constexpr float kBias = 64.0f;

// v from another lane of the same 16-lane row (a full permutation, so every
// lane has a source).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Column parameters are read with wave-uniform addresses from memory the
// kernel never writes; the constant address space lets them come in through
// scalar loads into SGPRs.  Each step loads its own column's: a copy carried
// over from the step before (a prefetch) is kept in VGPRs by the compiler and
// costs seven moves per step, more than the load's latency, which the other
// waves of the SIMD cover.
typedef const __attribute__((address_space(4))) ColPar* ConstColPar;

__device__ __forceinline__ ColPar load_colpar(const ColPar* p, int i) {
    ConstColPar c = (ConstColPar)p + i;
    ColPar v;
    v.invcool = c->invcool;
    v.ia = c->ia;
    v.fa = c->fa;
    v.kb = c->kb;
    v.ke = c->ke;
    v.jstar = c->jstar;
    v.invgap = c->invgap;
    return v;
}

// Two values of v, one from each 16-lane row of a pair of rows (ROW16) or
// from each 32-lane half of the wave; their combination is the same on every
// lane of the 32-lane (64-lane) group.
template <bool ROW16>
__device__ __forceinline__ void swap_halves(double v, double& a, double& b) {
    const unsigned lo = static_cast<unsigned>(__double2loint(v));
    const unsigned hi = static_cast<unsigned>(__double2hiint(v));
    if constexpr (ROW16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a = __hiloint2double(static_cast<int>(h[0]), static_cast<int>(l[0]));
        b = __hiloint2double(static_cast<int>(h[1]), static_cast<int>(l[1]));
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a = __hiloint2double(static_cast<int>(h[0]), static_cast<int>(l[0]));
        b = __hiloint2double(static_cast<int>(h[1]), static_cast<int>(l[1]));
    }
}

// Sum over the P lanes of each segment; every lane of a segment gets the same
// bits (each combining step is symmetric).
template <int P>
__device__ __forceinline__ double seg_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    if constexpr (P >= 16) v += dpp_f64<0x140>(v);   // row_mirror
    if constexpr (P >= 32) {
        double a, b;
        swap_halves<true>(v, a, b);
        v = a + b;
    }
    if constexpr (P >= 64) {
        double a, b;
        swap_halves<false>(v, a, b);
        v = a + b;
    }
    return v;
}

template <int P>
__device__ __forceinline__ double seg_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    if constexpr (P >= 16) v = fmax(v, dpp_f64<0x140>(v));
    if constexpr (P >= 32) {
        double a, b;
        swap_halves<true>(v, a, b);
        v = fmax(a, b);
    }
    if constexpr (P >= 64) {
        double a, b;
        swap_halves<false>(v, a, b);
        v = fmax(a, b);
    }
    return v;
}

template <int P>
__device__ __forceinline__ float seg_maxf(float v) {
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ double clean_field(double u, bool& bad) {
    if (!(u >= 0.0) || !(u < INFINITY)) {
        bad = true;
        return 0.0;
    }
    return u;
}

// Integer clamp in one instruction (the compiler keeps max + min when the
// bounds are not constants).
__device__ __forceinline__ int med3_i32(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

template <int R>
struct Rec {
    double G[R];       // H(k) = G(k) / (c0 r^k) of the lane's rows, then X_k once row k is passed
    float intra[R];    // continuous-heating rate into each row from the row below (register variant)
    double part;       // this lane's share of sum_{k >= f} G(k) for the next step
    double lf;         // c0 r^((R-1) P + q - s0): the factor of the lane's row in the top slot
    double srep;       // LDS-table variant: the lane's finished rows' sum of X_k Cum(jrep_k) / total
    int nres;          // rescales so far
};

struct StepEnv {
    int q, nb, Lm1;
    int s0;            // row k sits at position k + s0 (s0 = R P - nb): the tail slot holds the top bin
    double irP;        // r^-P: the factor between a lane's consecutive slots, downwards (1 for given rates)
    double total;      // the pair's absorbed power (Cum_0)
    const ColPar* colpar;
    const int* jrep;   // per row: first grid index of the photons it can absorb within the grid (L: none)
    const DPar* dpar;  // LDS
    const float* tab;  // LDS, this pair's log2 table
    int tlo, thi;      // LDS byte addresses of table entries -1 and L
    const float* cum;  // LDS, this pair's Cum / total (LDS-table variant)
    const double* Ap;  // given-rates hook: this pair's rate matrix
    const double* cp;  // given-rates hook: this pair's cooling rates
};

// Per-step values the slot groups need.
struct StepState {
    int pf, l, kb, ke;     // column position pf = f + s0, lane of the diagonal, grid-resident rows (positions)
    double Xg;         // X_f
    int cb;            // LDS byte address of table entry ia1 of the column
    float fa;
};

// One group of KG row slots starting at slot R0 (>= RO) for step f: rates of
// the column into the group's rows, the FP64 update H += 2^(...) X, and the
// group's Horner steps of the next suffix sum (acc = acc r^-P + H, lowest slot
// first).  Straight-line, so the group's LDS reads are in flight together;
// skipped by a wave-uniform test when none of its rows is grid-resident for
// this column.
template <int P, int R, int KG, bool GIVEN, int RO, int R0>
__device__ __forceinline__ void slot_group(Rec<R>& st, const StepEnv& e, const StepState& ss, double& acc) {
    constexpr int NS = (R - R0) < KG ? (R - R0) : KG;
    const int q = e.q, nb = e.nb;
    const int lo_pos = R0 * P, hi_pos = (R0 + NS) * P - 1;
    if (hi_pos >= ss.kb && lo_pos <= ss.ke) {
        double A[NS];
        if constexpr (GIVEN) {
            const int f = ss.pf - e.s0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int pos = (R0 + s) * P + q;
                const int k = min(max(pos - e.s0, 0), nb - 1);
                const double v = e.Ap[static_cast<size_t>(k) * nb + f];
                A[s] = (pos >= ss.kb && pos <= ss.ke) ? v : 0.0;
            }
        } else {
            DPar dp[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int d = (R0 + s) * P + q - ss.pf;
                dp[s] = e.dpar[R0 + s == RO ? max(d, 0) : d];
            }
            // the grid interval of transition_index (hsd_index.h) as an LDS byte
            // address: cb + 4 nib + 4 fl = address of entry jlo, with the column's
            // and the distance's parts pre-scaled by 4 (cb, dpar.nib), clamped to
            // entries -1 .. L
            float t0[NS], t1[NS], w[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float fd = ss.fa - dp[s].fb;
                const int fl = static_cast<int>(fd);
                w[s] = __builtin_amdgcn_fractf(fd);
                const int off = med3_i32(ss.cb + dp[s].nib + (fl << 2), e.tlo, e.thi);
                typedef const __attribute__((address_space(3))) float* LdsF;
                const LdsF p = (LdsF)static_cast<size_t>(static_cast<unsigned>(off));
                t0[s] = p[0];
                t1[s] = p[1];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s)
                A[s] = static_cast<double>(__builtin_amdgcn_exp2f(fmaf(w[s], t1[s] - t0[s], t0[s])));
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) st.G[R0 + s] = fma(A[s], ss.Xg, st.G[R0 + s]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (R0 + s == RO) acc = (q > ss.l) ? st.G[R0 + s] : 0.0;    // the first term: acc is 0
        else acc = fma(acc, e.irP, st.G[R0 + s]);
    }
}

template <int P, int R, int KG, bool GIVEN, int RO, int... G>
__device__ __forceinline__ void all_groups(Rec<R>& st, const StepEnv& e, const StepState& ss, double& acc,
                                           std::integer_sequence<int, G...>) {
    (slot_group<P, R, KG, GIVEN, RO, RO + G * KG>(st, e, ss, acc), ...);
}

// All steps f = RO*P .. RO*P + P - 1 (the columns whose rows sit in slot RO).
// Slots below RO are finished and untouched; slot RO holds the diagonal.
//
// The rate of column f into row k = f + d is
//     A = exp2(tab[jlo] + w (tab[jlo+1] - tab[jlo])) * c0 r^k;
// the register of row k accumulates the exp2 terms times X_f (H units), and
// the row factor enters once per lane and column through the Horner sum.
// Rates need no per-lane masks: the log2 table carries a non-field sentinel
// one entry below lambda_0 and two above lambda_(L-1), the interval index is
// clamped into [-1, L], and distance 0 (rows at or below the diagonal) maps far
// below the grid, so every transition off the wavelength grid evaluates to
// exp2(-1e30-ish) = 0 exactly.  Positions below row 0 (the head of slot 0 when
// the bin count is not a multiple of P) hold no row: they are never summed or
// written.  Slots are handled KG at a time as straight-line code, so the LDS
// reads of a group are in flight together; a group wholly outside the
// column's grid-resident rows kb..ke is skipped by a wave-uniform test.
template <int P, int R, int KG, bool GIVEN, bool LDSCUM, int RO>
__device__ __forceinline__ void column_block(Rec<R>& st, const StepEnv& e) {
    const int q = e.q, nb = e.nb, s0 = e.s0;
    if (RO * P + P - 1 < s0) return;          // only positions below row 0
    // LDS-table variant: the representable-power share of the lane's row in this
    // slot, added once the block's steps have made it final (its table index is
    // fetched now, so the load's latency passes under the steps)
    const int kro = max(RO * P + q - s0, 0);
    int jrk = 0;
    if constexpr (LDSCUM && !GIVEN) jrk = e.jrep[kro];
#pragma unroll 1
    for (int l = 0; l < P; ++l) {
        const int pf = RO * P + l;
        const int f = pf - s0;
        if (f < 0) continue;
        ColPar cc{};
        if constexpr (!GIVEN) {
            cc = load_colpar(e.colpar, f);
        }
        double Xf = 1.0;
        if (f > 0) {
            const double S = seg_sum<P>(st.part);
            if constexpr (GIVEN) Xf = S / e.cp[f];
            else Xf = S * cc.invcool;
        }
        if (Xf > kBig) {
            Xf *= kShrink;
#pragma unroll
            for (int r = 0; r < R; ++r) st.G[r] *= kShrink;
            if constexpr (LDSCUM && !GIVEN) st.srep *= kShrink;
            ++st.nres;
        }
        if (q == l) st.G[RO] = Xf;

        int kb, ke;
        if constexpr (GIVEN) {
            kb = pf + 1;
            ke = nb - 1 + s0;
        } else {
            kb = max(cc.kb + s0, pf + 1);
            ke = cc.ke + s0;
        }
        double acc = 0.0;
        StepState ss{pf, l, kb, ke, Xf, 4 * cc.ia + e.tlo + 4, cc.fa};
        all_groups<P, R, KG, GIVEN, RO>(st, e, ss, acc, std::make_integer_sequence<int, (R - RO + KG - 1) / KG>{});
        double part = acc * st.lf;
        if constexpr (!GIVEN) {
            // continuous heating of row f+1 (its owner: lane l+1 of slot RO, or lane 0 of slot RO+1).
            // Row f+1 enters only the next step's suffix sum (then it is the diagonal, masked
            // out of the sums and overwritten by X_(f+1)), so the term counts through part
            // alone; the write into the row's register is never read, but without it the
            // compiler keeps far more registers live across the column loop.
            double cin = 0.0;
            if constexpr (LDSCUM) {
                cin = (cc.jstar <= e.Lm1) ? static_cast<double>(e.cum[cc.jstar]) * e.total *
                                                static_cast<double>(cc.invgap)
                                          : 0.0;
            }
            if (l + 1 < P) {
                if (q == l + 1 && f + 1 < nb) {
                    double c;
                    if constexpr (LDSCUM) c = cin;
                    else c = static_cast<double>(st.intra[RO]);
                    const double inc = c * Xf;
                    st.G[RO] += inc;
                    part += inc;
                }
            } else if constexpr (RO + 1 < R) {
                if (q == 0 && f + 1 < nb) {
                    double c;
                    if constexpr (LDSCUM) c = cin;
                    else c = static_cast<double>(st.intra[RO + 1]);
                    const double inc = c * Xf;
                    st.G[RO + 1] += inc;
                    part += inc;
                }
            }
        }
        st.part = part;
    }
    if constexpr (LDSCUM && !GIVEN) {
        // X of the row is final up to the exact rescales, which scale the sum too
        const float cv = e.cum[min(jrk, e.Lm1)];
        if (RO * P + q >= s0 && jrk <= e.Lm1) st.srep = fma(st.G[RO], static_cast<double>(cv), st.srep);
    }
}

template <int P, int R, int KG, bool GIVEN, bool LDSCUM, int... RO>
__device__ __forceinline__ void all_columns(Rec<R>& st, const StepEnv& e, std::integer_sequence<int, RO...>) {
    (column_block<P, R, KG, GIVEN, LDSCUM, RO>(st, e), ...);
}

struct KArgs {
    const double* u;
    const double* lam;
    int L;
    int tabstride;             // floats per pair in LDS (log2 table with sentinels, then Cum), padded
    float dlam2;               // log2(lambda_(j+1) / lambda_j)
    int n_cells;
    int n_gslots;
    const GrainView* views;
    const long long* offs;
    float* Pt;
    int psplit;                // P~ rows as two BF16 planes (hi, then lo) instead of FP32
    float* pscale;
    float* diag;
    double* P64;
    unsigned* errword;
    const int2* items;
    int n_items;               // work items (physical) or blocks of pairs (given rates)
    unsigned* queue;           // persistent launch: next-item counter (zero at launch), else null
    const int* cellmap;        // optional: cells of each slot's pairs, slot s at seg_off[s] .. + seg_cnt[s]
    const int* seg_off;
    const int* seg_cnt;
    // given-rates test hook
    const double* A;
    const double* cool;
    int nb_given;
    int n_pairs;
};

// LDSCUM: the pair's Cum table stays in LDS for the whole solve (the
// continuous-heating and representable-power terms read it), instead of
// being folded into per-row registers; chosen for the large bin counts, where
// registers are scarcer than LDS.
//
// One work item per workgroup (item = block index), or (PERSIST) a grid of
// the workgroups that fit on the device at once in which every workgroup
// takes the next item from an atomic counter until the list is exhausted, so
// the items, ordered longest first, go to whichever workgroup frees up first.
// Every workgroup leaves the loop once the counter has passed the last item.
// (The body stays in the kernel itself: moved into a function that takes the
// kernel arguments by reference, it costs 10-20 more VGPRs.)
//
// Occupancy: the kernel is held to 128 VGPRs, 4 waves per SIMD, where the
// fourth wave hides the LDS and exp2 latencies of the rate groups (the
// ~1024-bin class runs 10% faster than at 3 waves, the ~256-bin class 14%).
// The ordinary-grid kernels fit that budget with no scratch (the epilogue's
// inputs are made opaque after the recursion, below, so the compiler does not
// hoist their address arithmetic above it and park the results in scratch);
// the persistent variants keep a few dozen values in scratch, once per item.
template <int P, int R, int KG, int WAVES, bool GIVEN, bool LDSCUM, bool PERSIST>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(4))) k_solve(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_next;
    int item = blockIdx.x;
    if constexpr (PERSIST) {
        if (threadIdx.x == 0) s_next = static_cast<int>(atomicAdd(a.queue, 1u));
        __syncthreads();
        item = s_next;
    }
    for (;;) {
        if constexpr (PERSIST) {
            if (item >= a.n_items) break;
        }
        constexpr int PPW = 64 / P;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int q = lane & (P - 1);
        const int seg = lane / P;

        int gslot = 0, cell, nb, rowk;   // rowk: the pair's row in its slot's P~ block
        bool live;
        GrainView gv{};
        if constexpr (!GIVEN) {
            const int2 it = a.items[item];
            gslot = it.x;
            rowk = it.y + wave * PPW + seg;
            gv = a.views[gslot];
            nb = gv.nb;
            if (a.cellmap) {
                // a list of cells per slot (the surrogate's fallback pairs)
                live = rowk < a.seg_cnt[gslot];
                cell = live ? a.cellmap[a.seg_off[gslot] + rowk] : 0;
            } else {
                live = rowk < a.n_cells;
                cell = rowk;
            }
        } else {
            cell = (item * WAVES + wave) * PPW + seg;
            rowk = cell;
            nb = a.nb_given;
            live = cell < a.n_pairs;
        }
        const int cellc = live ? cell : 0;

        Rec<R> st;
        float rep[R];      // representable absorbed power from each row's bin, / total (register variant)
        double total = 0.0;
        double cf0 = 1.0;
        bool bad = false;
        DPar* dpar_s = reinterpret_cast<DPar*>(smem);
        float* tab = nullptr;
        float* cum = nullptr;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            st.intra[r] = 0.0f;
            rep[r] = 0.0f;
        }

        if constexpr (!GIVEN) {
            const int L = a.L;
            // log2 table with sentinels: tab[-1], tab[L], tab[L+1] hold kNoField
            float* base = reinterpret_cast<float*>(smem + sizeof(DPar) * R * P) + (wave * PPW + seg) * a.tabstride;
            tab = base + 1;
            cum = LDSCUM ? base + (L + 3) : tab;   // else pass 2 overwrites Cum with the log2 table
            for (int d = threadIdx.x; d < nb; d += 64 * WAVES) {
                DPar v = gv.dpar[d];
                v.nib *= 4;              // table entries are 4 bytes
                dpar_s[d] = v;
            }

            // Pass 1: absorbed-power suffix integrals Cum_j = int_{lambda_j} c u C_abs dlambda
            // (trapezoid), FP64, kept normalised by the total in FP32.  The
            // segment reads P consecutive wavelengths at a time (coalesced), from
            // the top of the grid down; interval j's trapezoid t_j takes rho_(j+1)
            // from the next lane (the last lane: from the block above).  A first
            // sweep sums the t_j for the total; the second adds, per block, the
            // suffix sums across the lanes to the sum of the blocks above.
            const double* uc = a.u + static_cast<size_t>(cellc) * L;
            const int jtop = (L - 1) / P * P;
            auto interval = [&](int j, double& rho_up) {
                const double rho = j < L ? kLight * clean_field(uc[j], bad) * gv.cabs[j] : 0.0;
                double rn = __shfl_down(rho, 1, P);
                if (q == P - 1) rn = rho_up;
                rho_up = __shfl(rho, 0, P);
                return (j + 1 < L) ? 0.5 * (rho + rn) * (a.lam[j + 1] - a.lam[j]) : 0.0;
            };
            double csum = 0.0, rho_up = 0.0;
            for (int j0 = jtop; j0 >= 0; j0 -= P) csum += interval(j0 + q, rho_up);
            total = seg_sum<P>(csum);
            const double inv_total = total > 0.0 ? 1.0 / total : 0.0;
            double above = 0.0;
            rho_up = 0.0;
            for (int j0 = jtop; j0 >= 0; j0 -= P) {
                double sfx = interval(j0 + q, rho_up);
#pragma unroll
                for (int m = 1; m < P; m <<= 1) {
                    const double o = __shfl_down(sfx, m, P);
                    if (q + m < P) sfx += o;
                }
                if (j0 + q < L) cum[j0 + q] = static_cast<float>((above + sfx) * inv_total);
                above += __shfl(sfx, 0, P);
            }
            __syncthreads();
            if constexpr (!LDSCUM) {
                // Continuous heating of row k from column k-1 (Draine & Li intrabin
                // term): absorbed power of photons too soft for the step, per unit step.
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = r * P + q - (R * P - nb);
                    if (k >= 1 && k < nb) {
                        const int js = gv.jstar[k - 1];
                        if (js < L && total > 0.0)
                            st.intra[r] = static_cast<float>(static_cast<double>(cum[js]) * total * gv.invgap[k - 1]);
                    }
                    if (k >= 0 && k < nb) {
                        const int jr = gv.jrep[k];
                        if (jr < L) rep[r] = cum[jr];
                    }
                }
                __syncthreads();
            }
            // Pass 2: tab_j = log2(u_j C_abs_j) + 3 j dlog2(lambda) - off + kBias, off =
            // the pair's largest entry (restored through c0, so the exponent stays small).
            float mx = -INFINITY;
            for (int j = q; j < L; j += P) {
                const double om = clean_field(uc[j], bad) * gv.cabs[j];
                float v = kNoField;
                if (om > 0.0) {
                    int e;
                    const double m = frexp(om, &e);
                    v = static_cast<float>(e) + __builtin_amdgcn_logf(static_cast<float>(m)) + 3.0f * a.dlam2 * j;
                    mx = fmaxf(mx, v);
                }
                tab[j] = v;
            }
            mx = seg_maxf<P>(mx);
            const float off = (mx > -INFINITY) ? mx : 0.0f;
            for (int j = q; j < L; j += P) {
                const float v = tab[j];
                tab[j] = (v > kNoField) ? (v - off) + kBias : kNoField;
            }
            if (q == 0) {
                tab[-1] = kNoField;
                tab[L] = kNoField;
                tab[L + 1] = kNoField;
            }
            cf0 = exp2(gv.gam[0] + static_cast<double>(off) - static_cast<double>(kBias));
            __syncthreads();
        }

        // ---- recursion ----
#pragma unroll
        for (int r = 0; r < R; ++r) st.G[r] = 0.0;
        st.part = 0.0;
        st.srep = 0.0;
        st.nres = 0;
        if constexpr (GIVEN) {
            st.lf = 1.0;
        } else {
            // c0 r^((R-1) P + q - s0), the factor of the lane's row in the top slot
            st.lf = cf0 * exp2(static_cast<double>((R - 1) * P + q - (R * P - nb)) * log2(gv.rbin));
        }
        StepEnv env;
        env.q = q;
        env.nb = nb;
        env.s0 = R * P - nb;
        env.Lm1 = a.L - 1;
        env.irP = GIVEN ? 1.0 : exp2(-static_cast<double>(P) * log2(gv.rbin));
        env.total = total;
        env.colpar = gv.colpar;
        env.jrep = gv.jrep;
        env.dpar = dpar_s;
        env.tab = tab;
        if constexpr (!GIVEN) {
            typedef __attribute__((address_space(3))) float* LdsF;
            env.tlo = static_cast<int>(reinterpret_cast<size_t>((LdsF)tab)) - 4;
            env.thi = env.tlo + 4 * (a.L + 1);
        }
        env.cum = cum;
        if constexpr (GIVEN) {
            env.Ap = a.A + static_cast<size_t>(cellc) * nb * nb;
            env.cp = a.cool + static_cast<size_t>(cellc) * nb;
        }
        all_columns<P, R, KG, GIVEN, LDSCUM>(st, env, std::make_integer_sequence<int, R>{});
        double* G = st.G;
        const int nres = st.nres;
        // The output addresses depend on the lane and the pair's row; made opaque
        // here, they are formed after the recursion instead of being hoisted
        // above it by the compiler (and kept in scratch memory across it).
        int qo = q, rowko = rowk;
        asm volatile("" : "+v"(qo), "+v"(rowko));

        // ---- normalisation (eq:renormalization) and outputs ----
        const int s0 = R * P - nb;
        double sx = 0.0, mxx = 0.0, srep = 0.0;
        if constexpr (LDSCUM && !GIVEN) {
            // positions below row 0 hold 0 (no rate reaches them and no step ends
            // there); the representable power was accumulated block by block
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sx += G[r];
                mxx = fmax(mxx, G[r]);
            }
            srep = seg_sum<P>(st.srep);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = r * P + qo - s0;
                if (k >= 0) {
                    sx += G[r];
                    mxx = fmax(mxx, G[r]);
                    float rv = rep[r];
                    asm volatile("" : "+v"(rv));   // converted here, not before the recursion
                    srep += G[r] * static_cast<double>(rv);
                }
            }
            srep = seg_sum<P>(srep);
        }
        sx = seg_sum<P>(sx);
        mxx = seg_max<P>(mxx);
        bad = seg_maxf<P>(bad ? 1.0f : 0.0f) > 0.0f;
        if (live) {
            if (a.P64) {
                double* prow = a.P64 + static_cast<size_t>(cell) * nb;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = r * P + qo - s0;
                    if (k >= 0) prow[k] = G[r] / sx;
                }
            }
            if constexpr (!GIVEN) {
                if (a.Pt) {
                    float* prow = a.Pt + a.offs[gslot] + static_cast<size_t>(rowko) * nb;
                    const double inv = 1.0 / mxx;
                    if (a.psplit) {
                        // the row's nb floats of space hold P~ = hi + lo as BF16
                        // planes, hi = bf16(P~) at [0, nb), lo = bf16(P~ - hi) at [nb, 2 nb)
                        unsigned short* hrow = reinterpret_cast<unsigned short*>(prow);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int k = r * P + qo - s0;
                            if (k >= 0) {
                                const float v = static_cast<float>(G[r] * inv);
                                const __bf16 h = static_cast<__bf16>(v);
                                const __bf16 l = static_cast<__bf16>(v - static_cast<float>(h));
                                hrow[k] = __builtin_bit_cast(unsigned short, h);
                                hrow[nb + k] = __builtin_bit_cast(unsigned short, l);
                            }
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int k = r * P + qo - s0;
                            if (k >= 0) prow[k] = static_cast<float>(G[r] * inv);
                        }
                    }
                }
                const size_t pair = static_cast<size_t>(cell) * a.n_gslots + gslot;
                if (q == 0) {
                    if (a.pscale) a.pscale[pair] = static_cast<float>(mxx / sx);
                    // no heating term anywhere leaves X = (1, 0, ..., 0): the sum is exactly 1
                    const unsigned flags = (sx == 1.0 && nres == 0 ? 1u : 0u) | (nres > 0 ? 2u : 0u) | (bad ? 4u : 0u);
                    if (a.diag) {
                        a.diag[pair * 4 + 0] = static_cast<float>(total);
                        a.diag[pair * 4 + 2] = static_cast<float>(total * (srep / sx));
                        a.diag[pair * 4 + 3] = static_cast<float>(flags);
                    }
                    if (bad && a.errword) atomicOr(a.errword, 1u);
                }
            }
        }
        if constexpr (!PERSIST) {
            break;
        } else {
            __syncthreads();     // the item's LDS tables are dead and every thread has read s_next
            if (threadIdx.x == 0) s_next = static_cast<int>(atomicAdd(a.queue, 1u));
            __syncthreads();
            item = s_next;
        }
    }
}

__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Workgroups of one kernel that fit on the device at once (persistent grid).
template <typename K>
int resident_blocks(K kern, int threads, size_t lds) {
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess) return -1;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return (per_cu > 0 ? per_cu : 1) * ncu;
}

template <int P, int R, int KG, int WAVES, bool LDSCUM>
size_t phys_lds(int tabstride) {
    return sizeof(DPar) * R * P + sizeof(float) * static_cast<size_t>(WAVES) * (64 / P) * tabstride;
}

// Cached per kernel and LDS stride (the stride depends on the grid length).
template <int P, int R, int KG, int WAVES, bool LDSCUM>
int phys_cap(int tabstride) {
    static std::atomic<long long> memo{-1};
    const long long m = memo.load(std::memory_order_relaxed);
    if (m >= 0 && static_cast<int>(m >> 32) == tabstride) return static_cast<int>(m & 0xffffffffLL);
    const int cap = resident_blocks(k_solve<P, R, KG, WAVES, false, LDSCUM, true>, 64 * WAVES,
                                    phys_lds<P, R, KG, WAVES, LDSCUM>(tabstride));
    if (cap > 0) memo.store((static_cast<long long>(tabstride) << 32) | cap, std::memory_order_relaxed);
    return cap;
}

template <int P, int R, int KG, int WAVES, bool LDSCUM>
hipError_t launch_phys_kg(KArgs ka, int n_items, unsigned* queue, hipStream_t s) {
    const size_t lds = phys_lds<P, R, KG, WAVES, LDSCUM>(ka.tabstride);
    ka.n_items = n_items;
    ka.queue = queue;
    int grid = n_items;
    if (queue) {
        const int cap = phys_cap<P, R, KG, WAVES, LDSCUM>(ka.tabstride);
        if (cap <= 0) return hipErrorInvalidValue;
        grid = n_items < cap ? n_items : cap;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, queue, 1);
    }
    if (queue)
        hipLaunchKernelGGL((k_solve<P, R, KG, WAVES, false, LDSCUM, true>), dim3(grid), dim3(64 * WAVES), lds, s, ka);
    else
        hipLaunchKernelGGL((k_solve<P, R, KG, WAVES, false, LDSCUM, false>), dim3(grid), dim3(64 * WAVES), lds, s, ka);
    return hipGetLastError();
}

template <int P, int R, int WAVES, bool LDSCUM>
hipError_t launch_phys(const KArgs& ka, int n_items, int kg, unsigned* queue, hipStream_t s) {
    if (kg == 4) return launch_phys_kg<P, R, 4, WAVES, LDSCUM>(ka, n_items, queue, s);
    return launch_phys_kg<P, R, 2, WAVES, LDSCUM>(ka, n_items, queue, s);
}

template <int P, int R, int WAVES, bool LDSCUM>
int cap_phys(int kg, int tabstride) {
    if (kg == 4) return phys_cap<P, R, 4, WAVES, LDSCUM>(tabstride);
    return phys_cap<P, R, 2, WAVES, LDSCUM>(tabstride);
}

template <int P, int R, int WAVES>
hipError_t launch_given(KArgs ka, int n_pairs, hipStream_t s) {
    const int per_block = WAVES * (64 / P);
    const int blocks = (n_pairs + per_block - 1) / per_block;
    ka.n_items = blocks;
    ka.queue = nullptr;
    hipLaunchKernelGGL((k_solve<P, R, 4, WAVES, true, false, false>), dim3(blocks), dim3(64 * WAVES), 0, s, ka);
    return hipGetLastError();
}

constexpr int kWaves = 4;

}  // namespace

// Bin-count classes: lanes per pair P and row slots per lane R (P R >= bins).
//   <= 128 bins: P 16, R 8, or (alternate layout) P 8, R 16: twice the rows
//           per lane and step, a segmented sum one step shorter, eight pairs
//           per wave (the LDS tables of 32 pairs per workgroup allow two
//           workgroups per CU);
//   <= 256: P 16, R 16;
//   <= 512: P 32, R 16, or (alternate layout) P 16, R 32 with the Cum table
//           kept in LDS: twice the rows per lane and step, so the per-step
//           work (suffix sums, the column's X) is spread over twice the rates;
//   <= 1024: P 32, R 32 with the Cum table kept in LDS, or (alternate) P 64, R 16.
namespace {
int class_lanes(const ClassCfg& cfg, int cls) {
    if (cls == 0) return cfg.wide ? 64 : 32;
    if (cls == 1) return cfg.wide ? 16 : 32;
    if (cls == 3) return cfg.wide ? 8 : 16;
    return 16;
}
bool class_ldscum(const ClassCfg& cfg, int cls) { return (cls == 0 && !cfg.wide) || (cls == 1 && cfg.wide); }
}  // namespace

int solve_cells_per_item(const ClassCfg& cfg, int cls) { return kWaves * (64 / class_lanes(cfg, cls)); }

// LDS floats per pair: the log2 table with its sentinels, plus the Cum table
// when it stays in LDS.
int tab_stride(const Ctx& c, int cls) {
    if (!class_ldscum(c.cfg[cls], cls)) return (c.L + 3 + 3) & ~3;
    return (2 * c.L + 3 + 3) & ~3;
}

int solve_capacity(const Ctx& c, int cls) {
    if (cls < 0 || cls >= kClasses) return -1;
    const ClassCfg& cfg = c.cfg[cls];
    const int ts = tab_stride(c, cls);
    switch (cls) {
        case 3:
            if (cfg.wide) return cap_phys<8, 16, kWaves, false>(cfg.kg, ts);
            return cap_phys<16, 8, kWaves, false>(cfg.kg, ts);
        case 2: return cap_phys<16, 16, kWaves, false>(cfg.kg, ts);
        case 1:
            if (cfg.wide) return cap_phys<16, 32, kWaves, true>(cfg.kg, ts);
            return cap_phys<32, 16, kWaves, false>(cfg.kg, ts);
        default:
            if (cfg.wide) return cap_phys<64, 16, kWaves, false>(cfg.kg, ts);
            return cap_phys<32, 32, kWaves, true>(cfg.kg, ts);
    }
}

hipError_t launch_solve(const Ctx& c, const SolveLaunch& sl, int cls, const int2* items_dev, int n_items,
                        unsigned* queue, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (cls < 0 || cls >= kClasses) return hipErrorInvalidValue;
    const ClassCfg& cfg = c.cfg[cls];
    KArgs ka{};
    ka.u = sl.u;
    ka.lam = c.lam;
    ka.L = c.L;
    ka.dlam2 = static_cast<float>(c.dlnlam / std::log(2.0));
    ka.n_cells = sl.n_cells;
    ka.n_gslots = sl.n_gslots;
    ka.views = sl.views;
    ka.offs = sl.offs;
    ka.Pt = sl.Pt;
    ka.psplit = c.contract == 1;
    ka.pscale = sl.pscale;
    ka.diag = sl.diag;
    ka.P64 = sl.P64;
    ka.errword = sl.errword;
    ka.items = items_dev;
    ka.cellmap = sl.cellmap;
    ka.seg_off = sl.seg_off;
    ka.seg_cnt = sl.seg_cnt;
    unsigned* q = cfg.persistent ? queue : nullptr;
    if (cfg.persistent && !queue) return hipErrorInvalidValue;
    ka.tabstride = tab_stride(c, cls);
    switch (cls) {
        case 3:
            if (cfg.wide) return launch_phys<8, 16, kWaves, false>(ka, n_items, cfg.kg, q, s);
            return launch_phys<16, 8, kWaves, false>(ka, n_items, cfg.kg, q, s);
        case 2: return launch_phys<16, 16, kWaves, false>(ka, n_items, cfg.kg, q, s);
        case 1:
            if (cfg.wide) return launch_phys<16, 32, kWaves, true>(ka, n_items, cfg.kg, q, s);
            return launch_phys<32, 16, kWaves, false>(ka, n_items, cfg.kg, q, s);
        default:
            if (cfg.wide) return launch_phys<64, 16, kWaves, false>(ka, n_items, cfg.kg, q, s);
            return launch_phys<32, 32, kWaves, true>(ka, n_items, cfg.kg, q, s);
    }
}

hipError_t launch_from_rates(const Ctx& c, int nb, int n_pairs, const double* A, const double* cool, double* P,
                             hipStream_t s) {
    KArgs ka{};
    ka.A = A;
    ka.cool = cool;
    ka.nb_given = nb;
    ka.n_pairs = n_pairs;
    ka.P64 = P;
    ka.L = 1;
    if (nb <= 128) return launch_given<16, 8, kWaves>(ka, n_pairs, s);
    if (nb <= 256) return launch_given<16, 16, kWaves>(ka, n_pairs, s);
    if (nb <= 512) return launch_given<32, 16, kWaves>(ka, n_pairs, s);
    return launch_given<64, 16, kWaves>(ka, n_pairs, s);
}

}  // namespace hsd
