// The fused per-pair solve: heating rates -> cumulative sums -> X recursion ->
// normalised P, for a batch of (cell, grain) pairs.
//
// Layout.  A pair is served by a segment of P consecutive lanes of one
// wavefront (P = 16, 32 or 64, so a wave serves 64/P pairs of the same grain
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
// over k is a segmented wavefront reduction in FP64.
//
// Rates.  Column f's rates A_kf are produced in the update itself: on
// log-uniform grids the transition's wavelength-grid coordinate is
// a_f - b_(k-f) (see hsd_index.h); the log-log interpolation of
// Omega = u_lambda C_abs (eq:interpolation) and the factor lambda^3 dE_k / (h^2 c)
// of eq:heating fold into one exp2 of
//     tab[jlo] + w (tab[jlo+1] - tab[jlo]) + gamma_k
// with tab_j = log2(u_j C_abs_j) + 3 j dlog2(lambda) (per pair, in LDS) and
// gamma_k = log2(dE_k) + 3 log2(lambda_0) - log2(h^2 c) (per row, in registers).
// The exponent and exp2 are single precision; the product with X_f and every
// sum are double precision.
//
// Rescaling.  When a new X_f exceeds 2^500 the pair's whole state (X_0..X_f and
// every pending G) is multiplied by 2^-500, exactly (the appendix on precision
// control rescales by 1e-30 above 1e30 in single precision).
#include <cmath>

#include "hsd_index.h"
#include "hsd_internal.h"

namespace hsd {
namespace {

constexpr double kBig = 0x1p500;
constexpr double kShrink = 0x1p-500;
constexpr float kNoField = -1.0e30f;   // log2 table entry of a non-positive Omega

template <int P>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int P>
__device__ __forceinline__ double seg_max(double v) {
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

template <int P>
__device__ __forceinline__ float seg_maxf(float v) {
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

// Sum of v over the lanes q' > q of the segment (no subtraction).
template <int P>
__device__ __forceinline__ double seg_suffix_exclusive(double v, int q) {
    double s = __shfl_down(v, 1, P);
    if (q + 1 >= P) s = 0.0;
#pragma unroll
    for (int m = 1; m < P; m <<= 1) {
        const double o = __shfl_down(s, m, P);
        if (q + m < P) s += o;
    }
    return s;
}

__device__ __forceinline__ double clean_field(double u, bool& bad) {
    if (!(u >= 0.0) || !(u < INFINITY)) {
        bad = true;
        return 0.0;
    }
    return u;
}

struct KArgs {
    const double* u;
    const double* lam;
    int L;
    int tabstride;
    float dlam2;               // log2(lambda_(j+1) / lambda_j)
    int n_cells;
    int n_gslots;
    const GrainView* views;
    const long long* offs;
    float* Pt;
    float* pscale;
    float* diag;
    double* P64;
    unsigned* errword;
    const int2* items;
    // given-rates test hook
    const double* A;
    const double* cool;
    int nb_given;
    int n_pairs;
};

template <int P, int R, int WAVES, bool GIVEN>
__global__ void __launch_bounds__(64 * WAVES) k_solve(KArgs a) {
    constexpr int PPW = 64 / P;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane & (P - 1);
    const int seg = lane / P;

    int gslot = 0, cell, nb;
    GrainView gv{};
    if constexpr (!GIVEN) {
        const int2 it = a.items[blockIdx.x];
        gslot = it.x;
        cell = it.y + wave * PPW + seg;
        gv = a.views[gslot];
        nb = gv.nb;
    } else {
        cell = (blockIdx.x * WAVES + wave) * PPW + seg;
        nb = a.nb_given;
    }
    const int n_live = GIVEN ? a.n_pairs : a.n_cells;
    const bool live = cell < n_live;
    const int cellc = live ? cell : 0;

    float gm[R];
    float intra[R];
    double total = 0.0;
    bool bad = false;
    DPar* dpar_s = reinterpret_cast<DPar*>(smem);
    float* tab = nullptr;

    if constexpr (!GIVEN) {
        const int L = a.L;
        tab = reinterpret_cast<float*>(smem + sizeof(DPar) * R * P) + (wave * PPW + seg) * a.tabstride;
        for (int d = threadIdx.x; d < nb; d += 64 * WAVES) dpar_s[d] = gv.dpar[d];

        // Pass 1: absorbed-power suffix integrals Cum_j = int_{lambda_j} c u C_abs dlambda
        // (trapezoid), FP64, chunked over the segment's lanes.
        const double* uc = a.u + static_cast<size_t>(cellc) * L;
        const int cs = (L + P - 1) / P;
        const int j0 = q * cs;
        const int j1 = min(j0 + cs, L);
        double csum = 0.0;
        if (j0 < j1) {
            double rho_n = kLight * clean_field(uc[j0], bad) * gv.cabs[j0];
            for (int j = j0; j < j1; ++j) {
                const double rho = rho_n;
                if (j + 1 < L) {
                    rho_n = kLight * clean_field(uc[j + 1], bad) * gv.cabs[j + 1];
                    csum += 0.5 * (rho + rho_n) * (a.lam[j + 1] - a.lam[j]);
                }
            }
        }
        const double carry = seg_suffix_exclusive<P>(csum, q);
        total = seg_sum<P>(csum);
        const double inv_total = total > 0.0 ? 1.0 / total : 0.0;
        if (j0 < j1) {
            double cum = carry;
            double rho_n = (j1 < L) ? kLight * clean_field(uc[j1], bad) * gv.cabs[j1] : 0.0;
            for (int j = j1 - 1; j >= j0; --j) {
                const double rho = kLight * clean_field(uc[j], bad) * gv.cabs[j];
                if (j + 1 < L) cum += 0.5 * (rho + rho_n) * (a.lam[j + 1] - a.lam[j]);
                rho_n = rho;
                tab[j] = static_cast<float>(cum * inv_total);
            }
        }
        __syncthreads();
        // Continuous heating of row k from column k-1 (Draine & Li intrabin
        // term): absorbed power of photons too soft for the step, per unit step.
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = r * P + q;
            intra[r] = 0.0f;
            if (k >= 1 && k < nb) {
                const int js = gv.jstar[k - 1];
                if (js < L && total > 0.0)
                    intra[r] = static_cast<float>(static_cast<double>(tab[js]) * total * gv.invgap[k - 1]);
            }
        }
        __syncthreads();
        // Pass 2: tab_j = log2(u_j C_abs_j) + 3 j dlog2(lambda) - off, off = the
        // pair's largest entry (kept in gamma, so the exponent stays small).
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
            tab[j] = (v > kNoField) ? v - off : kNoField;
        }
        if (q == 0) tab[L] = kNoField;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = r * P + q;
            gm[r] = (k < nb) ? static_cast<float>(gv.gam[k] + static_cast<double>(off)) : 0.0f;
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            gm[r] = 0.0f;
            intra[r] = 0.0f;
        }
    }

    // ---- recursion ----
    double G[R];
#pragma unroll
    for (int r = 0; r < R; ++r) G[r] = 0.0;
    double part = 0.0;
    int nres = 0;
    const double* Ap = nullptr;
    const double* cp = nullptr;
    if constexpr (GIVEN) {
        Ap = a.A + static_cast<size_t>(cellc) * nb * nb;
        cp = a.cool + static_cast<size_t>(cellc) * nb;
    }

#pragma unroll
    for (int ro = 0; ro < R; ++ro) {
        if (ro * P < nb) {
            for (int l = 0; l < P; ++l) {
                const int f = ro * P + l;
                if (f >= nb) break;
                double Xf = 1.0;
                if (f > 0) {
                    const double S = seg_sum<P>(part);
                    if constexpr (GIVEN) Xf = S / cp[f];
                    else Xf = S * gv.colpar[f].invcool;
                }
                if (Xf > kBig) {
                    Xf *= kShrink;
#pragma unroll
                    for (int r = 0; r < R; ++r) G[r] *= kShrink;
                    ++nres;
                }
                if (q == l) G[ro] = Xf;

                int kb, ke, ia = 0;
                float fa = 0.0f;
                if constexpr (GIVEN) {
                    kb = f + 1;
                    ke = nb - 1;
                } else {
                    const ColPar c = gv.colpar[f];
                    kb = max(c.kb, f + 1);
                    ke = c.ke;
                    ia = c.ia;
                    fa = c.fa;
                }
                part = 0.0;
#pragma unroll
                for (int r = ro; r < R; ++r) {
                    const int kbase = r * P;
                    if (kbase < nb) {
                        const bool first = (r == ro);
                        const int k = kbase + q;
                        if (kbase + P - 1 >= kb && kbase <= ke) {
                            const bool whole = !first && kbase >= kb && kbase + P - 1 <= ke;
                            const bool on = whole || ((k >= kb) && (k <= ke) && (!first || q > l));
                            if (on) {
                                double A;
                                if constexpr (GIVEN) {
                                    A = Ap[static_cast<size_t>(k) * nb + f];
                                } else {
                                    const DPar dp = dpar_s[k - f];
                                    int jlo;
                                    float w;
                                    transition_index(ia, fa, dp.nib, dp.fb, jlo, w);
                                    // kb..ke already keep jlo in [0, L-1]; the clamp is a
                                    // single v_med3 and guards the LDS read regardless
                                    jlo = min(max(jlo, 0), a.L - 1);
                                    const float lo = tab[jlo];
                                    const float hi = tab[jlo + 1];
                                    const float x = fmaf(w, hi - lo, lo) + gm[r];
                                    A = static_cast<double>(__builtin_amdgcn_exp2f(x));
                                }
                                G[r] = fma(A, Xf, G[r]);
                            }
                        }
                        if (!first || q > l) part += G[r];
                    }
                }
                if constexpr (!GIVEN) {
                    if (l + 1 < P) {
                        if (q == l + 1 && f + 1 < nb) {
                            const double inc = static_cast<double>(intra[ro]) * Xf;
                            G[ro] += inc;
                            part += inc;
                        }
                    } else if (ro + 1 < R) {
                        if (q == 0 && f + 1 < nb) {
                            const double inc = static_cast<double>(intra[ro + 1]) * Xf;
                            G[ro + 1] += inc;
                            part += inc;
                        }
                    }
                }
            }
        }
    }

    // ---- normalisation (eq:renormalization) and outputs ----
    double sx = 0.0, mxx = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = r * P + q;
        if (k < nb) {
            sx += G[r];
            mxx = fmax(mxx, G[r]);
        }
    }
    sx = seg_sum<P>(sx);
    mxx = seg_max<P>(mxx);
    const double x0 = __shfl(G[0], seg * P, 64);
    bad = seg_maxf<P>(bad ? 1.0f : 0.0f) > 0.0f;
    if (!live) return;
    if (a.P64) {
        double* prow = a.P64 + static_cast<size_t>(cell) * nb;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = r * P + q;
            if (k < nb) prow[k] = G[r] / sx;
        }
    }
    if constexpr (!GIVEN) {
        if (a.Pt) {
            float* prow = a.Pt + a.offs[gslot] + static_cast<size_t>(cell) * nb;
            const double inv = 1.0 / mxx;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = r * P + q;
                if (k < nb) prow[k] = static_cast<float>(G[r] * inv);
            }
        }
        const size_t pair = static_cast<size_t>(cell) * a.n_gslots + gslot;
        if (q == 0) {
            if (a.pscale) a.pscale[pair] = static_cast<float>(mxx / sx);
            const unsigned flags = (sx == x0 ? 1u : 0u) | (nres > 0 ? 2u : 0u) | (bad ? 4u : 0u);
            if (a.diag) {
                a.diag[pair * 4 + 0] = static_cast<float>(total);
                a.diag[pair * 4 + 3] = static_cast<float>(flags);
            }
            if (bad && a.errword) atomicOr(a.errword, 1u);
        }
    }
}

template <int P, int R, int WAVES>
hipError_t launch_phys(const KArgs& ka, int n_items, hipStream_t s) {
    const size_t lds = sizeof(DPar) * R * P + sizeof(float) * static_cast<size_t>(WAVES) * (64 / P) * ka.tabstride;
    hipLaunchKernelGGL((k_solve<P, R, WAVES, false>), dim3(n_items), dim3(64 * WAVES), lds, s, ka);
    return hipGetLastError();
}

template <int P, int R, int WAVES>
hipError_t launch_given(const KArgs& ka, int n_pairs, hipStream_t s) {
    const int per_block = WAVES * (64 / P);
    const int blocks = (n_pairs + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_solve<P, R, WAVES, true>), dim3(blocks), dim3(64 * WAVES), 0, s, ka);
    return hipGetLastError();
}

constexpr int kWaves = 4;

}  // namespace

int solve_cells_per_item(int nb_max) {
    if (nb_max <= 256) return kWaves * 4;
    if (nb_max <= 512) return kWaves * 2;
    return kWaves;
}

hipError_t launch_solve(const Ctx& c, const SolveLaunch& sl, int nb_max, const int2* items_dev, int n_items,
                        int, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    KArgs ka{};
    ka.u = sl.u;
    ka.lam = c.lam;
    ka.L = c.L;
    ka.tabstride = (c.L + 2 + 1) & ~1;
    ka.dlam2 = static_cast<float>(c.dlnlam / std::log(2.0));
    ka.n_cells = sl.n_cells;
    ka.n_gslots = sl.n_gslots;
    ka.views = sl.views;
    ka.offs = sl.offs;
    ka.Pt = sl.Pt;
    ka.pscale = sl.pscale;
    ka.diag = sl.diag;
    ka.P64 = sl.P64;
    ka.errword = sl.errword;
    ka.items = items_dev;
    if (nb_max <= 128) return launch_phys<16, 8, kWaves>(ka, n_items, s);
    if (nb_max <= 256) return launch_phys<16, 16, kWaves>(ka, n_items, s);
    if (nb_max <= 512) return launch_phys<32, 16, kWaves>(ka, n_items, s);
    return launch_phys<64, 16, kWaves>(ka, n_items, s);
}

hipError_t launch_from_rates(const Ctx& c, int nb, int n_pairs, const double* A, const double* cool, double* P,
                             hipStream_t s) {
    KArgs ka{};
    ka.A = A;
    ka.cool = cool;
    ka.nb_given = nb;
    ka.n_pairs = n_pairs;
    ka.P64 = P;
    if (nb <= 128) return launch_given<16, 8, kWaves>(ka, n_pairs, s);
    if (nb <= 256) return launch_given<16, 16, kWaves>(ka, n_pairs, s);
    if (nb <= 512) return launch_given<32, 16, kWaves>(ka, n_pairs, s);
    return launch_given<64, 16, kWaves>(ka, n_pairs, s);
}

}  // namespace hsd
