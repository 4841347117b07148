// The table method: spectra precomputed at log-spaced field strengths and
// interpolated in the field strength alone.  The paper's introduction names
// such precomputed emissivity tables as the cheap alternative to the full
// solve that other codes use; here it is the yardstick of the learned
// surrogate.  Each node of the table is a plain solve (the library's own
// kernels) of the reference field shape scaled to U_k; a cell is looked up by
// its field's total energy relative to the reference, U = int u / int u_ref,
// and its spectrum is A 2^y with y interpolated linearly in log10 U between
// the two bracketing nodes of y_k = log2(j_k / A_k) (A: absorbed power of the
// pair, so that every looked-up spectrum carries the cell's own absorbed
// power).
#include <cmath>

#include "hsd_internal.h"

namespace hsd {
namespace {

constexpr float kNoEmission = -1.0e30f;   // log2 of a zero spectrum value

// u_out[k][l] = 10^(lo + k step) u_ref[l].
__global__ void __launch_bounds__(256) k_node_fields(const double* u_ref, double lo, double step, int n_nodes, int L,
                                                     double* u_out) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= static_cast<long long>(n_nodes) * L) return;
    const int k = static_cast<int>(i / L);
    const int l = static_cast<int>(i % L);
    u_out[i] = exp10(lo + k * step) * u_ref[l];
}

// Per cell: the field's energy int u dlambda (trapezoid, FP64), and per
// listed grain its absorbed power A = int c u C_abs dlambda.  One block per
// cell; the weighted field c u w (trapezoid weights w) is staged in LDS and
// each wave takes every fourth grain, lanes striding the wavelengths, the
// partial sums combined in a fixed order.
__global__ void __launch_bounds__(256) k_cell_energies(const double* u, const double* lam, int L, int G,
                                                       const double* const* cabs, double* energy, double* A) {
    __shared__ double wu[kMaxLambda];
    __shared__ double red[4];
    const int cell = blockIdx.x;
    const double* uc = u + static_cast<long long>(cell) * L;
    double e = 0.0;
    for (int l = threadIdx.x; l < L; l += 256) {
        double w = 0.0;
        if (l > 0) w += 0.5 * (lam[l] - lam[l - 1]);
        if (l + 1 < L) w += 0.5 * (lam[l + 1] - lam[l]);
        wu[l] = w * uc[l];
        e += w * uc[l];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m, 64);
    if (lane == 0) red[wave] = e;
    __syncthreads();
    if (threadIdx.x == 0 && energy) energy[cell] = (red[0] + red[1]) + (red[2] + red[3]);
    for (int g = wave; g < G; g += 4) {
        const double* cg = cabs[g];
        double s = 0.0;
        for (int l = lane; l < L; l += 64) s += wu[l] * cg[l];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) A[static_cast<long long>(cell) * G + g] = kLight * s;
    }
}

// table[g][k][l] = log2(j[k][g][l] / A[k][g]) (kNoEmission where j = 0).
__global__ void __launch_bounds__(256) k_table_logs(const float* j, const double* A, int n_nodes, int G, int L,
                                                    float* table) {
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= static_cast<long long>(n_nodes) * G * L) return;
    const int l = static_cast<int>(i % L);
    const long long kg = i / L;
    const int g = static_cast<int>(kg % G);
    const int k = static_cast<int>(kg / G);
    const float v = j[i];
    const double a = A[kg];
    table[(static_cast<long long>(g) * n_nodes + k) * L + l] =
        (v > 0.f && a > 0.0) ? static_cast<float>(log2(static_cast<double>(v) / a)) : kNoEmission;
}

// j[c][g][l] = A[c][g] 2^((1 - w) y_k + w y_(k+1)), k and w from the cell's
// log10 U on the node grid (clamped to its ends).  Block (cell, group of four
// grains); each wave writes one grain's row.
__global__ void __launch_bounds__(256) k_table_eval(const double* energy, const double* ref_energy, const double* A,
                                                    const float* table, int n_nodes, double lo, double step, int G,
                                                    int L, float* j) {
    const int cell = blockIdx.x;
    const int g = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (g >= G) return;
    const int lane = threadIdx.x & 63;
    const double e = energy[cell];
    const double eref = *ref_energy;
    double t = (e > 0.0 && eref > 0.0) ? (log10(e / eref) - lo) / step : 0.0;
    t = fmin(fmax(t, 0.0), static_cast<double>(n_nodes - 1));
    int k = static_cast<int>(t);
    if (k > n_nodes - 2) k = n_nodes - 2;
    const float w = static_cast<float>(t - k);
    const double a = A[static_cast<long long>(cell) * G + g];
    const float* y0 = table + (static_cast<long long>(g) * n_nodes + k) * L;
    const float* y1 = y0 + L;
    float* out = j + (static_cast<long long>(cell) * G + g) * L;
    for (int l = lane; l < L; l += 64) {
        const float a0 = y0[l], a1 = y1[l];
        // a node without emission gives none, unless the weight puts the value wholly on the other node
        const bool some = (a0 > kNoEmission || w == 1.f) && (a1 > kNoEmission || w == 0.f);
        const float y = w == 0.f ? a0 : (w == 1.f ? a1 : fmaf(w, a1 - a0, a0));
        out[l] = some ? static_cast<float>(a * static_cast<double>(exp2f(y))) : 0.f;
    }
}

// Energy budget of the table (the reference of the HSD_CHECK_TABLE check):
// for each grain g and node k, the node spectrum's emitted power per unit
// absorbed power, rho[g][k] = 4 pi int 2^(y_k) dlambda (trapezoid on the grid,
// no emission where y_k holds none).  One wave per (g, k); FP64 sums in a
// fixed order (lane strides, then a shuffle tree).
__global__ void __launch_bounds__(256) k_budget_nodes(const float* table, int rows, int L, const double* lam,
                                                      double* rho) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int lane = threadIdx.x & 63;
    const float* y = table + static_cast<long long>(row) * L;
    double s = 0.0;
    for (int l = lane; l < L; l += 64) {
        double w = 0.0;
        if (l > 0) w += 0.5 * (lam[l] - lam[l - 1]);
        if (l + 1 < L) w += 0.5 * (lam[l + 1] - lam[l]);
        const float v = y[l];
        if (v > kNoEmission) s += w * exp2(static_cast<double>(v));
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) rho[row] = 4.0 * M_PI * s;
}

// Each cell's position on the table's node grid, t = (log10(E / E_ref) - lo)
// / step clamped to [0, n_nodes - 1], E the field's energy (the lookup of
// k_table_eval).
__global__ void __launch_bounds__(256) k_node_coord(const double* energy, const double* ref_energy, int n_cells,
                                                    double lo, double step, int n_nodes, double* t) {
    const int cell = blockIdx.x * 256 + threadIdx.x;
    if (cell >= n_cells) return;
    const double e = energy[cell], eref = *ref_energy;
    const double x = (e > 0.0 && eref > 0.0) ? (log10(e / eref) - lo) / step : 0.0;
    t[cell] = fmin(fmax(x, 0.0), static_cast<double>(n_nodes - 1));
}

}  // namespace

hipError_t launch_node_fields(const double* u_ref, double lo, double step, int n_nodes, int L, double* u_out,
                              hipStream_t s) {
    const long long n = static_cast<long long>(n_nodes) * L;
    hipLaunchKernelGGL(k_node_fields, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, u_ref, lo, step,
                       n_nodes, L, u_out);
    return hipGetLastError();
}

hipError_t launch_cell_energies(const double* u, const double* lam, int n_cells, int L, int G,
                                const double* const* cabs, double* energy, double* A, hipStream_t s) {
    if (n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_energies, dim3(n_cells), dim3(256), 0, s, u, lam, L, G, cabs, energy, A);
    return hipGetLastError();
}

hipError_t launch_table_logs(const float* j, const double* A, int n_nodes, int G, int L, float* table, hipStream_t s) {
    const long long n = static_cast<long long>(n_nodes) * G * L;
    hipLaunchKernelGGL(k_table_logs, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, j, A, n_nodes, G,
                       L, table);
    return hipGetLastError();
}

hipError_t launch_budget_nodes(const float* table, int n_nodes, int G, int L, const double* lam, double* rho,
                               hipStream_t s) {
    const int rows = n_nodes * G;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_budget_nodes, dim3((rows + 3) / 4), dim3(256), 0, s, table, rows, L, lam, rho);
    return hipGetLastError();
}

hipError_t launch_node_coord(const double* energy, const double* ref_energy, int n_cells, double lo, double step,
                             int n_nodes, double* t, hipStream_t s) {
    if (n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_coord, dim3((n_cells + 255) / 256), dim3(256), 0, s, energy, ref_energy, n_cells, lo,
                       step, n_nodes, t);
    return hipGetLastError();
}

hipError_t launch_table_eval(const double* energy, const double* ref_energy, const double* A, const float* table,
                             int n_nodes, double lo, double step, int n_cells, int G, int L, float* j, hipStream_t s) {
    if (n_cells <= 0 || G <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_eval, dim3(n_cells, (G + 3) / 4), dim3(256), 0, s, energy, ref_energy, A, table, n_nodes,
                       lo, step, G, L, j);
    return hipGetLastError();
}

}  // namespace hsd
