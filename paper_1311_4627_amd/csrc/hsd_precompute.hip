// Per-grain precompute on the device (everything in a grain's solve that does
// not depend on the field; Sec. 2.2 notes the cooling term can be precomputed).
// All arithmetic is IEEE double precision except the single-precision tables
// the hot kernels read.
#include <cmath>
#include <cstring>

#include "hsd_index.h"
#include "hsd_internal.h"

namespace hsd {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
GLRule gauss_legendre(int n) {
    GLRule r{};
    r.n = n;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        double w = 2.0 / ((1.0 - x * x) * dp * dp);
        r.x[i] = -x;
        r.w[i] = w;
        r.x[n - 1 - i] = x;
        r.w[n - 1 - i] = w;
    }
    return r;
}

namespace {

// D(y) = int_0^y x^3 / (e^x - 1) dx by composite Gauss-Legendre on panels of
// width <= 2; the integrand beyond x = 60 is below 1e-20 of the total.
__device__ double debye_integral(double y, const GLRule& gl) {
    const double top = y < 60.0 ? y : 60.0;
    const int np = static_cast<int>(ceil(top / 2.0));
    const double h = top / np;
    double s = 0.0;
    for (int p = 0; p < np; ++p) {
        const double mid = (p + 0.5) * h, half = 0.5 * h;
        double ps = 0.0;
        for (int q = 0; q < gl.n; ++q) {
            const double x = mid + half * gl.x[q];
            ps += gl.w[q] * x * x * x / expm1(x);
        }
        s += half * ps;
    }
    return s;
}

// Debye internal energy of 3N modes: E(T) = 9 N k T (T/theta)^3 D(theta/T).
__device__ double debye_energy(double T, double N, double theta, const GLRule& gl) {
    const double r = T / theta;
    return 9.0 * N * kBoltzmann * T * r * r * r * debye_integral(theta / T, gl);
}

// Bin enthalpies, widths and temperatures.  T(E) by bisection on ln T between
// two bounds that always bracket the root: E <= 3NkT (the classical value is
// never exceeded) and E >= 3Nk(T - 3 theta / 8) (the Debye deficit grows to
// 9 N k theta / 8), plus the low-temperature bound E <= (3 pi^4/5) N k T^4 / theta^3.
__global__ void k_grid_temps(int n, double E_lo, double E_hi, double N, double theta, GLRule gl,
                             double* E, double* dE, double* T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int M = n - 1;
    const double ratio = E_hi / E_lo;
    const double Ei = E_lo * pow(ratio, static_cast<double>(i) / M);
    const double r = pow(ratio, 1.0 / M);
    E[i] = Ei;
    dE[i] = Ei * (sqrt(r) - 1.0 / sqrt(r));
    const double Nk3 = 3.0 * N * kBoltzmann;
    double lo = Ei / Nk3;
    const double lowT = pow(Ei * theta * theta * theta / ((3.0 * kPi * kPi * kPi * kPi / 5.0) * N * kBoltzmann), 0.25);
    if (lowT > lo) lo = lowT;
    double hi = Ei / Nk3 + 0.375 * theta;
    double a = log(lo), b = log(hi);
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m <= a || m >= b) break;
        if (debye_energy(exp(m), N, theta, gl) < Ei) a = m; else b = m;
    }
    T[i] = exp(0.5 * (a + b));
}

// C_abs at photon energy E from the grain's table (log-log between nodes,
// lambda^-p beyond the long end, the end value beyond the short end).
struct CabsView {
    const double* cabs;
    double lnlam0, dlnlam;
    int L;
    double p_long;
};

__device__ double cabs_at_lnE(const CabsView& cv, double lnE) {
    const double lnlam = log(kHC) - lnE;
    const double t = (lnlam - cv.lnlam0) / cv.dlnlam;
    if (t >= cv.L - 1) {
        return cv.cabs[cv.L - 1] * exp(-cv.p_long * (lnlam - (cv.lnlam0 + (cv.L - 1) * cv.dlnlam)));
    }
    if (t <= 0.0) return cv.cabs[0];
    int j = static_cast<int>(floor(t));
    if (j > cv.L - 2) j = cv.L - 2;
    const double w = t - j;
    const double a = log(cv.cabs[j]), b = log(cv.cabs[j + 1]);
    return exp(a + w * (b - a));
}

// Cooling rate T_(f-1)f = [8 pi / (h^3 c^2)] int_0^{E_f} E^3 C_abs / (e^{E/kT_f} - 1) dE
// / (E_f - E_(f-1)) (Sec. 2.2, eq:cooling), integrated in u = ln E over all
// photon energies up to E_f.  One 64-thread block per bin; each thread sums
// a strided set of quadrature panels: 24 panels of width 2 (16-point rule)
// below the grid, one panel per wavelength-grid interval (6-point rule; the
// cross-section is a power law inside it), and panels of width 0.1
// (12-point rule) above the grid up to min(E_f, 900 kT).  The block sum is a
// fixed-order tree, so the result is deterministic.
__global__ void k_cooling(int n, const double* E, const double* T, CabsView cv, GLRule g16, GLRule g6,
                          GLRule g12, double* cool) {
    const int f = blockIdx.x;
    __shared__ double red[64];
    const int tid = threadIdx.x;
    double acc = 0.0;
    if (f >= 1) {
        const double Ef = E[f], kT = kBoltzmann * T[f];
        const double uf = log(Ef);
        const double u_nlo = log(kHC) - (cv.lnlam0 + (cv.L - 1) * cv.dlnlam);   // softest grid photon
        const double u_nhi = log(kHC) - cv.lnlam0;                               // hardest grid photon
        const int n_soft = 24;
        const int n_grid = cv.L - 1;
        const double u_hard_top = fmin(uf, log(900.0 * kT));
        const int n_hard = (uf > u_nhi && u_hard_top > u_nhi) ? static_cast<int>(ceil((u_hard_top - u_nhi) / 0.1)) : 0;
        const int total = n_soft + n_grid + n_hard;
        for (int p = tid; p < total; p += 64) {
            double a, b;
            const GLRule* g;
            if (p < n_soft) {
                const double top = fmin(uf, u_nlo);
                a = top - 48.0 + 2.0 * p;
                b = a + 2.0;
                g = &g16;
            } else if (p < n_soft + n_grid) {
                const int m = p - n_soft;                     // m-th interval in ascending energy
                a = u_nlo + m * cv.dlnlam;
                b = a + cv.dlnlam;
                if (m == n_grid - 1) b = u_nhi;
                if (a >= uf) continue;
                if (b > uf) b = uf;
                g = &g6;
            } else {
                const int m = p - n_soft - n_grid;
                a = u_nhi + 0.1 * m;
                b = fmin(a + 0.1, u_hard_top);
                if (b <= a) continue;
                g = &g12;
            }
            const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
            double ps = 0.0;
            for (int q = 0; q < g->n; ++q) {
                const double u = mid + half * g->x[q];
                const double Ee = exp(u);
                const double x = Ee / kT;
                if (x > 740.0) continue;
                ps += g->w[q] * Ee * Ee * Ee * Ee * cabs_at_lnE(cv, u) / expm1(x);
            }
            acc += half * ps;
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        if (f == 0) {
            cool[0] = 0.0;
        } else {
            const double pref = 8.0 * kPi / (kPlanck * kPlanck * kPlanck * kLight * kLight);
            cool[f] = pref * red[0] / (E[f] - E[f - 1]);
        }
    }
}

// Emission table: C_abs(lambda_j) B_lambda_j(T_i) [E_i >= hc / lambda_j]
// (Sec. 2.3, eq:emission-lambda without the stray P_i) in double precision,
// then scaled per wavelength by its largest entry so the single-precision
// contraction sees values in [0, 1].
__global__ void k_planck_raw(int n, int L, int Lp, const double* E, const double* T, const double* lam,
                             const double* cabs, double* raw) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= Lp) return;
    double v = 0.0;
    if (j < L) {
        const double l = lam[j];
        if (E[i] >= kHC / l) {
            const double x = kHC / (l * kBoltzmann * T[i]);
            const double l2 = l * l;
            v = cabs[j] * 2.0 * kPlanck * kLight * kLight / (l2 * l2 * l) / expm1(x);
        }
    }
    raw[static_cast<size_t>(i) * Lp + j] = v;
}

__global__ void k_planck_scale(int n, int Lp, const double* raw, float* Bt, float* bscale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Lp) return;
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, raw[static_cast<size_t>(i) * Lp + j]);
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (int i = 0; i < n; ++i) Bt[static_cast<size_t>(i) * Lp + j] = static_cast<float>(raw[static_cast<size_t>(i) * Lp + j] * inv);
    bscale[j] = static_cast<float>(m);
}

// The scaled Planck table as two BF16 terms for the split-BF16 contraction,
// transposed (wavelength-major) and zero padded to nbp bins:
// Bh[j][i] = bf16(Bt[i][j]), Bl[j][i] = bf16(Bt[i][j] - Bh[j][i]).
__global__ void k_planck_split(int n, int Lp, int nbp, const float* Bt, unsigned short* Bh, unsigned short* Bl) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long long>(Lp) * nbp) return;
    const int j = static_cast<int>(t / nbp), i = static_cast<int>(t - static_cast<long long>(j) * nbp);
    const float v = i < n ? Bt[static_cast<size_t>(i) * Lp + j] : 0.f;
    const __bf16 hi = static_cast<__bf16>(v);
    const __bf16 lo = static_cast<__bf16>(v - static_cast<float>(hi));
    Bh[t] = __builtin_bit_cast(unsigned short, hi);
    Bl[t] = __builtin_bit_cast(unsigned short, lo);
}

__device__ int first_at_least(const double* lam, int L, double lnlam0, double dlnlam, double x) {
    // first j with lam[j] >= x, L if none; closed-form guess corrected on the actual grid values
    if (!(x > 0.0)) return 0;
    double t = (log(x) - lnlam0) / dlnlam;
    int j;
    if (t <= 0.0) j = 0;
    else if (t >= L) j = L;
    else j = static_cast<int>(ceil(t));
    while (j > 0 && lam[j - 1] >= x) --j;
    while (j < L && lam[j] < x) ++j;
    return j;
}

__device__ void split_coord(double v, int& ip, float& fp) {
    double fl = floor(v);
    float fr = static_cast<float>(v - fl);
    if (fr >= 1.0f) {
        fl += 1.0;
        fr = 0.0f;
    }
    ip = static_cast<int>(fl);
    fp = fr;
}

// Solver tables.  For column i: a_i = (ln(hc) - ln E_i - ln lambda_0) / dln(lambda);
// for distance d: b_d = ln(r^d - 1) / dln(lambda); the transition's grid
// coordinate is a_i - b_d.  kb..ke are the rows whose coordinate falls in
// [0, L-1] under the exact index arithmetic the solver uses.
__global__ void k_tables(int n, int L, double E_lo, double E_hi, double lnlam0, double dlnlam,
                         const double* lam, const double* E, const double* dE, const double* cool,
                         ColPar* colpar, DPar* dpar, double* gam, double* invgap, int* jstar, int* jrep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int M = n - 1;
    const double lnr = log(E_hi / E_lo) / M;
    // distance table
    if (i >= 1) {
        const double b = log(expm1(i * lnr)) / dlnlam;
        int ib;
        float fb;
        split_coord(b, ib, fb);
        dpar[i].nib = -ib;
        dpar[i].fb = fb;
    } else {
        // distance 0 (a row at or below the diagonal) lands far below the grid
        dpar[0].nib = -(1 << 20);
        dpar[0].fb = 0.0f;
    }
    // column parameters
    const double lnEi = log(E_lo) + i * lnr;
    const double a = (log(kHC) - lnEi - lnlam0) / dlnlam;
    int ia;
    float fa;
    split_coord(a, ia, fa);
    ColPar cp;
    cp.invcool = (i >= 1) ? 1.0 / cool[i] : 0.0;
    cp.ia = ia - 1;
    cp.fa = fa + 1.0f;
    cp.jstar = L;
    cp.invgap = 0.0f;
    int kb = n, ke = -1;
    for (int k = i + 1; k < n; ++k) {
        const int d = k - i;
        const double b = log(expm1(d * lnr)) / dlnlam;
        int ib;
        float fb;
        split_coord(b, ib, fb);
        int jlo;
        float w;
        transition_index(cp.ia, cp.fa, -ib, fb, jlo, w);
        if (jlo >= 0 && jlo <= L - 1) {
            if (k < kb) kb = k;
            if (k > ke) ke = k;
        }
    }
    cp.kb = kb;
    cp.ke = ke;
    // row constant of the rate exponent: log2(dE_k) + 3 log2(lambda_0) - log2(h^2 c)
    gam[i] = log2(dE[i]) + 3.0 * lnlam0 / log(2.0) - log2(kPlanck * kPlanck * kLight);
    // continuous heating below the step to the next bin (Draine & Li intrabin term)
    if (i < M) {
        const double gap = E[i + 1] - E[i];
        invgap[i] = 1.0 / gap;
        int js;
        if (gap > kHC / lam[0]) {
            js = 0;
        } else {
            const double eps_lo = (E[i + 1] - 0.5 * dE[i + 1]) - E[i];
            js = eps_lo > 0.0 ? first_at_least(lam, L, lnlam0, dlnlam, kHC / eps_lo) : L;
        }
        jstar[i] = js;
        cp.jstar = js;
        cp.invgap = static_cast<float>(1.0 / gap);
    } else {
        invgap[i] = 0.0;
        jstar[i] = L;
    }
    colpar[i] = cp;
    // photons a grain in bin i can absorb without leaving the grid's top bin
    const double edge = E[M] + 0.5 * dE[M] - E[i];
    jrep[i] = edge > 0.0 ? first_at_least(lam, L, lnlam0, dlnlam, kHC / edge) : L;
}

}  // namespace

hipError_t build_grain_tables(Ctx& c, Grain& g) {
    const int n = g.n_bins, L = c.L, Lp = c.Lp;
    hipError_t e;
    const GLRule g16 = gauss_legendre(16), g6 = gauss_legendre(6), g12 = gauss_legendre(12);
    hipLaunchKernelGGL(k_grid_temps, dim3((n + 63) / 64), dim3(64), 0, 0, n, g.E_lo, g.E_hi, g.n_atoms, g.theta,
                       g16, g.E, g.dE, g.T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    CabsView cv{g.cabs, c.lnlam0, c.dlnlam, L, g.longwave};
    hipLaunchKernelGGL(k_cooling, dim3(n), dim3(64), 0, 0, n, g.E, g.T, cv, g16, g6, g12, g.cool);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* raw = nullptr;
    if ((e = hipMalloc(&raw, sizeof(double) * static_cast<size_t>(n) * Lp)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_planck_raw, dim3((Lp + 63) / 64, n), dim3(64), 0, 0, n, L, Lp, g.E, g.T, c.lam, g.cabs, raw);
    if ((e = hipGetLastError()) != hipSuccess) { hipFree(raw); return e; }
    hipLaunchKernelGGL(k_planck_scale, dim3((Lp + 63) / 64), dim3(64), 0, 0, n, Lp, raw, g.Bt, g.bscale);
    if ((e = hipGetLastError()) != hipSuccess) { hipFree(raw); return e; }
    {
        const long long tot = static_cast<long long>(Lp) * g.nbp;
        hipLaunchKernelGGL(k_planck_split, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, 0, n, Lp,
                           g.nbp, g.Bt, g.Bh, g.Bl);
        if ((e = hipGetLastError()) != hipSuccess) { hipFree(raw); return e; }
    }
    hipLaunchKernelGGL(k_tables, dim3((n + 63) / 64), dim3(64), 0, 0, n, L, g.E_lo, g.E_hi, c.lnlam0, c.dlnlam,
                       c.lam, g.E, g.dE, g.cool, g.colpar, g.dpar, g.gam, g.invgap, g.jstar, g.jrep);
    if ((e = hipGetLastError()) != hipSuccess) { hipFree(raw); return e; }
    e = hipDeviceSynchronize();
    hipFree(raw);
    return e;
}

}  // namespace hsd
