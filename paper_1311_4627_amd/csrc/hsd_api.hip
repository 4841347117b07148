// C ABI entry points (include/hsd.h): argument checks, device memory of the
// context and its grains, and the order of kernel launches of a solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hsd_internal.h"

using hsd::Ctx;
using hsd::Grain;

struct hsd_ctx {
    Ctx c;
    std::vector<hsd::GrainView> views_h;
    std::vector<long long> offs_h;
    std::vector<int2> items_h;
};

namespace {

hsd_status fail(hsd_ctx* ctx, hsd_status st, const std::string& msg) {
    if (ctx) ctx->c.err = msg;
    return st;
}

hsd_status hip_fail(hsd_ctx* ctx, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? HSD_ERR_OOM : HSD_ERR_HIP, m);
}

#define HSD_HIP(ctx, expr)                                             \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);       \
    } while (0)

template <typename T>
hipError_t grow(T*& p, size_t& cap, size_t need) {
    if (need <= cap && p) return hipSuccess;
    if (p) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        hipFree(p);
        p = nullptr;
        cap = 0;
    }
    size_t n = std::max<size_t>(need, 1);
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
}

void free_grain(Grain& g) {
    hipFree(g.E); hipFree(g.dE); hipFree(g.T); hipFree(g.cool); hipFree(g.colpar); hipFree(g.dpar);
    hipFree(g.gam); hipFree(g.invgap); hipFree(g.jstar); hipFree(g.jrep); hipFree(g.cabs); hipFree(g.Bt);
    hipFree(g.bscale);
    g = Grain{};
}

bool grain_ok(const hsd_ctx* ctx, int32_t id) {
    return id >= 0 && static_cast<size_t>(id) < ctx->c.grains.size();
}

// Solve launches shared by hsd_solve and hsd_solve_P.
hsd_status run_solve(hsd_ctx* ctx, int32_t n_cells, const double* u, int32_t n_grains, const int32_t* ids,
                     float* j, float* diag, double* P64, hipStream_t s) {
    Ctx& c = ctx->c;
    // per-slot row offsets in the scaled-P workspace
    ctx->views_h.resize(n_grains);
    ctx->offs_h.resize(n_grains);
    long long rows = 0;
    int nb_hi = 0;
    for (int g = 0; g < n_grains; ++g) {
        const Grain& gr = c.grains[ids[g]];
        hsd::GrainView v{gr.colpar, gr.dpar, gr.gam, gr.invgap, gr.jstar, gr.jrep, gr.cabs,
                         std::pow(gr.E_hi / gr.E_lo, 1.0 / (gr.n_bins - 1)), gr.n_bins, 0};
        ctx->views_h[g] = v;
        ctx->offs_h[g] = rows;
        rows += static_cast<long long>(n_cells) * gr.n_bins;
        nb_hi = std::max(nb_hi, gr.n_bins);
    }
    const bool want_pt = (j != nullptr) || (diag != nullptr);
    if (want_pt) HSD_HIP(ctx, grow(c.Pt, c.Pt_cap, static_cast<size_t>(rows)));
    HSD_HIP(ctx, grow(c.pscale, c.pscale_cap, static_cast<size_t>(n_cells) * n_grains));
    HSD_HIP(ctx, grow(c.views, c.views_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(c.offs, c.offs_cap, static_cast<size_t>(n_grains)));
    // work items: bin-count classes, longest first; within a class slots in order
    static const int class_hi[4] = {1024, 512, 256, 128};
    static const int class_lo[4] = {512, 256, 128, 0};
    ctx->items_h.clear();
    std::vector<int> cls_begin(5, 0);
    for (int ci = 0; ci < 4; ++ci) {
        cls_begin[ci] = static_cast<int>(ctx->items_h.size());
        const int cpi = hsd::solve_cells_per_item(class_hi[ci]);
        std::vector<int> slots;
        for (int g = 0; g < n_grains; ++g) {
            const int nb = c.grains[ids[g]].n_bins;
            if (nb > class_lo[ci] && nb <= class_hi[ci]) slots.push_back(g);
        }
        std::stable_sort(slots.begin(), slots.end(), [&](int x, int y) {
            return c.grains[ids[x]].n_bins > c.grains[ids[y]].n_bins;
        });
        // Work items (slot, first cell).  Workgroups are dealt to the 8 XCDs
        // round-robin by id, so item b runs on XCD b % 8: give each XCD whole
        // cell blocks, all grains of a block in a row, so the block's field rows
        // are fetched into that XCD's L2 once for every grain of the class.
        const int nsl = static_cast<int>(slots.size());
        const int ncb = (n_cells + cpi - 1) / cpi;
        if (nsl > 0) {
            const int ncb8 = (ncb + 7) / 8 * 8;
            for (int b = 0; b < ncb8 * nsl; ++b) {
                const int x = b % 8, m = b / 8;
                const int cb = 8 * (m / nsl) + x;
                if (cb >= ncb) continue;
                ctx->items_h.push_back(make_int2(slots[m % nsl], cb * cpi));
            }
        }
    }
    cls_begin[4] = static_cast<int>(ctx->items_h.size());
    HSD_HIP(ctx, grow(c.items, c.items_cap, std::max<size_t>(ctx->items_h.size(), 1)));
    HSD_HIP(ctx, hipMemcpyAsync(c.views, ctx->views_h.data(), sizeof(hsd::GrainView) * n_grains,
                                hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(c.offs, ctx->offs_h.data(), sizeof(long long) * n_grains, hipMemcpyHostToDevice, s));
    if (!ctx->items_h.empty())
        HSD_HIP(ctx, hipMemcpyAsync(c.items, ctx->items_h.data(), sizeof(int2) * ctx->items_h.size(),
                                    hipMemcpyHostToDevice, s));
    hsd::SolveLaunch sl{};
    sl.u = u;
    sl.n_cells = n_cells;
    sl.n_gslots = n_grains;
    sl.views = c.views;
    sl.offs = c.offs;
    sl.Pt = want_pt ? c.Pt : nullptr;
    sl.pscale = c.pscale;
    sl.diag = diag;
    sl.P64 = P64;
    sl.errword = c.errword;
    if (c.timing) HSD_HIP(ctx, hipEventRecord(c.ev[0], s));
    for (int ci = 0; ci < 4; ++ci) {
        const int n_it = cls_begin[ci + 1] - cls_begin[ci];
        if (n_it == 0) continue;
        HSD_HIP(ctx, hsd::launch_solve(c, sl, class_hi[ci], c.items + cls_begin[ci], n_it, 0, s));
    }
    if (c.timing) HSD_HIP(ctx, hipEventRecord(c.ev[1], s));
    if (j) {
        for (int g = 0; g < n_grains; ++g) {
            const Grain& gr = c.grains[ids[g]];
            hsd::ContractLaunch cl{c.Pt + ctx->offs_h[g], c.pscale, gr.Bt, gr.bscale, j, n_cells, gr.n_bins,
                                   c.L, c.Lp, n_grains, g};
            HSD_HIP(ctx, hsd::launch_contract(cl, s));
        }
    }
    if (c.timing) HSD_HIP(ctx, hipEventRecord(c.ev[2], s));
    if (diag && j) {
        hsd::DiagLaunch dl{c.lam, j, diag, n_cells, c.L, n_grains};
        HSD_HIP(ctx, hsd::launch_diag(dl, s));
    }
    if (c.timing) {
        HSD_HIP(ctx, hipEventRecord(c.ev[3], s));
        c.timed = true;
    }
    return HSD_OK;
}

}  // namespace

extern "C" {

hsd_status hsd_create(int32_t device, const double* lambda_host, int32_t n_lambda, hsd_ctx** out) {
    if (!out) return HSD_ERR_INVALID_ARG;
    *out = nullptr;
    if (!lambda_host || n_lambda < 16 || n_lambda > hsd::kMaxLambda) return HSD_ERR_INVALID_ARG;
    for (int i = 0; i < n_lambda; ++i)
        if (!(lambda_host[i] > 0.0) || !std::isfinite(lambda_host[i])) return HSD_ERR_INVALID_ARG;
    for (int i = 1; i < n_lambda; ++i)
        if (!(lambda_host[i] > lambda_host[i - 1])) return HSD_ERR_INVALID_ARG;
    const double ln0 = std::log(lambda_host[0]);
    const double dl = (std::log(lambda_host[n_lambda - 1]) - ln0) / (n_lambda - 1);
    for (int i = 0; i < n_lambda; ++i) {
        const double want = ln0 + i * dl;
        if (std::fabs(std::log(lambda_host[i]) - want) > 1e-9 * std::max(1.0, std::fabs(want)))
            return HSD_ERR_UNSUPPORTED_GRID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HSD_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return HSD_ERR_HIP;
    hsd_ctx* ctx = new (std::nothrow) hsd_ctx();
    if (!ctx) return HSD_ERR_OOM;
    Ctx& c = ctx->c;
    c.device = device;
    c.L = n_lambda;
    c.Lp = (n_lambda + 63) / 64 * 64;
    c.lnlam0 = ln0;
    c.dlnlam = dl;
    c.lam_host.assign(lambda_host, lambda_host + n_lambda);
    if (hipMalloc(&c.lam, sizeof(double) * n_lambda) != hipSuccess ||
        hipMalloc(&c.errword, sizeof(unsigned)) != hipSuccess) {
        hipFree(c.lam);
        delete ctx;
        return HSD_ERR_OOM;
    }
    if (hipMemcpy(c.lam, lambda_host, sizeof(double) * n_lambda, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c.errword, 0, sizeof(unsigned)) != hipSuccess) {
        hipFree(c.lam);
        hipFree(c.errword);
        delete ctx;
        return HSD_ERR_HIP;
    }
    *out = ctx;
    return HSD_OK;
}

void hsd_destroy(hsd_ctx* ctx) {
    if (!ctx) return;
    Ctx& c = ctx->c;
    hipSetDevice(c.device);
    hipDeviceSynchronize();
    for (auto& g : c.grains) free_grain(g);
    hipFree(c.lam);
    hipFree(c.errword);
    hipFree(c.Pt);
    hipFree(c.pscale);
    hipFree(c.diag_tmp);
    hipFree(c.views);
    hipFree(c.offs);
    hipFree(c.items);
    for (auto& e : c.ev)
        if (e) hipEventDestroy(e);
    delete ctx;
}

const char* hsd_last_error(const hsd_ctx* ctx) {
    return ctx ? ctx->c.err.c_str() : "null context";
}

hsd_status hsd_add_grain(hsd_ctx* ctx, const hsd_grain_desc* d, int32_t* grain_id) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!d || !grain_id) return fail(ctx, HSD_ERR_INVALID_ARG, "null descriptor or id pointer");
    Ctx& c = ctx->c;
    const int n = d->n_bins;
    if (n < 16 || n > hsd::kMaxBins || n % 16 != 0)
        return fail(ctx, HSD_ERR_INVALID_ARG, "n_bins must be a multiple of 16 in [16, 1024]");
    if (!(d->E_lo_erg > 0.0) || !(d->E_hi_erg > d->E_lo_erg) || !std::isfinite(d->E_hi_erg))
        return fail(ctx, HSD_ERR_INVALID_ARG, "need 0 < E_lo < E_hi");
    if (!(d->n_atoms > 0.0) || !(d->theta_debye_K > 0.0) || !std::isfinite(d->n_atoms))
        return fail(ctx, HSD_ERR_INVALID_ARG, "need n_atoms > 0 and theta > 0");
    if (!d->cabs_host) return fail(ctx, HSD_ERR_INVALID_ARG, "null C_abs table");
    for (int j = 0; j < c.L; ++j)
        if (!(d->cabs_host[j] > 0.0) || !std::isfinite(d->cabs_host[j]))
            return fail(ctx, HSD_ERR_INVALID_ARG, "C_abs must be finite and > 0");
    if (!std::isfinite(d->longwave_index)) return fail(ctx, HSD_ERR_INVALID_ARG, "bad longwave index");
    HSD_HIP(ctx, hipSetDevice(c.device));
    Grain g;
    g.n_bins = n;
    g.E_lo = d->E_lo_erg;
    g.E_hi = d->E_hi_erg;
    g.n_atoms = d->n_atoms;
    g.theta = d->theta_debye_K;
    g.longwave = d->longwave_index;
    const size_t Lp = c.Lp;
    hipError_t e = hipSuccess;
    auto al = [&](auto*& p, size_t count) {
        if (e == hipSuccess) e = hipMalloc(&p, count * sizeof(*p));
    };
    al(g.E, n); al(g.dE, n); al(g.T, n); al(g.cool, n); al(g.colpar, n); al(g.dpar, n); al(g.gam, n);
    al(g.invgap, n); al(g.jstar, n); al(g.jrep, n); al(g.cabs, c.L); al(g.Bt, static_cast<size_t>(n) * Lp);
    al(g.bscale, Lp);
    if (e == hipSuccess) e = hipMemcpy(g.cabs, d->cabs_host, sizeof(double) * c.L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hsd::build_grain_tables(c, g);
    if (e != hipSuccess) {
        free_grain(g);
        return hip_fail(ctx, e, "hsd_add_grain");
    }
    c.grains.push_back(g);
    *grain_id = static_cast<int32_t>(c.grains.size() - 1);
    return HSD_OK;
}

hsd_status hsd_grain_tables(hsd_ctx* ctx, int32_t grain_id, double* E, double* dE, double* T, double* cool) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!grain_ok(ctx, grain_id)) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    const Grain& g = ctx->c.grains[grain_id];
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    const size_t b = sizeof(double) * g.n_bins;
    if (E) HSD_HIP(ctx, hipMemcpy(E, g.E, b, hipMemcpyDeviceToHost));
    if (dE) HSD_HIP(ctx, hipMemcpy(dE, g.dE, b, hipMemcpyDeviceToHost));
    if (T) HSD_HIP(ctx, hipMemcpy(T, g.T, b, hipMemcpyDeviceToHost));
    if (cool) HSD_HIP(ctx, hipMemcpy(cool, g.cool, b, hipMemcpyDeviceToHost));
    return HSD_OK;
}

hsd_status hsd_solve(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                     const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0 || n_grains == 0) return HSD_OK;
    if (!u_dev || !grain_ids_host || !j_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    return run_solve(ctx, n_cells, u_dev, n_grains, grain_ids_host, j_dev, diag_dev, nullptr,
                     static_cast<hipStream_t>(stream));
}

hsd_status hsd_solve_P(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t grain_id, double* P_dev,
                       void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0) return HSD_OK;
    if (!u_dev || !P_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    if (!grain_ok(ctx, grain_id)) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    return run_solve(ctx, n_cells, u_dev, 1, &grain_id, nullptr, nullptr, P_dev, static_cast<hipStream_t>(stream));
}

hsd_status hsd_solve_from_rates(hsd_ctx* ctx, int32_t n_bins, int32_t n_pairs, const double* A_dev,
                                const double* cool_dev, double* P_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_bins < 16 || n_bins > hsd::kMaxBins || n_bins % 16 != 0)
        return fail(ctx, HSD_ERR_INVALID_ARG, "n_bins must be a multiple of 16 in [16, 1024]");
    if (n_pairs < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_pairs == 0) return HSD_OK;
    if (!A_dev || !cool_dev || !P_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hsd::launch_from_rates(ctx->c, n_bins, n_pairs, A_dev, cool_dev, P_dev,
                                        static_cast<hipStream_t>(stream)));
    return HSD_OK;
}

hsd_status hsd_set_timing(hsd_ctx* ctx, int32_t enable) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    Ctx& c = ctx->c;
    HSD_HIP(ctx, hipSetDevice(c.device));
    if (enable && !c.ev[0])
        for (auto& e : c.ev) HSD_HIP(ctx, hipEventCreate(&e));
    c.timing = enable != 0;
    c.timed = false;
    return HSD_OK;
}

hsd_status hsd_phase_ms(hsd_ctx* ctx, double* ms) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!ms) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    Ctx& c = ctx->c;
    if (!c.timed) return fail(ctx, HSD_ERR_STATE, "no timed solve recorded");
    HSD_HIP(ctx, hipEventSynchronize(c.ev[3]));
    for (int i = 0; i < 3; ++i) {
        float t = 0.f;
        HSD_HIP(ctx, hipEventElapsedTime(&t, c.ev[i], c.ev[i + 1]));
        ms[i] = t;
    }
    return HSD_OK;
}

hsd_status hsd_sync(hsd_ctx* ctx) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    unsigned w = 0;
    HSD_HIP(ctx, hipMemcpy(&w, ctx->c.errword, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (w) {
        HSD_HIP(ctx, hipMemset(ctx->c.errword, 0, sizeof(unsigned)));
        return fail(ctx, HSD_ERR_NONFINITE_INPUT, "a field value was NaN, infinite or negative");
    }
    return HSD_OK;
}

}  // extern "C"
