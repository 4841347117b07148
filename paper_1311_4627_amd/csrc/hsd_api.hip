// C ABI entry points (include/hsd.h): argument checks, device memory of the
// context and its grains, and the order of kernel launches of a solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hsd_ckpt.h"
#include "hsd_internal.h"

using hsd::Ctx;
using hsd::Grain;

// Host-side description of one batch: per-slot grain views and row offsets in
// the scaled-P workspace, and the work items of each bin-count class.
struct Batch {
    std::vector<hsd::GrainView> views;
    std::vector<long long> offs;
    std::vector<int2> items;
    int cls_begin[hsd::kClasses + 1] = {0, 0, 0, 0, 0};
    long long rows = 0;
    std::vector<hsd::ContractSlot> cslots;   // the grouped contraction's slots (those with rows)
    int c_blocks = 0;                        // its workgroups
    // The same slots by bin-count class, each class's workgroups numbered from
    // 0 (a concurrent plan contracts a class's spectra on its own branch), and
    // the class the plan contracts last, after every branch has joined (the
    // one with the most solver work, which finishes last).
    std::vector<hsd::ContractSlot> cslots_cls;
    int ccls_begin[hsd::kClasses + 1] = {0, 0, 0, 0, 0};
    int ccls_blocks[hsd::kClasses] = {0, 0, 0, 0};
    int c_last = 0;
};

// The contraction slots of a batch whose slot g holds rows[g] P~ rows at
// offs[g] (list_off[g] >= 0: a pair list starting there in the row map).
void contract_slots(const Ctx& c, int32_t n_grains, const int32_t* ids, const std::vector<int>& rows,
                    const std::vector<int>& list_off, Batch& b) {
    b.cslots.clear();
    for (int g = 0; g < n_grains; ++g) {
        if (rows[g] <= 0) continue;
        const Grain& gr = c.grains[ids[g]];
        hsd::ContractSlot sl{};
        sl.pt_off = b.offs[g];
        sl.Bt = gr.Bt;
        sl.Bh = gr.Bh;
        sl.Bl = gr.Bl;
        sl.bscale = gr.bscale;
        sl.nb = gr.n_bins;
        sl.nbp = gr.nbp;
        sl.rows = rows[g];
        sl.gslot = g;
        sl.rowmap_off = list_off.empty() ? -1 : list_off[g];
        b.cslots.push_back(sl);
    }
    b.c_blocks = hsd::contract_blocks(b.cslots);
    b.cslots_cls.clear();
    double most = -1.0;
    for (int ci = 0; ci < hsd::kClasses; ++ci) {
        const int hi = hsd::kClassHi[ci];
        const int lo = ci + 1 < hsd::kClasses ? hsd::kClassHi[ci + 1] : 0;
        std::vector<hsd::ContractSlot> mine;
        double work = 0.0;
        for (const hsd::ContractSlot& sl : b.cslots)
            if (sl.nb > lo && sl.nb <= hi) {
                mine.push_back(sl);
                work += static_cast<double>(sl.rows) * sl.nb * sl.nb;   // rates grow as bins^2
            }
        b.ccls_begin[ci] = static_cast<int>(b.cslots_cls.size());
        b.ccls_blocks[ci] = hsd::contract_blocks(mine);
        b.cslots_cls.insert(b.cslots_cls.end(), mine.begin(), mine.end());
        if (!mine.empty() && work > most) {
            most = work;
            b.c_last = ci;
        }
    }
    b.ccls_begin[hsd::kClasses] = static_cast<int>(b.cslots_cls.size());
}

// Workspace of surrogate solves (grown on demand, kept with the context).
struct SurWork {
    float* bands = nullptr;       size_t bands_cap = 0;
    double* A = nullptr;          size_t A_cap = 0;
    float* emit = nullptr;        size_t emit_cap = 0;    // emitted-power partials [column slice][chunk]
    float* rho = nullptr;         size_t rho_cap = 0;     // predicted energy ratios [chunk]
    long long* fblist = nullptr;  size_t fblist_cap = 0;  // flagged pairs, in the order the check found them
    unsigned short* xb = nullptr; size_t xb_cap = 0;      // BF16 normalised inputs, hi and lo [chunk][96]
    unsigned short* h0 = nullptr; size_t h0_cap = 0;      // BF16 activations [chunk][512] (hi, lo)
    unsigned short* h1 = nullptr; size_t h1_cap = 0;
    int* sel = nullptr;           size_t sel_cap = 0;
    const double** cabs = nullptr; size_t cabs_cap = 0;
    float* loga = nullptr;        size_t loga_cap = 0;
    double* wcT = nullptr;        size_t wcT_cap = 0;     // [L][n_sel] absorption weights
    unsigned* cnt = nullptr;      size_t cnt_cap = 0;     // [n_grains + 1]: per-slot flagged, then total
    int* seg_off = nullptr;       size_t seg_off_cap = 0;
    int* seg_cnt = nullptr;       size_t seg_cnt_cap = 0;
    int* cellmap = nullptr;       size_t cellmap_cap = 0;
    long long* pairs = nullptr;   size_t pairs_cap = 0;
};

// Workspace of the table method (grown on demand).
struct TableWork {
    double* u = nullptr;          size_t u_cap = 0;       // node fields [K][L]
    float* j = nullptr;           size_t j_cap = 0;       // node spectra [K][G][L]
    double* A = nullptr;          size_t A_cap = 0;       // absorbed powers [rows][G]
    double* energy = nullptr;     size_t energy_cap = 0;  // field energies [cells], then the reference's
    const double** cabs = nullptr; size_t cabs_cap = 0;   // C_abs table of each listed grain
};

// Energy budget of the HSD_CHECK_TABLE check (hsd_set_energy_budget).
struct Budget {
    std::vector<int32_t> ids;                            // grains with a budget: row r of rho is ids[r]'s
    int K = 0;                                           // nodes (0: no budget set)
    double lo = 0.0, step = 0.0;                         // node grid in log10 U
    double* rho = nullptr;        size_t rho_cap = 0;    // [rows][K] emitted / absorbed power of the node spectra
    double* eref = nullptr;       size_t eref_cap = 0;   // [1] the reference field's energy
    int* row = nullptr;           size_t row_cap = 0;    // per slot of a call: its row of rho
    double* energy = nullptr;     size_t energy_cap = 0; // per cell of a call: the field's energy
    double* t = nullptr;          size_t t_cap = 0;      // per cell of a call: node-grid coordinate
};

struct hsd_ctx {
    Ctx c;
    Batch batch;     // host description of the last eager solve
    SurWork sw;
    TableWork tw;
    Budget bud;
};

struct hsd_sur {
    hsd_ctx* ctx = nullptr;
    hsd::Sur s;
};

// A batch bound to fixed buffers, captured once as a HIP graph.
struct hsd_plan {
    hsd_ctx* ctx = nullptr;
    int32_t n_cells = 0, n_grains = 0;
    std::vector<int32_t> ids;
    Batch b;
    float* Pt = nullptr;
    float* pscale = nullptr;
    hsd::GrainView* views = nullptr;
    long long* offs = nullptr;
    int2* items = nullptr;
    unsigned* queue = nullptr;
    hsd::ContractSlot* cslots = nullptr;
    hsd::ContractSlot* cslots_cls = nullptr;
    hipStream_t cap = nullptr;
    hipStream_t side[hsd::kClasses] = {};
    hipEvent_t sev[hsd::kClasses + 1] = {};
    hipEvent_t ev[4] = {};
    bool timing = false;
    bool launched = false;
    int n_graphs = 0;                 // 1, or 2 with timing (solver; contraction with the diagnostics)
    hipGraph_t graph[3] = {};
    hipGraphExec_t exec[3] = {};
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
    hipFree(g.bscale); hipFree(g.Bh); hipFree(g.Bl);
    g = Grain{};
}

bool grain_ok(const hsd_ctx* ctx, int32_t id) {
    return id >= 0 && static_cast<size_t>(id) < ctx->c.grains.size();
}

void plan_batch(const Ctx& c, int32_t n_cells, int32_t n_grains, const int32_t* ids, Batch& b) {
    b.views.resize(n_grains);
    b.offs.resize(n_grains);
    b.items.clear();
    b.rows = 0;
    for (int g = 0; g < n_grains; ++g) {
        const Grain& gr = c.grains[ids[g]];
        b.views[g] = hsd::GrainView{gr.colpar, gr.dpar, gr.gam, gr.invgap, gr.jstar, gr.jrep, gr.cabs,
                                    std::pow(gr.E_hi / gr.E_lo, 1.0 / (gr.n_bins - 1)), gr.n_bins, 0};
        b.offs[g] = b.rows;
        b.rows += static_cast<long long>(n_cells) * gr.n_bins;
    }
    for (int ci = 0; ci < hsd::kClasses; ++ci) {
        b.cls_begin[ci] = static_cast<int>(b.items.size());
        const int hi = hsd::kClassHi[ci];
        const int lo = ci + 1 < hsd::kClasses ? hsd::kClassHi[ci + 1] : 0;
        const int cpi = hsd::solve_cells_per_item(c.cfg[ci], ci);
        std::vector<int> slots;
        for (int g = 0; g < n_grains; ++g) {
            const int nb = c.grains[ids[g]].n_bins;
            if (nb > lo && nb <= hi) slots.push_back(g);
        }
        const int nsl = static_cast<int>(slots.size());
        if (nsl == 0) continue;
        const int ncb = (n_cells + cpi - 1) / cpi;
        if (c.cfg[ci].persistent) {
            // Atomic queue: items longest first (cost grows as bins^2), so the
            // last items dealt out are the cheapest and the tail is short; one
            // grain's cell blocks in a row.
            std::stable_sort(slots.begin(), slots.end(), [&](int x, int y) {
                return c.grains[ids[x]].n_bins > c.grains[ids[y]].n_bins;
            });
            for (int g : slots)
                for (int cb = 0; cb < ncb; ++cb) b.items.push_back(make_int2(g, cb * cpi));
        } else {
            // One item per workgroup.  Workgroups are dealt to the 8 XCDs
            // round-robin by id, so item k runs on XCD k % 8: give each XCD
            // whole cell blocks, all grains of a block in a row, so the block's
            // field rows are fetched into that XCD's L2 once for every grain
            // of the class.
            const int ncb8 = (ncb + 7) / 8 * 8;
            for (int k = 0; k < ncb8 * nsl; ++k) {
                const int x = k % 8, m = k / 8;
                const int cb = 8 * (m / nsl) + x;
                if (cb >= ncb) continue;
                b.items.push_back(make_int2(slots[m % nsl], cb * cpi));
            }
        }
    }
    b.cls_begin[hsd::kClasses] = static_cast<int>(b.items.size());
    contract_slots(c, n_grains, ids, std::vector<int>(n_grains, n_cells), {}, b);
}

// Batch of per-slot pair lists (counts[g] pairs of slot g, in list order;
// the list of slot g starts at list_off[g] in the row map).
void plan_batch_lists(const Ctx& c, const std::vector<int>& counts, const std::vector<int>& list_off,
                      int32_t n_grains, const int32_t* ids, Batch& b) {
    b.views.resize(n_grains);
    b.offs.resize(n_grains);
    b.items.clear();
    b.rows = 0;
    for (int g = 0; g < n_grains; ++g) {
        const Grain& gr = c.grains[ids[g]];
        b.views[g] = hsd::GrainView{gr.colpar, gr.dpar, gr.gam, gr.invgap, gr.jstar, gr.jrep, gr.cabs,
                                    std::pow(gr.E_hi / gr.E_lo, 1.0 / (gr.n_bins - 1)), gr.n_bins, 0};
        b.offs[g] = b.rows;
        b.rows += static_cast<long long>(counts[g]) * gr.n_bins;
    }
    for (int ci = 0; ci < hsd::kClasses; ++ci) {
        b.cls_begin[ci] = static_cast<int>(b.items.size());
        const int hi = hsd::kClassHi[ci];
        const int lo = ci + 1 < hsd::kClasses ? hsd::kClassHi[ci + 1] : 0;
        const int cpi = hsd::solve_cells_per_item(c.cfg[ci], ci);
        for (int g = 0; g < n_grains; ++g) {
            const int nb = c.grains[ids[g]].n_bins;
            if (nb <= lo || nb > hi) continue;
            for (int k0 = 0; k0 < counts[g]; k0 += cpi) b.items.push_back(make_int2(g, k0));
        }
    }
    b.cls_begin[hsd::kClasses] = static_cast<int>(b.items.size());
    contract_slots(c, n_grains, ids, counts, list_off, b);
}

// Device buffers one batch runs on (the context's workspace, or a plan's own).
struct Bufs {
    float* Pt;
    float* pscale;
    hsd::GrainView* views;
    long long* offs;
    int2* items;
    unsigned* queue;     // kClasses counters
    hsd::ContractSlot* cslots;
    hsd::ContractSlot* cslots_cls;   // by class (concurrent plans), or null
};

struct Events {
    hipEvent_t ev[4];    // phase boundaries, or null
};

hipError_t record(const Events& t, int i, hipStream_t s) {
    if (!t.ev[i]) return hipSuccess;
    return hipEventRecord(t.ev[i], s);
}

// Enqueue the whole batch on stream s: the solver classes (on the side
// streams, in parallel, when `side` is given), then the contraction of every
// grain's spectra, whose epilogue also writes the emitted power.  With side
// streams and the slots by class, each class except the last (b.c_last) is
// contracted on its own branch right after its solve, beside the solves
// still running (the contraction runs on the matrix cores, the solver on
// the vector ALUs), and the last class after the branches join; with phases,
// those early contractions belong to the solver phase.
constexpr int kPhaseSolve = 1, kPhaseContract = 2, kPhaseAll = 3;

hsd_status enqueue(hsd_ctx* ctx, const Batch& b, const Bufs& d, int32_t n_cells, const double* u, int32_t n_grains,
                   const int32_t* ids, float* j, float* diag, double* P64, hipStream_t s, const Events& t,
                   hipStream_t* side, hipEvent_t* sev, int phases = kPhaseAll) {
    Ctx& c = ctx->c;
    hsd::SolveLaunch sl{};
    sl.u = u;
    sl.n_cells = n_cells;
    sl.n_gslots = n_grains;
    sl.views = d.views;
    sl.offs = d.offs;
    sl.Pt = d.Pt;
    sl.pscale = d.pscale;
    sl.diag = diag;
    sl.P64 = P64;
    sl.errword = c.errword;
    const bool by_cls = side && d.cslots_cls && j;
    auto contract_class = [&](int ci, hipStream_t st) -> hsd_status {
        const int n_sl = b.ccls_begin[ci + 1] - b.ccls_begin[ci];
        if (n_sl == 0) return HSD_OK;
        hsd::ContractLaunch cl{d.cslots_cls + b.ccls_begin[ci], n_sl, b.ccls_blocks[ci], d.Pt, d.pscale, nullptr,
                               j, diag, c.wtrap, c.L, c.Lp, n_grains, c.contract, c.contract_waves};
        HSD_HIP(ctx, hsd::launch_contract(cl, st));
        return HSD_OK;
    };
    HSD_HIP(ctx, record(t, 0, s));
    if (!(phases & kPhaseSolve)) {
    } else if (side) {
        HSD_HIP(ctx, hipEventRecord(sev[0], s));
        for (int ci = 0; ci < hsd::kClasses; ++ci) {
            const int n_it = b.cls_begin[ci + 1] - b.cls_begin[ci];
            if (n_it == 0) continue;
            HSD_HIP(ctx, hipStreamWaitEvent(side[ci], sev[0], 0));
            HSD_HIP(ctx, hsd::launch_solve(c, sl, ci, d.items + b.cls_begin[ci], n_it, d.queue + ci, side[ci]));
            if (by_cls && ci != b.c_last) {
                const hsd_status st = contract_class(ci, side[ci]);
                if (st != HSD_OK) return st;
            }
            HSD_HIP(ctx, hipEventRecord(sev[1 + ci], side[ci]));
            HSD_HIP(ctx, hipStreamWaitEvent(s, sev[1 + ci], 0));
        }
    } else {
        for (int ci = 0; ci < hsd::kClasses; ++ci) {
            const int n_it = b.cls_begin[ci + 1] - b.cls_begin[ci];
            if (n_it == 0) continue;
            HSD_HIP(ctx, hsd::launch_solve(c, sl, ci, d.items + b.cls_begin[ci], n_it, d.queue + ci, s));
        }
    }
    HSD_HIP(ctx, record(t, 1, s));
    if (by_cls && (phases & kPhaseContract)) {
        const hsd_status st = contract_class(b.c_last, s);
        if (st != HSD_OK) return st;
    } else if (j && (phases & kPhaseContract)) {
        // every grain in one launch; its epilogue also writes the emitted
        // power (diag entry 1), so the diagnostics phase has no work left
        hsd::ContractLaunch cl{d.cslots, static_cast<int>(b.cslots.size()), b.c_blocks, d.Pt, d.pscale, nullptr,
                               j, diag, c.wtrap, c.L, c.Lp, n_grains, c.contract, c.contract_waves};
        HSD_HIP(ctx, hsd::launch_contract(cl, s));
    }
    HSD_HIP(ctx, record(t, 2, s));
    HSD_HIP(ctx, record(t, 3, s));
    return HSD_OK;
}

// Copy the batch's host description into the device buffers d and enqueue
// its launches (eager solves: hsd_solve, hsd_solve_P, hsd_solve_noalloc).
hsd_status run_batch(hsd_ctx* ctx, const Bufs& d, int32_t n_cells, const double* u, int32_t n_grains,
                     const int32_t* ids, float* j, float* diag, double* P64, hipStream_t s, bool branches = false) {
    Ctx& c = ctx->c;
    const Batch& b = ctx->batch;
    if (branches && d.cslots_cls && !b.cslots_cls.empty())
        HSD_HIP(ctx, hipMemcpyAsync(d.cslots_cls, b.cslots_cls.data(), sizeof(hsd::ContractSlot) * b.cslots_cls.size(),
                                    hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(d.views, b.views.data(), sizeof(hsd::GrainView) * n_grains,
                                hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(d.offs, b.offs.data(), sizeof(long long) * n_grains, hipMemcpyHostToDevice, s));
    if (!b.items.empty())
        HSD_HIP(ctx, hipMemcpyAsync(d.items, b.items.data(), sizeof(int2) * b.items.size(),
                                    hipMemcpyHostToDevice, s));
    if (!b.cslots.empty())
        HSD_HIP(ctx, hipMemcpyAsync(d.cslots, b.cslots.data(), sizeof(hsd::ContractSlot) * b.cslots.size(),
                                    hipMemcpyHostToDevice, s));
    Events t{{nullptr, nullptr, nullptr, nullptr}};
    if (c.timing)
        for (int i = 0; i < 4; ++i) t.ev[i] = c.ev[i];
    hsd_status st = enqueue(ctx, b, d, n_cells, u, n_grains, ids, j, diag, P64, s, t, branches ? c.side : nullptr,
                            branches ? c.sev : nullptr);
    if (st == HSD_OK && c.timing) c.timed = true;
    return st;
}

// Whether eager solves run their classes as concurrent branches: yes unless
// a class is configured persistent (its grid takes every workgroup slot);
// the branch streams and events are made on first use, at the default
// priority.
bool side_streams(hsd_ctx* ctx) {
    Ctx& c = ctx->c;
    for (int ci = 0; ci < hsd::kClasses; ++ci)
        if (c.cfg[ci].persistent) return false;
    if (c.sev[hsd::kClasses]) return true;
    for (int i = 0; i < hsd::kClasses; ++i)
        if (!c.side[i] && hipStreamCreateWithFlags(&c.side[i], hipStreamNonBlocking) != hipSuccess) return false;
    for (int i = 0; i <= hsd::kClasses; ++i)
        if (!c.sev[i] && hipEventCreateWithFlags(&c.sev[i], hipEventDisableTiming) != hipSuccess) {
            c.sev[i] = nullptr;       // made again on the next call; the others are kept
            return false;
        }
    return true;
}

// Eager solve on the context's workspace (hsd_solve and hsd_solve_P).
hsd_status run_solve(hsd_ctx* ctx, int32_t n_cells, const double* u, int32_t n_grains, const int32_t* ids,
                     float* j, float* diag, double* P64, hipStream_t s, bool keep_pt = false) {
    Ctx& c = ctx->c;
    Batch& b = ctx->batch;
    plan_batch(c, n_cells, n_grains, ids, b);
    const bool want_pt = keep_pt || (j != nullptr) || (diag != nullptr);
    if (want_pt) HSD_HIP(ctx, grow(c.Pt, c.Pt_cap, static_cast<size_t>(b.rows)));
    HSD_HIP(ctx, grow(c.pscale, c.pscale_cap, static_cast<size_t>(n_cells) * n_grains));
    HSD_HIP(ctx, grow(c.views, c.views_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(c.offs, c.offs_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(c.items, c.items_cap, std::max<size_t>(b.items.size(), 1)));
    HSD_HIP(ctx, grow(c.cslots, c.cslots_cap, std::max<size_t>(b.cslots.size(), 1)));
    const bool branches = side_streams(ctx);
    if (branches) HSD_HIP(ctx, grow(c.cslots_cls, c.cslots_cls_cap, std::max<size_t>(b.cslots_cls.size(), 1)));
    Bufs d{want_pt ? c.Pt : nullptr, c.pscale, c.views, c.offs, c.items, c.queue, c.cslots,
           branches ? c.cslots_cls : nullptr};
    return run_batch(ctx, d, n_cells, u, n_grains, ids, j, diag, P64, s, branches);
}

// ---- fixed device scratch for hsd_solve_noalloc ----
// The whole workspace of one solve (grain views, row offsets, work items,
// per-pair scales and the scaled-P rows) carved out of one file-scope device
// array, so that the call allocates nothing.  Each device holds its own copy
// of the array; host code uses only its device address (from
// hipGetSymbolAddress, looked up once per device when a context is created),
// never the array's name.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The device address of `scratch` on the current device `dev` (looked up on
// the first call per device).
hipError_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

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
    void* scr = nullptr;
    if (scratch_address(device, &scr) != hipSuccess) return HSD_ERR_HIP;
    hsd_ctx* ctx = new (std::nothrow) hsd_ctx();
    if (!ctx) return HSD_ERR_OOM;
    Ctx& c = ctx->c;
    c.device = device;
    c.scratch = static_cast<unsigned char*>(scr);
    c.L = n_lambda;
    c.Lp = (n_lambda + 63) / 64 * 64;
    c.lnlam0 = ln0;
    c.dlnlam = dl;
    c.lam_host.assign(lambda_host, lambda_host + n_lambda);
    std::vector<double> wt(n_lambda, 0.0);       // 4 pi x trapezoid weights of the grid
    for (int i = 0; i + 1 < n_lambda; ++i) {
        const double h = 0.5 * (lambda_host[i + 1] - lambda_host[i]);
        wt[i] += h;
        wt[i + 1] += h;
    }
    for (double& x : wt) x *= 4.0 * hsd::kPi;
    if (hipMalloc(&c.wtrap, sizeof(double) * n_lambda) != hipSuccess ||
        hipMemcpy(c.wtrap, wt.data(), sizeof(double) * n_lambda, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(c.wtrap);
        delete ctx;
        return HSD_ERR_OOM;
    }
    if (hipMalloc(&c.lam, sizeof(double) * n_lambda) != hipSuccess ||
        hipMalloc(&c.errword, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&c.queue, sizeof(unsigned) * hsd::kClasses) != hipSuccess) {
        hipFree(c.lam);
        hipFree(c.errword);
        hipFree(c.queue);
        hipFree(c.wtrap);
        delete ctx;
        return HSD_ERR_OOM;
    }
    if (hipMemcpy(c.lam, lambda_host, sizeof(double) * n_lambda, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c.errword, 0, sizeof(unsigned)) != hipSuccess ||
        hipMemset(c.queue, 0, sizeof(unsigned) * hsd::kClasses) != hipSuccess) {
        hipFree(c.lam);
        hipFree(c.errword);
        hipFree(c.queue);
        hipFree(c.wtrap);
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
    hipFree(c.wtrap);
    hipFree(c.errword);
    hipFree(c.queue);
    hipFree(c.sizew);
    hipFree(c.cslots);
    SurWork& w = ctx->sw;
    hipFree(w.bands); hipFree(w.A); hipFree(w.emit); hipFree(w.rho); hipFree(w.fblist); hipFree(w.h0); hipFree(w.h1);
    hipFree(w.xb); hipFree(w.wcT);
    hipFree(w.sel); hipFree(w.cabs); hipFree(w.loga); hipFree(w.cnt); hipFree(w.seg_off); hipFree(w.seg_cnt);
    hipFree(w.cellmap); hipFree(w.pairs);
    TableWork& tw = ctx->tw;
    hipFree(tw.u); hipFree(tw.j); hipFree(tw.A); hipFree(tw.energy); hipFree(tw.cabs);
    Budget& bd = ctx->bud;
    hipFree(bd.rho); hipFree(bd.eref); hipFree(bd.row); hipFree(bd.energy); hipFree(bd.t);
    hipFree(c.Pt);
    hipFree(c.pscale);
    hipFree(c.diag_tmp);
    hipFree(c.views);
    hipFree(c.offs);
    hipFree(c.items);
    hipFree(c.cslots_cls);
    for (auto& e : c.ev)
        if (e) hipEventDestroy(e);
    for (auto& e : c.sev)
        if (e) hipEventDestroy(e);
    for (auto& st : c.side)
        if (st) hipStreamDestroy(st);
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
    g.radius = d->radius_cm;
    const size_t Lp = c.Lp;
    hipError_t e = hipSuccess;
    auto al = [&](auto*& p, size_t count) {
        if (e == hipSuccess) e = hipMalloc(&p, count * sizeof(*p));
    };
    al(g.E, n); al(g.dE, n); al(g.T, n); al(g.cool, n); al(g.colpar, n); al(g.dpar, n); al(g.gam, n);
    al(g.invgap, n); al(g.jstar, n); al(g.jrep, n); al(g.cabs, c.L); al(g.Bt, static_cast<size_t>(n) * Lp);
    al(g.bscale, Lp);
    g.nbp = (n + 63) / 64 * 64;
    al(g.Bh, Lp * static_cast<size_t>(g.nbp)); al(g.Bl, Lp * static_cast<size_t>(g.nbp));
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

hsd_status hsd_solve_noalloc(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                             const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0 || n_grains == 0) return HSD_OK;
    if (!u_dev || !grain_ids_host || !j_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    Batch& b = ctx->batch;
    plan_batch(c, n_cells, n_grains, grain_ids_host, b);
    // scratch layout: views | offs | items | contraction slots | pscale | P~ rows, each 256-byte aligned
    const size_t o_views = 0;
    const size_t o_offs = o_views + align256(sizeof(hsd::GrainView) * n_grains);
    const size_t o_items = o_offs + align256(sizeof(long long) * n_grains);
    const size_t o_cslots = o_items + align256(sizeof(int2) * std::max<size_t>(b.items.size(), 1));
    const size_t o_pscale = o_cslots + align256(sizeof(hsd::ContractSlot) * std::max<size_t>(b.cslots.size(), 1));
    const size_t o_pt = o_pscale + align256(sizeof(float) * static_cast<size_t>(n_cells) * n_grains);
    const size_t need = o_pt + sizeof(float) * static_cast<size_t>(b.rows);
    if (need > kScratchBytes)
        return fail(ctx, HSD_ERR_INVALID_ARG,
                    "hsd_solve_noalloc: the batch needs " + std::to_string(need) + " bytes of scratch, more than its " +
                        std::to_string(kScratchBytes) + " (use hsd_solve, or fewer cells per call)");
    HSD_HIP(ctx, hipSetDevice(c.device));
    unsigned char* base = c.scratch;
    Bufs d{reinterpret_cast<float*>(base + o_pt), reinterpret_cast<float*>(base + o_pscale),
           reinterpret_cast<hsd::GrainView*>(base + o_views), reinterpret_cast<long long*>(base + o_offs),
           reinterpret_cast<int2*>(base + o_items), c.queue, reinterpret_cast<hsd::ContractSlot*>(base + o_cslots),
           nullptr};
    return run_batch(ctx, d, n_cells, u_dev, n_grains, grain_ids_host, j_dev, diag_dev, nullptr,
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

hsd_status hsd_get_class_cfg(hsd_ctx* ctx, int32_t cls, hsd_class_cfg* out) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!out || cls < 0 || cls >= hsd::kClasses) return fail(ctx, HSD_ERR_INVALID_ARG, "bad class or null output");
    const hsd::ClassCfg& k = ctx->c.cfg[cls];
    out->kg = k.kg;
    out->wide = k.wide;
    out->persistent = k.persistent;
    return HSD_OK;
}

hsd_status hsd_set_class_cfg(hsd_ctx* ctx, int32_t cls, const hsd_class_cfg* cfg) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!cfg || cls < 0 || cls >= hsd::kClasses) return fail(ctx, HSD_ERR_INVALID_ARG, "bad class or null config");
    if (cfg->kg != 2 && cfg->kg != 4) return fail(ctx, HSD_ERR_INVALID_ARG, "kg must be 2 or 4");
    if (cfg->wide != 0 && (cfg->wide != 1 || !hsd::class_has_wide(cls)))
        return fail(ctx, HSD_ERR_INVALID_ARG, "wide is 0 or 1, and 1 only for classes 0, 1 and 3");
    if (cfg->persistent != 0 && cfg->persistent != 1) return fail(ctx, HSD_ERR_INVALID_ARG, "persistent is 0 or 1");
    hsd::ClassCfg& k = ctx->c.cfg[cls];
    k.kg = cfg->kg;
    k.wide = cfg->wide;
    k.persistent = cfg->persistent;
    return HSD_OK;
}

hsd_status hsd_set_contract(hsd_ctx* ctx, int32_t mode) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (mode != HSD_CONTRACT_FP32 && mode != HSD_CONTRACT_BF16X3)
        return fail(ctx, HSD_ERR_INVALID_ARG, "mode must be HSD_CONTRACT_FP32 or HSD_CONTRACT_BF16X3");
    ctx->c.contract = mode;
    return HSD_OK;
}

hsd_status hsd_get_contract(hsd_ctx* ctx, int32_t* mode) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!mode) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    *mode = ctx->c.contract;
    return HSD_OK;
}

hsd_status hsd_set_contract_waves(hsd_ctx* ctx, int32_t waves) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (waves != 4 && waves != 8) return fail(ctx, HSD_ERR_INVALID_ARG, "contraction waves must be 4 or 8");
    ctx->c.contract_waves = waves;
    return HSD_OK;
}

hsd_status hsd_get_contract_waves(hsd_ctx* ctx, int32_t* waves) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!waves) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    *waves = ctx->c.contract_waves;
    return HSD_OK;
}

hsd_status hsd_autotune(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                        const int32_t* grain_ids_host, int32_t runs, hsd_tune_record* records_host,
                        int32_t max_records, int32_t* n_records) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells <= 0 || n_grains <= 0 || runs < 2) return fail(ctx, HSD_ERR_INVALID_ARG, "need n_cells, n_grains > 0 and runs >= 2");
    if (!u_dev || !grain_ids_host || !n_records || (max_records > 0 && !records_host))
        return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    HSD_HIP(ctx, hipSetDevice(c.device));
    *n_records = 0;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hsd_status st = HSD_OK;
    hipError_t he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const bool was_timing = c.timing;
    c.timing = false;
    for (int ci = 0; ci < hsd::kClasses && he == hipSuccess && st == HSD_OK; ++ci) {
        const int hi = hsd::kClassHi[ci];
        const int lo = ci + 1 < hsd::kClasses ? hsd::kClassHi[ci + 1] : 0;
        std::vector<int32_t> ids;
        for (int g = 0; g < n_grains; ++g) {
            const int nb = c.grains[grain_ids_host[g]].n_bins;
            if (nb > lo && nb <= hi) ids.push_back(grain_ids_host[g]);
        }
        if (ids.empty()) continue;
        const hsd::ClassCfg keep = c.cfg[ci];
        hsd::ClassCfg best = keep;
        double best_ms = 1e300;
        for (int wide = 0; wide <= (hsd::class_has_wide(ci) ? 1 : 0) && st == HSD_OK; ++wide)
            for (int pers = 0; pers <= 1 && st == HSD_OK; ++pers)
                for (int kg = 2; kg <= 4 && st == HSD_OK; kg += 2) {
                    c.cfg[ci] = hsd::ClassCfg{kg, wide, pers};
                    double sum = 0.0;
                    for (int r = 0; r < runs && he == hipSuccess && st == HSD_OK; ++r) {
                        he = hipEventRecord(e0, s);
                        if (he != hipSuccess) break;
                        st = run_solve(ctx, n_cells, u_dev, static_cast<int32_t>(ids.size()), ids.data(), nullptr,
                                       nullptr, nullptr, s, true);
                        if (st != HSD_OK) break;
                        he = hipEventRecord(e1, s);
                        if (he == hipSuccess) he = hipEventSynchronize(e1);
                        float ms = 0.f;
                        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                        if (r > 0) sum += ms;      // the first run is a warm-up
                    }
                    if (he != hipSuccess || st != HSD_OK) break;
                    const double mean = sum / (runs - 1);
                    if (*n_records < max_records) {
                        hsd_tune_record& rec = records_host[*n_records];
                        rec.cls = ci;
                        rec.cfg = hsd_class_cfg{kg, wide, pers};
                        rec.contract_waves = c.contract_waves;
                        rec.n_grains = static_cast<int32_t>(ids.size());
                        rec.ms = mean;
                    }
                    ++*n_records;
                    if (mean < best_ms) {
                        best_ms = mean;
                        best = c.cfg[ci];
                    }
                }
        c.cfg[ci] = (he == hipSuccess && st == HSD_OK) ? best : keep;
    }
    c.timing = was_timing;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    if (st != HSD_OK) return st;
    if (he != hipSuccess) return hip_fail(ctx, he, "hsd_autotune");
    return HSD_OK;
}

hsd_status hsd_autotune_plan(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                             const int32_t* grain_ids_host, int32_t runs, hsd_tune_record* records_host,
                             int32_t max_records, int32_t* n_records) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells <= 0 || n_grains <= 0 || runs < 2) return fail(ctx, HSD_ERR_INVALID_ARG, "need n_cells, n_grains > 0 and runs >= 2");
    if (!u_dev || !grain_ids_host || !n_records || (max_records > 0 && !records_host))
        return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    HSD_HIP(ctx, hipSetDevice(c.device));
    *n_records = 0;
    // classes the batch occupies, and their grain counts
    int cls_grains[hsd::kClasses] = {};
    for (int g = 0; g < n_grains; ++g) {
        const int nb = c.grains[grain_ids_host[g]].n_bins;
        for (int ci = 0; ci < hsd::kClasses; ++ci) {
            const int lo = ci + 1 < hsd::kClasses ? hsd::kClassHi[ci + 1] : 0;
            if (nb > lo && nb <= hsd::kClassHi[ci]) ++cls_grains[ci];
        }
    }
    const size_t jn = static_cast<size_t>(n_cells) * n_grains * c.L;
    float* j = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipMalloc(&j, sizeof(float) * jn);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    hsd_status st = HSD_OK;
    hsd::ClassCfg keep[hsd::kClasses];
    for (int ci = 0; ci < hsd::kClasses; ++ci) keep[ci] = c.cfg[ci];
    const int keep_waves = c.contract_waves;
    // one candidate: a concurrent plan of the batch (solver classes as
    // parallel branches, then the contraction), replayed `runs` times; the
    // first replay is a warm-up and the mean of the others is the score
    auto time_plan = [&](int cls, double& ms) -> bool {
        hsd_plan* p = nullptr;
        st = hsd_plan_create(ctx, n_cells, u_dev, n_grains, grain_ids_host, j, nullptr, HSD_PLAN_CONCURRENT, &p);
        if (st != HSD_OK) return false;
        double sum = 0.0;
        for (int r = 0; r < runs && he == hipSuccess && st == HSD_OK; ++r) {
            he = hipEventRecord(e0, s);
            if (he != hipSuccess) break;
            st = hsd_plan_launch(p, s);
            if (st != HSD_OK) break;
            he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float t = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
            if (r > 0) sum += t;
        }
        hsd_plan_destroy(p);
        if (he != hipSuccess || st != HSD_OK) return false;
        ms = sum / (runs - 1);
        if (*n_records < max_records) {
            hsd_tune_record& rec = records_host[*n_records];
            rec.cls = cls;
            rec.cfg = cls >= 0 ? hsd_class_cfg{c.cfg[cls].kg, c.cfg[cls].wide, c.cfg[cls].persistent}
                               : hsd_class_cfg{0, 0, 0};
            rec.contract_waves = c.contract_waves;
            rec.n_grains = cls >= 0 ? cls_grains[cls] : n_grains;
            rec.ms = ms;
        }
        ++*n_records;
        return true;
    };
    // start from the current configuration as ordinary grids (a concurrent
    // plan takes no persistent class), then one class at a time, the largest
    // first, try each alternative with the others fixed and keep what is
    // faster; the contraction's workgroup size last
    for (int ci = 0; ci < hsd::kClasses; ++ci) c.cfg[ci].persistent = 0;
    double best = 0.0;
    bool ok = he == hipSuccess && time_plan(-1, best);
    for (int ci = 0; ci < hsd::kClasses && ok; ++ci) {
        if (cls_grains[ci] == 0) continue;
        const hsd::ClassCfg cur = c.cfg[ci];
        hsd::ClassCfg win = cur;
        for (int wide = 0; wide <= (hsd::class_has_wide(ci) ? 1 : 0) && ok; ++wide)
            for (int kg = 2; kg <= 4 && ok; kg += 2) {
                if (wide == cur.wide && kg == cur.kg) continue;
                c.cfg[ci] = hsd::ClassCfg{kg, wide, 0};
                double ms = 0.0;
                ok = time_plan(ci, ms);
                if (ok && ms < best) {
                    best = ms;
                    win = c.cfg[ci];
                }
            }
        c.cfg[ci] = win;
    }
    if (ok && c.contract == HSD_CONTRACT_BF16X3) {
        const int cur = c.contract_waves;
        c.contract_waves = cur == 4 ? 8 : 4;
        double ms = 0.0;
        ok = time_plan(-1, ms);
        if (!(ok && ms < best)) c.contract_waves = cur;
    }
    if (!ok) {
        for (int ci = 0; ci < hsd::kClasses; ++ci) c.cfg[ci] = keep[ci];
        c.contract_waves = keep_waves;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    if (j) hipFree(j);
    if (st != HSD_OK) return st;
    if (he != hipSuccess) return hip_fail(ctx, he, "hsd_autotune_plan");
    return HSD_OK;
}

void hsd_plan_destroy(hsd_plan* p) {
    if (!p) return;
    hipSetDevice(p->ctx->c.device);
    hipDeviceSynchronize();
    for (int i = 0; i < 3; ++i) {
        if (p->exec[i]) hipGraphExecDestroy(p->exec[i]);
        if (p->graph[i]) hipGraphDestroy(p->graph[i]);
    }
    for (auto& e : p->ev)
        if (e) hipEventDestroy(e);
    for (auto& e : p->sev)
        if (e) hipEventDestroy(e);
    for (auto& st : p->side)
        if (st) hipStreamDestroy(st);
    if (p->cap) hipStreamDestroy(p->cap);
    hipFree(p->Pt);
    hipFree(p->pscale);
    hipFree(p->views);
    hipFree(p->offs);
    hipFree(p->items);
    hipFree(p->cslots_cls);
    hipFree(p->queue);
    hipFree(p->cslots);
    delete p;
}

hsd_status hsd_plan_create(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                           const int32_t* grain_ids_host, float* j_dev, float* diag_dev, int32_t flags,
                           hsd_plan** out) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!out) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    if (n_cells <= 0 || n_grains <= 0) return fail(ctx, HSD_ERR_INVALID_ARG, "a plan needs n_cells > 0 and n_grains > 0");
    if (!u_dev || !grain_ids_host || !j_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    if (flags & ~(HSD_PLAN_TIMING | HSD_PLAN_CONCURRENT)) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown flag");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    if (flags & HSD_PLAN_CONCURRENT) {
        // a persistent grid takes every workgroup slot of the device and would
        // hold the other branches off it: the two do not combine
        for (int ci = 0; ci < hsd::kClasses; ++ci)
            if (c.cfg[ci].persistent)
                return fail(ctx, HSD_ERR_INVALID_ARG,
                            "HSD_PLAN_CONCURRENT needs every class configured with persistent = 0");
    }
    HSD_HIP(ctx, hipSetDevice(c.device));
    hsd_plan* p = new (std::nothrow) hsd_plan();
    if (!p) return fail(ctx, HSD_ERR_OOM, "host allocation");
    p->ctx = ctx;
    p->n_cells = n_cells;
    p->n_grains = n_grains;
    p->ids.assign(grain_ids_host, grain_ids_host + n_grains);
    p->timing = (flags & HSD_PLAN_TIMING) != 0;
    const bool conc = (flags & HSD_PLAN_CONCURRENT) != 0;
    plan_batch(c, n_cells, n_grains, p->ids.data(), p->b);
    hipError_t e = hipSuccess;
    auto al = [&](auto*& ptr, size_t count) {
        if (e == hipSuccess) e = hipMalloc(&ptr, std::max<size_t>(count, 1) * sizeof(*ptr));
    };
    al(p->Pt, static_cast<size_t>(p->b.rows));
    al(p->pscale, static_cast<size_t>(n_cells) * n_grains);
    al(p->views, static_cast<size_t>(n_grains));
    al(p->offs, static_cast<size_t>(n_grains));
    al(p->items, p->b.items.size());
    al(p->queue, static_cast<size_t>(hsd::kClasses));
    al(p->cslots, p->b.cslots.size());
    if (conc) al(p->cslots_cls, p->b.cslots_cls.size());
    if (e == hipSuccess)
        e = hipMemcpy(p->views, p->b.views.data(), sizeof(hsd::GrainView) * n_grains, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->offs, p->b.offs.data(), sizeof(long long) * n_grains, hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->b.items.empty())
        e = hipMemcpy(p->items, p->b.items.data(), sizeof(int2) * p->b.items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->b.cslots.empty())
        e = hipMemcpy(p->cslots, p->b.cslots.data(), sizeof(hsd::ContractSlot) * p->b.cslots.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && conc && !p->b.cslots_cls.empty())
        e = hipMemcpy(p->cslots_cls, p->b.cslots_cls.data(), sizeof(hsd::ContractSlot) * p->b.cslots_cls.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->queue, 0, sizeof(unsigned) * hsd::kClasses);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    for (int i = 0; conc && i < hsd::kClasses && e == hipSuccess; ++i)
        e = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking);
    for (int i = 0; conc && i <= hsd::kClasses && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&p->sev[i], hipEventDisableTiming);
    for (int i = 0; p->timing && i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&p->ev[i]);
    // persistent grid sizes come from occupancy queries: make them before the capture
    for (int ci = 0; ci < hsd::kClasses && e == hipSuccess; ++ci)
        if (c.cfg[ci].persistent && hsd::solve_capacity(c, ci) <= 0) e = hipErrorInvalidValue;
    if (e != hipSuccess) {
        hsd_plan_destroy(p);
        return hip_fail(ctx, e, "hsd_plan_create");
    }
    Bufs d{p->Pt, p->pscale, p->views, p->offs, p->items, p->queue, p->cslots, conc ? p->cslots_cls : nullptr};
    const Events none{{nullptr, nullptr, nullptr, nullptr}};
    // Without timing the whole batch is one graph.  With timing, the solver
    // and the contraction (whose epilogue writes the diagnostics) are graphs
    // of their own and the launch records the phase events between them on
    // the caller's stream.
    static const int whole[1] = {kPhaseAll};
    static const int split[2] = {kPhaseSolve, kPhaseContract};
    p->n_graphs = p->timing ? 2 : 1;
    for (int gi = 0; gi < p->n_graphs; ++gi) {
        e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            hsd_plan_destroy(p);
            return hip_fail(ctx, e, "hipStreamBeginCapture");
        }
        const int phases = p->timing ? split[gi] : whole[0];
        const hsd_status st = enqueue(ctx, p->b, d, n_cells, u_dev, n_grains, p->ids.data(), j_dev, diag_dev,
                                      nullptr, p->cap, none, conc ? p->side : nullptr, p->sev, phases);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->cap, &g);
        p->graph[gi] = g;
        if (st != HSD_OK) {
            hsd_plan_destroy(p);
            return st;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec[gi], p->graph[gi], nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hsd_plan_destroy(p);
            return hip_fail(ctx, e, "graph capture");
        }
    }
    *out = p;
    return HSD_OK;
}

hsd_status hsd_plan_launch(hsd_plan* p, void* stream) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    if (p->timing) {
        for (int gi = 0; gi < 2; ++gi) {
            HSD_HIP(ctx, hipEventRecord(p->ev[gi], s));
            HSD_HIP(ctx, hipGraphLaunch(p->exec[gi], s));
        }
        HSD_HIP(ctx, hipEventRecord(p->ev[2], s));
        HSD_HIP(ctx, hipEventRecord(p->ev[3], s));     // the diagnostics run inside the contraction
    } else {
        HSD_HIP(ctx, hipGraphLaunch(p->exec[0], s));
    }
    p->launched = true;
    return HSD_OK;
}

hsd_status hsd_plan_phase_ms(hsd_plan* p, double* ms) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!ms) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    if (!p->timing || !p->launched) return fail(ctx, HSD_ERR_STATE, "plan made without timing, or never launched");
    HSD_HIP(ctx, hipEventSynchronize(p->ev[3]));
    for (int i = 0; i < 3; ++i) {
        float t = 0.f;
        HSD_HIP(ctx, hipEventElapsedTime(&t, p->ev[i], p->ev[i + 1]));
        ms[i] = t;
    }
    return HSD_OK;
}

hsd_status hsd_size_convolve(hsd_ctx* ctx, int32_t n_cells, int32_t n_grains, const float* j_dev,
                             const double* weights_host, int32_t flags, double* out_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (flags & ~(HSD_SIZE_LAMBDA | HSD_SIZE_EV)) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown flag");
    if (n_cells == 0) return HSD_OK;
    if (!j_dev || !out_dev || (n_grains > 0 && !weights_host)) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!std::isfinite(weights_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "non-finite weight");
    Ctx& c = ctx->c;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    HSD_HIP(ctx, hipStreamSynchronize(s));          // the weight buffer may still be read by earlier work
    HSD_HIP(ctx, grow(c.sizew, c.sizew_cap, static_cast<size_t>(std::max(n_grains, 1))));
    if (n_grains > 0)
        HSD_HIP(ctx, hipMemcpy(c.sizew, weights_host, sizeof(double) * n_grains, hipMemcpyHostToDevice));
    HSD_HIP(ctx, hsd::launch_sizedist(j_dev, c.sizew, c.lam, n_cells, n_grains, c.L, flags, out_dev, s));
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

namespace {

// C_abs tables of the listed grains, on the device, for the energy kernel.
hsd_status table_cabs(hsd_ctx* ctx, int32_t n_grains, const int32_t* ids, hipStream_t s) {
    TableWork& tw = ctx->tw;
    std::vector<const double*> p(n_grains);
    for (int g = 0; g < n_grains; ++g) p[g] = ctx->c.grains[ids[g]].cabs;
    HSD_HIP(ctx, grow(tw.cabs, tw.cabs_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, hipMemcpyAsync(tw.cabs, p.data(), sizeof(double*) * n_grains, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipStreamSynchronize(s));      // the host vector goes out of scope
    return HSD_OK;
}

hsd_status table_args(hsd_ctx* ctx, int32_t n_grains, const int32_t* ids, int32_t n_nodes, double lo, double hi) {
    if (n_grains <= 0 || !ids) return fail(ctx, HSD_ERR_INVALID_ARG, "need n_grains > 0 and grain ids");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, ids[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    if (n_nodes < 2 || n_nodes > 4096) return fail(ctx, HSD_ERR_INVALID_ARG, "need 2 <= n_nodes <= 4096");
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
        return fail(ctx, HSD_ERR_INVALID_ARG, "need finite log10U_lo < log10U_hi");
    return HSD_OK;
}

}  // namespace

hsd_status hsd_table_build(hsd_ctx* ctx, int32_t n_grains, const int32_t* grain_ids_host, const double* u_ref_dev,
                           int32_t n_nodes, double log10U_lo, double log10U_hi, float* table_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    hsd_status st = table_args(ctx, n_grains, grain_ids_host, n_nodes, log10U_lo, log10U_hi);
    if (st != HSD_OK) return st;
    if (!u_ref_dev || !table_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    Ctx& c = ctx->c;
    TableWork& tw = ctx->tw;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    const size_t K = static_cast<size_t>(n_nodes), G = static_cast<size_t>(n_grains);
    HSD_HIP(ctx, grow(tw.u, tw.u_cap, K * c.L));
    HSD_HIP(ctx, grow(tw.j, tw.j_cap, K * G * c.L));
    HSD_HIP(ctx, grow(tw.A, tw.A_cap, K * G));
    st = table_cabs(ctx, n_grains, grain_ids_host, s);
    if (st != HSD_OK) return st;
    const double step = (log10U_hi - log10U_lo) / (n_nodes - 1);
    HSD_HIP(ctx, hsd::launch_node_fields(u_ref_dev, log10U_lo, step, n_nodes, c.L, tw.u, s));
    st = run_solve(ctx, n_nodes, tw.u, n_grains, grain_ids_host, tw.j, nullptr, nullptr, s);
    if (st != HSD_OK) return st;
    HSD_HIP(ctx, hsd::launch_cell_energies(tw.u, c.lam, n_nodes, c.L, n_grains, tw.cabs, nullptr, tw.A, s));
    HSD_HIP(ctx, hsd::launch_table_logs(tw.j, tw.A, n_nodes, n_grains, c.L, table_dev, s));
    return HSD_OK;
}

hsd_status hsd_table_eval(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                          const int32_t* grain_ids_host, const double* u_ref_dev, int32_t n_nodes, double log10U_lo,
                          double log10U_hi, const float* table_dev, float* j_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    hsd_status st = table_args(ctx, n_grains, grain_ids_host, n_nodes, log10U_lo, log10U_hi);
    if (st != HSD_OK) return st;
    if (n_cells == 0) return HSD_OK;
    if (!u_dev || !u_ref_dev || !table_dev || !j_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    Ctx& c = ctx->c;
    TableWork& tw = ctx->tw;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    const size_t G = static_cast<size_t>(n_grains);
    HSD_HIP(ctx, grow(tw.A, tw.A_cap, static_cast<size_t>(n_cells) * G));
    HSD_HIP(ctx, grow(tw.energy, tw.energy_cap, static_cast<size_t>(n_cells) + 1));
    st = table_cabs(ctx, n_grains, grain_ids_host, s);
    if (st != HSD_OK) return st;
    HSD_HIP(ctx, hsd::launch_cell_energies(u_dev, c.lam, n_cells, c.L, n_grains, tw.cabs, tw.energy, tw.A, s));
    HSD_HIP(ctx, hsd::launch_cell_energies(u_ref_dev, c.lam, 1, c.L, 0, tw.cabs, tw.energy + n_cells, nullptr, s));
    const double step = (log10U_hi - log10U_lo) / (n_nodes - 1);
    HSD_HIP(ctx, hsd::launch_table_eval(tw.energy, tw.energy + n_cells, tw.A, table_dev, n_nodes, log10U_lo, step,
                                        n_cells, n_grains, c.L, j_dev, s));
    return HSD_OK;
}

hsd_status hsd_set_energy_budget(hsd_ctx* ctx, int32_t n_grains, const int32_t* grain_ids_host,
                                 const double* u_ref_dev, int32_t n_nodes, double log10U_lo, double log10U_hi,
                                 const float* table_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    hsd_status st = table_args(ctx, n_grains, grain_ids_host, n_nodes, log10U_lo, log10U_hi);
    if (st != HSD_OK) return st;
    if (!u_ref_dev || !table_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int a = 0; a < n_grains; ++a)
        for (int b = 0; b < a; ++b)
            if (grain_ids_host[a] == grain_ids_host[b]) return fail(ctx, HSD_ERR_INVALID_ARG, "repeated grain id");
    Ctx& c = ctx->c;
    Budget& bd = ctx->bud;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    bd.K = 0;                                   // no budget until this one is complete
    HSD_HIP(ctx, grow(bd.rho, bd.rho_cap, static_cast<size_t>(n_grains) * n_nodes));
    HSD_HIP(ctx, grow(bd.eref, bd.eref_cap, 1));
    HSD_HIP(ctx, hsd::launch_budget_nodes(table_dev, n_nodes, n_grains, c.L, c.lam, bd.rho, s));
    HSD_HIP(ctx, hsd::launch_cell_energies(u_ref_dev, c.lam, 1, c.L, 0, nullptr, bd.eref, nullptr, s));
    HSD_HIP(ctx, hipStreamSynchronize(s));
    bd.ids.assign(grain_ids_host, grain_ids_host + n_grains);
    bd.lo = log10U_lo;
    bd.step = (log10U_hi - log10U_lo) / (n_nodes - 1);
    bd.K = n_nodes;
    return HSD_OK;
}

hsd_status hsd_measure_exp2(hsd_ctx* ctx, double* per_second_host) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!per_second_host) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hsd::measure_exp2(per_second_host));
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

// ---- learned surrogate ----

hsd_status hsd_sur_create(hsd_ctx* ctx, hsd_sur** out) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (!out) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    hsd_sur* p = new (std::nothrow) hsd_sur();
    if (!p) return fail(ctx, HSD_ERR_OOM, "host allocation");
    p->ctx = ctx;
    p->s.c = &ctx->c;
    p->s.L = ctx->c.L;
    p->s.n_out = ctx->c.L + 1;
    p->s.widths[4] = p->s.n_out;
    const hipError_t e = hsd::sur_alloc(p->s);
    if (e != hipSuccess) {
        hsd::sur_free(p->s);
        delete p;
        return hip_fail(ctx, e, "hsd_sur_create");
    }
    *out = p;
    return HSD_OK;
}

void hsd_sur_destroy(hsd_sur* p) {
    if (!p) return;
    hipSetDevice(p->ctx->c.device);
    hipDeviceSynchronize();
    hsd::sur_free(p->s);
    delete p;
}

hsd_status hsd_sur_n_params(hsd_sur* p, int64_t* n) {
    if (!p) return HSD_ERR_INVALID_ARG;
    if (!n) return fail(p->ctx, HSD_ERR_INVALID_ARG, "null output");
    *n = p->s.n_params;
    return HSD_OK;
}

hsd_status hsd_sur_set_params(hsd_sur* p, const float* params_host) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!params_host) return fail(ctx, HSD_ERR_INVALID_ARG, "null parameters");
    for (long long i = 0; i < p->s.n_params; ++i)
        if (!std::isfinite(params_host[i])) return fail(ctx, HSD_ERR_INVALID_ARG, "non-finite parameter");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipMemcpy(p->s.w, params_host, sizeof(float) * p->s.n_params, hipMemcpyHostToDevice));
    HSD_HIP(ctx, hipMemset(p->s.m, 0, sizeof(float) * p->s.n_params));
    HSD_HIP(ctx, hipMemset(p->s.v, 0, sizeof(float) * p->s.n_params));
    p->s.t = 0;
    p->s.wb_fresh = false;
    return HSD_OK;
}

hsd_status hsd_sur_get_params(hsd_sur* p, float* params_host) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!params_host) return fail(ctx, HSD_ERR_INVALID_ARG, "null output");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    HSD_HIP(ctx, hipMemcpy(params_host, p->s.w, sizeof(float) * p->s.n_params, hipMemcpyDeviceToHost));
    return HSD_OK;
}

hsd_status hsd_sur_set_loss(hsd_sur* p, float band_weight) {
    if (!p) return HSD_ERR_INVALID_ARG;
    if (!(band_weight >= 0.f && band_weight <= 1.f)) return fail(p->ctx, HSD_ERR_INVALID_ARG, "band_weight must be in [0, 1]");
    p->s.band_weight = band_weight;
    return HSD_OK;
}

hsd_status hsd_sur_set_norm(hsd_sur* p, const double* x_mean, const double* x_std, const double* y_mean,
                            const double* y_std) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!x_mean || !x_std || !y_mean || !y_std) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    const int L = p->s.n_out;
    std::vector<float> a(33), b(33), c(L), d(L);
    for (int k = 0; k < 33; ++k) {
        if (!(x_std[k] > 0.0) || !std::isfinite(x_mean[k])) return fail(ctx, HSD_ERR_INVALID_ARG, "bad input statistics");
        a[k] = static_cast<float>(x_mean[k]);
        b[k] = static_cast<float>(x_std[k]);
    }
    for (int k = 0; k < L; ++k) {
        if (!(y_std[k] > 0.0) || !std::isfinite(y_mean[k])) return fail(ctx, HSD_ERR_INVALID_ARG, "bad target statistics");
        c[k] = static_cast<float>(y_mean[k]);
        d[k] = static_cast<float>(y_std[k]);
    }
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipMemcpy(p->s.xm, a.data(), sizeof(float) * 33, hipMemcpyHostToDevice));
    HSD_HIP(ctx, hipMemcpy(p->s.xs, b.data(), sizeof(float) * 33, hipMemcpyHostToDevice));
    HSD_HIP(ctx, hipMemcpy(p->s.ym, c.data(), sizeof(float) * L, hipMemcpyHostToDevice));
    HSD_HIP(ctx, hipMemcpy(p->s.ys, d.data(), sizeof(float) * L, hipMemcpyHostToDevice));
    p->s.have_norm = true;
    return HSD_OK;
}

hsd_status hsd_sur_get_norm(hsd_sur* p, double* x_mean, double* x_std, double* y_mean, double* y_std) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!x_mean || !x_std || !y_mean || !y_std) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    if (!p->s.have_norm) return fail(ctx, HSD_ERR_STATE, "no statistics set");
    const int L = p->s.n_out;
    std::vector<float> a(33), b(33), c(L), d(L);
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipMemcpy(a.data(), p->s.xm, sizeof(float) * 33, hipMemcpyDeviceToHost));
    HSD_HIP(ctx, hipMemcpy(b.data(), p->s.xs, sizeof(float) * 33, hipMemcpyDeviceToHost));
    HSD_HIP(ctx, hipMemcpy(c.data(), p->s.ym, sizeof(float) * L, hipMemcpyDeviceToHost));
    HSD_HIP(ctx, hipMemcpy(d.data(), p->s.ys, sizeof(float) * L, hipMemcpyDeviceToHost));
    for (int k = 0; k < 33; ++k) {
        x_mean[k] = a[k];
        x_std[k] = b[k];
    }
    for (int k = 0; k < L; ++k) {
        y_mean[k] = c[k];
        y_std[k] = d[k];
    }
    return HSD_OK;
}

}  // extern "C"

// ---- checkpoint files of a network ----

namespace {

bool host_is_little_endian() {
    const uint32_t one = 1;
    unsigned char b[4];
    std::memcpy(b, &one, 4);
    return b[0] == 1;
}

struct SurSection {
    const char* name;
    float* dev;
    long long n;
};

std::vector<SurSection> sur_sections(hsd::Sur& s, bool optimizer) {
    std::vector<SurSection> v = {{"params", s.w, s.n_params}, {"x_mean", s.xm, 33}, {"x_std", s.xs, 33},
                                 {"y_mean", s.ym, s.n_out}, {"y_std", s.ys, s.n_out}};
    if (optimizer) {
        v.push_back({"adam_m", s.m, s.n_params});
        v.push_back({"adam_v", s.v, s.n_params});
    }
    return v;
}

}  // namespace

extern "C" {

hsd_status hsd_surrogate_save(hsd_sur* p, const char* path, int32_t flags) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!path) return fail(ctx, HSD_ERR_INVALID_ARG, "null path");
    if (flags & ~HSD_SAVE_WEIGHTS_ONLY) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown flag");
    if (!host_is_little_endian()) return fail(ctx, HSD_ERR_STATE, "checkpoints are written on little-endian hosts only");
    hsd::Sur& s = p->s;
    if (!s.have_norm) return fail(ctx, HSD_ERR_STATE, "surrogate has no input/target statistics");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    const bool opt = (flags & HSD_SAVE_WEIGHTS_ONLY) == 0;
    const std::vector<SurSection> secs = sur_sections(s, opt);
    std::string h = "{\"format\": \"hsd-surrogate\", \"widths\": [";
    for (int i = 0; i < 5; ++i) h += std::to_string(s.widths[i]) + (i < 4 ? ", " : "]");
    char bw[32];
    std::snprintf(bw, sizeof(bw), "%.9g", static_cast<double>(s.band_weight));
    h += ", \"n_params\": " + std::to_string(s.n_params) + ", \"step\": " + std::to_string(s.t) +
         ", \"loss_band_weight\": " + bw +
         ", \"optimizer\": " + (opt ? "true" : "false") + ", \"byte_order\": \"little\", \"sections\": [";
    for (size_t i = 0; i < secs.size(); ++i)
        h += std::string(i ? ", " : "") + "{\"name\": \"" + secs[i].name + "\", \"dtype\": \"f32\", \"count\": " +
             std::to_string(secs[i].n) + "}";
    h += "]}";
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(ctx, HSD_ERR_INVALID_ARG, std::string("cannot open for writing: ") + path);
    bool ok = std::fputs("HSDSUR 1\n", f) >= 0 && std::fputs(h.c_str(), f) >= 0 && std::fputc('\n', f) != EOF;
    std::vector<float> buf;
    for (const SurSection& sec : secs) {
        if (!ok) break;
        buf.resize(static_cast<size_t>(sec.n));
        const hipError_t e = hipMemcpy(buf.data(), sec.dev, sizeof(float) * sec.n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            std::fclose(f);
            return hip_fail(ctx, e, "hsd_surrogate_save");
        }
        ok = std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(ctx, HSD_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return HSD_OK;
}

hsd_status hsd_surrogate_load(hsd_sur* p, const char* path) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (!path) return fail(ctx, HSD_ERR_INVALID_ARG, "null path");
    if (!host_is_little_endian()) return fail(ctx, HSD_ERR_STATE, "checkpoints are read on little-endian hosts only");
    hsd::Sur& s = p->s;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ctx, HSD_ERR_INVALID_ARG, std::string("cannot open: ") + path);
    std::string data;
    char chunk[65536];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) data.append(chunk, got);
    const bool read_err = std::ferror(f) != 0;
    std::fclose(f);
    if (read_err) return fail(ctx, HSD_ERR_INVALID_ARG, std::string("read failed: ") + path);
    hsd::CkptHeader hd;
    const std::string why = hsd::ckpt_parse(data, s.widths, s.n_params, hd);
    if (!why.empty()) return fail(ctx, HSD_ERR_INVALID_ARG, why);
    const bool opt = hd.optimizer;
    const long long step = hd.step;
    const double bw = hd.band_weight;
    const std::vector<SurSection> secs = sur_sections(s, opt);
    std::vector<std::vector<float>> host(secs.size());
    size_t off = hd.payload_off;
    for (size_t i = 0; i < secs.size(); ++i) {
        host[i].resize(static_cast<size_t>(secs[i].n));
        std::memcpy(host[i].data(), data.data() + off, sizeof(float) * secs[i].n);
        off += sizeof(float) * secs[i].n;
        for (float v : host[i])
            if (!std::isfinite(v)) return fail(ctx, HSD_ERR_INVALID_ARG, std::string("non-finite value in ") + secs[i].name);
    }
    for (int k : {2, 4})
        for (float v : host[k])
            if (!(v > 0.f)) return fail(ctx, HSD_ERR_INVALID_ARG, "standard deviations must be > 0");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    for (size_t i = 0; i < secs.size(); ++i)
        HSD_HIP(ctx, hipMemcpy(secs[i].dev, host[i].data(), sizeof(float) * secs[i].n, hipMemcpyHostToDevice));
    if (!opt) {
        HSD_HIP(ctx, hipMemset(s.m, 0, sizeof(float) * s.n_params));
        HSD_HIP(ctx, hipMemset(s.v, 0, sizeof(float) * s.n_params));
    }
    s.t = opt ? step : 0;
    s.band_weight = static_cast<float>(bw);
    s.have_norm = true;
    s.wb_fresh = false;
    return HSD_OK;
}

}  // extern "C"

namespace {

// Per-slot tables of the selected grains for the feature kernels.
hsd_status sur_select(hsd_ctx* ctx, const std::vector<int>& slots, const int32_t* ids, hipStream_t s) {
    Ctx& c = ctx->c;
    SurWork& w = ctx->sw;
    const size_t n = slots.size();
    std::vector<const double*> cabs(n);
    std::vector<float> loga(n);
    for (size_t k = 0; k < n; ++k) {
        const Grain& g = c.grains[ids[slots[k]]];
        if (!(g.radius > 0.0)) return fail(ctx, HSD_ERR_INVALID_ARG, "the surrogate needs grains with radius_cm > 0");
        cabs[k] = g.cabs;
        loga[k] = static_cast<float>(std::log10(g.radius));
    }
    HSD_HIP(ctx, grow(w.sel, w.sel_cap, n));
    HSD_HIP(ctx, grow(w.cabs, w.cabs_cap, n));
    HSD_HIP(ctx, grow(w.loga, w.loga_cap, n));
    HSD_HIP(ctx, hipMemcpyAsync(w.sel, slots.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(w.cabs, cabs.data(), sizeof(double*) * n, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(w.loga, loga.data(), sizeof(float) * n, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, grow(w.wcT, w.wcT_cap, n * c.L));
    HSD_HIP(ctx, hsd::sur_wc(c, w.cabs, static_cast<int>(n), w.wcT, s));
    HSD_HIP(ctx, hipStreamSynchronize(s));      // host vectors go out of scope
    return HSD_OK;
}

constexpr long long kSurChunk = 1048576;  // pair rows per inference chunk (fewer, longer launches; 1.7 GB of activations)

// Surrogate spectra of every (cell, slot) pair of `slots` into j, with diag
// entries and the energy-balance flags (bit 4, check HSD_CHECK_*) counted in
// sw.cnt.
hsd_status sur_run(hsd_ctx* ctx, hsd::Sur& sur, int32_t n_cells, const double* u, int32_t n_grains,
                   const int32_t* ids, const std::vector<int>& slots, float tol, int check, float* j, float* diag,
                   long long* list, long long list_cap, hipStream_t s) {
    Ctx& c = ctx->c;
    SurWork& w = ctx->sw;
    if (!sur.have_norm) return fail(ctx, HSD_ERR_STATE, "surrogate has no input/target statistics");
    const hsd_status st = sur_select(ctx, slots, ids, s);
    if (st != HSD_OK) return st;
    const int n_sel = static_cast<int>(slots.size());
    const long long rows = static_cast<long long>(n_cells) * n_sel;
    const size_t ch = static_cast<size_t>(std::min(rows, kSurChunk));
    HSD_HIP(ctx, grow(w.A, w.A_cap, ch));
    const int n_parts = hsd::sur_emit_parts(sur.n_out);
    HSD_HIP(ctx, grow(w.emit, w.emit_cap, ch * n_parts));
    HSD_HIP(ctx, grow(w.rho, w.rho_cap, ch));
    HSD_HIP(ctx, grow(w.xb, w.xb_cap, ch * 96));
    HSD_HIP(ctx, grow(w.h0, w.h0_cap, ch * 512));
    HSD_HIP(ctx, grow(w.h1, w.h1_cap, ch * 256));
    for (long long r0 = 0; r0 < rows; r0 += kSurChunk) {
        const long long n = std::min(kSurChunk, rows - r0);
        HSD_HIP(ctx, hsd::sur_pairs(c, u, w.bands, w.wcT, w.loga, r0, n, n_sel, nullptr, w.A, w.xb, sur.xm, sur.xs,
                                    s));
        HSD_HIP(ctx, hsd::sur_infer_rows(sur, static_cast<int>(n), w.xb, w.A, r0, n_sel, n_grains, w.sel, j, w.emit,
                                         w.rho, w.h0, w.h1, s));
        if (diag) {
            const Budget& bd = ctx->bud;
            const bool tab = check == HSD_CHECK_TABLE;
            HSD_HIP(ctx, hsd::sur_diag(w.A, w.emit, n_parts, check == HSD_CHECK_MODEL ? w.rho : nullptr,
                                       tab ? bd.rho : nullptr, bd.row, bd.K, bd.t, r0, n, n_sel, n_grains, w.sel, tol,
                                       diag, w.cnt, list, list_cap, s));
        }
    }
    return HSD_OK;
}

}  // namespace

extern "C" {

hsd_status hsd_sur_features(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                            const int32_t* grain_ids_host, float* X_dev, double* A_dev, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0 || n_grains == 0) return HSD_OK;
    if (!u_dev || !grain_ids_host || (!X_dev && !A_dev)) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    std::vector<int> slots(n_grains);
    for (int g = 0; g < n_grains; ++g) slots[g] = g;
    const hsd_status st = sur_select(ctx, slots, grain_ids_host, s);
    if (st != HSD_OK) return st;
    SurWork& w = ctx->sw;
    HSD_HIP(ctx, grow(w.bands, w.bands_cap, static_cast<size_t>(n_cells) * 32));
    HSD_HIP(ctx, hsd::sur_bands(c, u_dev, n_cells, w.bands, s));
    HSD_HIP(ctx, hsd::sur_pairs(c, u_dev, w.bands, w.wcT, w.loga, 0, static_cast<long long>(n_cells) * n_grains,
                                n_grains, X_dev, A_dev, nullptr, nullptr, nullptr, s));
    return HSD_OK;
}

hsd_status hsd_sur_targets(hsd_ctx* ctx, int64_t n, const float* j_dev, const double* A_dev, float* Y_dev,
                           void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n == 0) return HSD_OK;
    if (!j_dev || !A_dev || !Y_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hsd::sur_targets(j_dev, A_dev, ctx->c.lam, n, ctx->c.L, Y_dev, static_cast<hipStream_t>(stream)));
    return HSD_OK;
}

hsd_status hsd_sur_fit_norm(hsd_sur* p, int64_t n, const float* X_dev, const float* Y_dev) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (n <= 0 || !X_dev || !Y_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "need n > 0 and both arrays");
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hipDeviceSynchronize());
    std::vector<double> xm, xs, ym, ys;
    HSD_HIP(ctx, hsd::sur_colstats(X_dev, n, 33, xm, xs));
    HSD_HIP(ctx, hsd::sur_colstats(Y_dev, n, p->s.n_out, ym, ys));
    // spectrum targets: one pooled standard deviation for every wavelength;
    // the energy-ratio target: kRatioScale times its own (a smaller weight in
    // the loss, so that the ratio does not take the spectrum's capacity)
    const int L = p->s.L;
    double pooled = 0.0;
    for (int k = 0; k < L; ++k) pooled += ys[k] * ys[k];
    pooled = std::sqrt(pooled / L);
    if (!(pooled > 0.0)) pooled = 1.0;
    std::fill(ys.begin(), ys.begin() + L, pooled);
    ys[L] *= hsd::kRatioScale;
    return hsd_sur_set_norm(p, xm.data(), xs.data(), ym.data(), ys.data());
}

hsd_status hsd_sur_loss_grad(hsd_sur* p, int32_t n, const float* X_dev, const float* Y_dev, double* loss_host,
                             float* grad_host) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (n <= 0 || n > 65536 || !X_dev || !Y_dev || !loss_host)
        return fail(ctx, HSD_ERR_INVALID_ARG, "need 0 < n <= 65536 and non-null arrays");
    if (!p->s.have_norm) return fail(ctx, HSD_ERR_STATE, "surrogate has no input/target statistics");
    hsd::Sur& s = p->s;
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    const hipStream_t st = nullptr;
    HSD_HIP(ctx, hsd::sur_grow(s, n));
    HSD_HIP(ctx, hsd::sur_seq_idx(s, 0, n, st));
    HSD_HIP(ctx, hsd::sur_gather(s, X_dev, Y_dev, n, st));
    HSD_HIP(ctx, hsd::sur_forward(s, n, s.Xb, st, true));
    HSD_HIP(ctx, hsd::sur_loss(s, n, st));
    HSD_HIP(ctx, hsd::sur_backward(s, n, s.Xb, st));
    HSD_HIP(ctx, hipDeviceSynchronize());
    double l = 0.0;
    HSD_HIP(ctx, hipMemcpy(&l, s.loss, sizeof(double), hipMemcpyDeviceToHost));
    *loss_host = l / (static_cast<double>(n) * s.n_out);
    if (grad_host) HSD_HIP(ctx, hipMemcpy(grad_host, s.g, sizeof(float) * s.n_params, hipMemcpyDeviceToHost));
    return HSD_OK;
}

hsd_status hsd_sur_train(hsd_sur* p, int64_t n, const float* X_dev, const float* Y_dev, int32_t steps, int32_t batch,
                         float lr, uint64_t seed, float* loss_host) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (n <= 0 || !X_dev || !Y_dev || steps < 0 || batch <= 0 || batch > 65536 || !(lr > 0.f))
        return fail(ctx, HSD_ERR_INVALID_ARG, "need n > 0, steps >= 0, 0 < batch <= 65536, lr > 0");
    if (!p->s.have_norm) return fail(ctx, HSD_ERR_STATE, "surrogate has no input/target statistics");
    hsd::Sur& s = p->s;
    HSD_HIP(ctx, hipSetDevice(ctx->c.device));
    HSD_HIP(ctx, hsd::sur_grow(s, batch));
    if (steps == 0) return HSD_OK;
    HSD_HIP(ctx, hipDeviceSynchronize());          // the inputs may come from any stream
    const int warm = std::max(1, steps / 50);
    // the trained parameters are the moving average of the iterates (decay
    // min(0.999, 1 - 20 / steps)), which smooths the last steps' noise
    const float ema_decay = static_cast<float>(std::min(0.999, 1.0 - 20.0 / std::max(steps, 1)));
    const bool ema = ema_decay > 0.f;
    // step sizes of every step: linear warm-up, then cosine decay to 5% of lr,
    // with Adam's bias corrections of steps t0 + 1 .. t0 + steps
    const long long t0 = s.t;
    std::vector<float2> sched(steps);
    std::vector<float> lr_k(steps);
    for (int k = 0; k < steps; ++k) {
        double f = 1.0;
        if (k < warm) f = static_cast<double>(k + 1) / warm;
        else f = 0.05 + 0.95 * 0.5 * (1.0 + std::cos(hsd::kPi * (k - warm) / std::max(1, steps - warm)));
        lr_k[k] = static_cast<float>(lr * f);
        sched[k] = hsd::adam_step_sizes(lr_k[k], t0 + k + 1);
    }
    double* trace = nullptr;
    long long* ctr = nullptr;
    float2* dsched = nullptr;
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess && loss_host) e = hipMalloc(&trace, sizeof(double) * steps);
    if (e == hipSuccess && ema) e = hipMemcpyAsync(s.we, s.w, sizeof(float) * s.n_params, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && s.train_graph) {
        // One step captured once and replayed: its per-step values (the
        // minibatch counter, the step sizes) live in device memory, so every
        // replay runs exactly the launches of an eager step.
        e = hipMalloc(&ctr, sizeof(long long));
        if (e == hipSuccess) e = hipMalloc(&dsched, sizeof(float2) * steps);
        if (e == hipSuccess) e = hipMemcpyAsync(ctr, &t0, sizeof(long long), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dsched, sched.data(), sizeof(float2) * steps, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ce = hsd::sur_batch_idx(s, seed, 0, batch, n, st, ctr);
            if (ce == hipSuccess) ce = hsd::sur_gather(s, X_dev, Y_dev, batch, st);
            if (ce == hipSuccess) ce = hsd::sur_forward(s, batch, s.Xb, st, true);
            if (ce == hipSuccess) ce = hsd::sur_loss(s, batch, st);
            if (ce == hipSuccess) ce = hsd::sur_backward(s, batch, s.Xb, st);
            if (ce == hipSuccess) ce = hsd::sur_adam_sched(s, dsched, ctr, t0, st, ema, ema_decay);
            if (ce == hipSuccess) ce = hsd::sur_step_end(ctr, t0, s.loss, trace, st);
            e = hipStreamEndCapture(st, &graph);
            if (e == hipSuccess) e = ce;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (int k = 0; k < steps && e == hipSuccess; ++k) e = hipGraphLaunch(exec, st);
        if (e == hipSuccess) {
            s.t = t0 + steps;
            s.wb_fresh = false;
        }
    } else {
        for (int k = 0; k < steps && e == hipSuccess; ++k) {
            e = hsd::sur_batch_idx(s, seed, s.t, batch, n, st);
            if (e == hipSuccess) e = hsd::sur_gather(s, X_dev, Y_dev, batch, st);
            if (e == hipSuccess) e = hsd::sur_forward(s, batch, s.Xb, st, true);
            if (e == hipSuccess) e = hsd::sur_loss(s, batch, st);
            if (e == hipSuccess && trace)
                e = hipMemcpyAsync(trace + k, s.loss, sizeof(double), hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hsd::sur_backward(s, batch, s.Xb, st);
            if (e == hipSuccess) e = hsd::sur_adam(s, lr_k[k], st, ema, ema_decay);
        }
    }
    if (e == hipSuccess && ema) {
        e = hipMemcpyAsync(s.w, s.we, sizeof(float) * s.n_params, hipMemcpyDeviceToDevice, st);
        s.wb_fresh = false;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && trace) {
        std::vector<double> h(steps);
        e = hipMemcpy(h.data(), trace, sizeof(double) * steps, hipMemcpyDeviceToHost);
        for (int k = 0; k < steps; ++k) loss_host[k] = static_cast<float>(h[k] / (static_cast<double>(batch) * s.n_out));
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (st) (void)hipStreamDestroy(st);
    if (trace) (void)hipFree(trace);
    if (ctr) (void)hipFree(ctr);
    if (dsched) (void)hipFree(dsched);
    if (e != hipSuccess) return hip_fail(ctx, e, "hsd_sur_train");
    return HSD_OK;
}

hsd_status hsd_sur_set_train_graph(hsd_sur* p, int32_t enable) {
    if (!p) return HSD_ERR_INVALID_ARG;
    p->s.train_graph = enable != 0;
    return HSD_OK;
}

hsd_status hsd_sur_predict(hsd_sur* p, int32_t n_cells, const double* u_dev, int32_t n_grains,
                           const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream) {
    if (!p) return HSD_ERR_INVALID_ARG;
    hsd_ctx* ctx = p->ctx;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0 || n_grains == 0) return HSD_OK;
    if (!u_dev || !grain_ids_host || !j_dev) return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    for (int g = 0; g < n_grains; ++g)
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
    Ctx& c = ctx->c;
    SurWork& w = ctx->sw;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    HSD_HIP(ctx, grow(w.bands, w.bands_cap, static_cast<size_t>(n_cells) * 32));
    HSD_HIP(ctx, grow(w.cnt, w.cnt_cap, static_cast<size_t>(n_grains) + 1));
    HSD_HIP(ctx, hipMemsetAsync(w.cnt, 0, sizeof(unsigned) * (n_grains + 1), s));
    HSD_HIP(ctx, hsd::sur_bands(c, u_dev, n_cells, w.bands, s));
    std::vector<int> slots(n_grains);
    for (int g = 0; g < n_grains; ++g) slots[g] = g;
    return sur_run(ctx, p->s, n_cells, u_dev, n_grains, grain_ids_host, slots, 0.01f, HSD_CHECK_MODEL, j_dev,
                   diag_dev, nullptr, 0, s);
}

hsd_status hsd_solve_surrogate(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                               const int32_t* grain_ids_host, hsd_sur* const* surs_host, float tol, int32_t check,
                               float* j_dev, float* diag_dev, int64_t* n_fallback_host, void* stream) {
    if (!ctx) return HSD_ERR_INVALID_ARG;
    if (n_cells < 0 || n_grains < 0) return fail(ctx, HSD_ERR_INVALID_ARG, "negative size");
    if (!n_fallback_host) return fail(ctx, HSD_ERR_INVALID_ARG, "null fallback count");
    *n_fallback_host = 0;
    if (n_cells == 0 || n_grains == 0) return HSD_OK;
    if (!u_dev || !grain_ids_host || !surs_host || !j_dev || !diag_dev)
        return fail(ctx, HSD_ERR_INVALID_ARG, "null pointer");
    if (!(tol >= 0.f)) return fail(ctx, HSD_ERR_INVALID_ARG, "tol must be >= 0");
    if (check != HSD_CHECK_ABSORBED && check != HSD_CHECK_MODEL && check != HSD_CHECK_TABLE)
        return fail(ctx, HSD_ERR_INVALID_ARG, "check must be HSD_CHECK_ABSORBED, HSD_CHECK_MODEL or HSD_CHECK_TABLE");
    for (int g = 0; g < n_grains; ++g) {
        if (!grain_ok(ctx, grain_ids_host[g])) return fail(ctx, HSD_ERR_INVALID_ARG, "unknown grain id");
        if (!surs_host[g] || surs_host[g]->ctx != ctx) return fail(ctx, HSD_ERR_INVALID_ARG, "missing or foreign surrogate");
    }
    Budget& bd = ctx->bud;
    std::vector<int> rows;
    if (check == HSD_CHECK_TABLE) {
        if (bd.K == 0) return fail(ctx, HSD_ERR_STATE, "HSD_CHECK_TABLE needs hsd_set_energy_budget first");
        for (int g = 0; g < n_grains; ++g) {
            const auto it = std::find(bd.ids.begin(), bd.ids.end(), grain_ids_host[g]);
            if (it == bd.ids.end()) return fail(ctx, HSD_ERR_STATE, "a grain of the batch has no energy budget");
            rows.push_back(static_cast<int>(it - bd.ids.begin()));
        }
    }
    Ctx& c = ctx->c;
    SurWork& w = ctx->sw;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HSD_HIP(ctx, hipSetDevice(c.device));
    if (check == HSD_CHECK_TABLE) {
        // each cell's position on the budget's node grid, each slot's row of it
        HSD_HIP(ctx, grow(bd.row, bd.row_cap, static_cast<size_t>(n_grains)));
        HSD_HIP(ctx, grow(bd.energy, bd.energy_cap, static_cast<size_t>(n_cells)));
        HSD_HIP(ctx, grow(bd.t, bd.t_cap, static_cast<size_t>(n_cells)));
        HSD_HIP(ctx, hipMemcpyAsync(bd.row, rows.data(), sizeof(int) * n_grains, hipMemcpyHostToDevice, s));
        HSD_HIP(ctx, hsd::launch_cell_energies(u_dev, c.lam, n_cells, c.L, 0, nullptr, bd.energy, nullptr, s));
        HSD_HIP(ctx, hsd::launch_node_coord(bd.energy, bd.eref, n_cells, bd.lo, bd.step, bd.K, bd.t, s));
    }
    HSD_HIP(ctx, grow(w.bands, w.bands_cap, static_cast<size_t>(n_cells) * 32));
    HSD_HIP(ctx, grow(w.cnt, w.cnt_cap, static_cast<size_t>(n_grains) + 1));
    HSD_HIP(ctx, hipMemsetAsync(w.cnt, 0, sizeof(unsigned) * (n_grains + 1), s));
    HSD_HIP(ctx, hsd::sur_bands(c, u_dev, n_cells, w.bands, s));
    // flagged pairs are listed by the check, up to an eighth of the pairs (at
    // least 2^20); beyond that the fallback scans every pair's flags
    const long long n_pairs = static_cast<long long>(n_cells) * n_grains;
    const long long list_cap = std::min(n_pairs, std::max(1LL << 20, n_pairs / 8));
    HSD_HIP(ctx, grow(w.fblist, w.fblist_cap, static_cast<size_t>(list_cap)));
    // one pass per network over the grains it serves
    std::vector<hsd_sur*> nets;
    for (int g = 0; g < n_grains; ++g)
        if (std::find(nets.begin(), nets.end(), surs_host[g]) == nets.end()) nets.push_back(surs_host[g]);
    for (hsd_sur* net : nets) {
        std::vector<int> slots;
        for (int g = 0; g < n_grains; ++g)
            if (surs_host[g] == net) slots.push_back(g);
        const hsd_status st = sur_run(ctx, net->s, n_cells, u_dev, n_grains, grain_ids_host, slots, tol, check, j_dev,
                                      diag_dev, w.fblist, list_cap, s);
        if (st != HSD_OK) return st;
    }
    // flagged pairs per slot
    std::vector<unsigned> cnt(n_grains + 1);
    HSD_HIP(ctx, hipMemcpyAsync(cnt.data(), w.cnt, sizeof(unsigned) * (n_grains + 1), hipMemcpyDeviceToHost, s));
    HSD_HIP(ctx, hipStreamSynchronize(s));
    const long long nfb = cnt[n_grains];
    *n_fallback_host = nfb;
    if (nfb == 0) return HSD_OK;
    // fallback: the plain solve on the flagged pairs, written in place
    std::vector<int> counts(n_grains), off(n_grains);
    long long acc = 0;
    for (int g = 0; g < n_grains; ++g) {
        counts[g] = static_cast<int>(cnt[g]);
        off[g] = static_cast<int>(acc);
        acc += cnt[g];
    }
    HSD_HIP(ctx, grow(w.seg_off, w.seg_off_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(w.seg_cnt, w.seg_cnt_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(w.cellmap, w.cellmap_cap, static_cast<size_t>(nfb)));
    HSD_HIP(ctx, grow(w.pairs, w.pairs_cap, static_cast<size_t>(nfb)));
    HSD_HIP(ctx, hipMemcpyAsync(w.seg_off, off.data(), sizeof(int) * n_grains, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(w.seg_cnt, counts.data(), sizeof(int) * n_grains, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemsetAsync(w.cnt, 0, sizeof(unsigned) * n_grains, s));        // reused as cursors
    if (nfb <= list_cap)
        HSD_HIP(ctx, hsd::sur_fb_scatter_list(w.fblist, nfb, n_grains, w.seg_off, w.cnt, w.cellmap, w.pairs, s));
    else            // more flagged pairs than the list holds: scan every pair's flags
        HSD_HIP(ctx, hsd::sur_fb_scatter(diag_dev, static_cast<long long>(n_cells) * n_grains, n_grains, w.seg_off,
                                         w.cnt, w.cellmap, w.pairs, s));
    Batch& b = ctx->batch;
    plan_batch_lists(c, counts, off, n_grains, grain_ids_host, b);
    HSD_HIP(ctx, grow(c.Pt, c.Pt_cap, static_cast<size_t>(std::max(b.rows, 1LL))));
    HSD_HIP(ctx, grow(c.pscale, c.pscale_cap, static_cast<size_t>(n_cells) * n_grains));
    HSD_HIP(ctx, grow(c.views, c.views_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(c.offs, c.offs_cap, static_cast<size_t>(n_grains)));
    HSD_HIP(ctx, grow(c.items, c.items_cap, std::max<size_t>(b.items.size(), 1)));
    HSD_HIP(ctx, grow(c.cslots, c.cslots_cap, std::max<size_t>(b.cslots.size(), 1)));
    HSD_HIP(ctx, hipMemcpyAsync(c.views, b.views.data(), sizeof(hsd::GrainView) * n_grains, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(c.offs, b.offs.data(), sizeof(long long) * n_grains, hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(c.items, b.items.data(), sizeof(int2) * b.items.size(), hipMemcpyHostToDevice, s));
    HSD_HIP(ctx, hipMemcpyAsync(c.cslots, b.cslots.data(), sizeof(hsd::ContractSlot) * b.cslots.size(),
                                hipMemcpyHostToDevice, s));
    hsd::SolveLaunch sl{};
    sl.u = u_dev;
    sl.n_cells = n_cells;
    sl.n_gslots = n_grains;
    sl.views = c.views;
    sl.offs = c.offs;
    sl.Pt = c.Pt;
    sl.pscale = c.pscale;
    sl.diag = diag_dev;
    sl.errword = c.errword;
    sl.cellmap = w.cellmap;
    sl.seg_off = w.seg_off;
    sl.seg_cnt = w.seg_cnt;
    if (side_streams(ctx)) {
        // the classes as concurrent branches, each smaller class's spectra and
        // emitted power contracted on its branch, the largest after the join
        HSD_HIP(ctx, grow(c.cslots_cls, c.cslots_cls_cap, std::max<size_t>(b.cslots_cls.size(), 1)));
        HSD_HIP(ctx, hipMemcpyAsync(c.cslots_cls, b.cslots_cls.data(), sizeof(hsd::ContractSlot) * b.cslots_cls.size(),
                                    hipMemcpyHostToDevice, s));
        auto contract_class = [&](int ci, hipStream_t st) -> hipError_t {
            const int n_sl = b.ccls_begin[ci + 1] - b.ccls_begin[ci];
            if (n_sl == 0) return hipSuccess;
            hsd::ContractLaunch cl{c.cslots_cls + b.ccls_begin[ci], n_sl, b.ccls_blocks[ci], c.Pt, c.pscale,
                                   w.cellmap, j_dev, diag_dev, c.wtrap, c.L, c.Lp, n_grains, c.contract,
                                   c.contract_waves};
            return hsd::launch_contract(cl, st);
        };
        HSD_HIP(ctx, hipEventRecord(c.sev[0], s));
        for (int ci = 0; ci < hsd::kClasses; ++ci) {
            const int n_it = b.cls_begin[ci + 1] - b.cls_begin[ci];
            if (n_it == 0) continue;
            HSD_HIP(ctx, hipStreamWaitEvent(c.side[ci], c.sev[0], 0));
            HSD_HIP(ctx, hsd::launch_solve(c, sl, ci, c.items + b.cls_begin[ci], n_it, c.queue + ci, c.side[ci]));
            if (ci != b.c_last) HSD_HIP(ctx, contract_class(ci, c.side[ci]));
            HSD_HIP(ctx, hipEventRecord(c.sev[1 + ci], c.side[ci]));
            HSD_HIP(ctx, hipStreamWaitEvent(s, c.sev[1 + ci], 0));
        }
        HSD_HIP(ctx, contract_class(b.c_last, s));
        return HSD_OK;
    }
    for (int ci = 0; ci < hsd::kClasses; ++ci) {
        const int n_it = b.cls_begin[ci + 1] - b.cls_begin[ci];
        if (n_it == 0) continue;
        HSD_HIP(ctx, hsd::launch_solve(c, sl, ci, c.items + b.cls_begin[ci], n_it, c.queue + ci, s));
    }
    // the flagged pairs' spectra and emitted power, every slot in one launch
    hsd::ContractLaunch cl{c.cslots, static_cast<int>(b.cslots.size()), b.c_blocks, c.Pt, c.pscale, w.cellmap,
                           j_dev, diag_dev, c.wtrap, c.L, c.Lp, n_grains, c.contract, c.contract_waves};
    HSD_HIP(ctx, hsd::launch_contract(cl, s));
    return HSD_OK;
}

}  // extern "C"
