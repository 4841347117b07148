// Internal declarations of the HIP library behind include/hsd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hsd.h"

namespace hsd {

// CODATA 2018 exact values (CGS); the library's own copy.
constexpr double kPlanck = 6.62607015e-27;   // erg s
constexpr double kLight = 2.99792458e10;     // cm s^-1
constexpr double kBoltzmann = 1.380649e-16;  // erg K^-1
constexpr double kHC = kPlanck * kLight;
constexpr double kPi = 3.14159265358979323846;

constexpr int kMaxBins = 1024;
constexpr int kMaxLambda = 1024;

// Per-step (column) parameters of the heating-rate recursion, one per lower
// bin i.  Read with wave-uniform addresses.
struct alignas(32) ColPar {
    double invcool;   // 1 / T_(i-1)i (0 for i = 0)
    int ia;           // integer part of the column's grid coordinate, minus 1
    float fa;         // fractional part plus 1, in [1, 2)
    int kb, ke;       // rows k with a grid-resident transition i -> k: kb..ke (kb > ke: none)
    int jstar;        // first grid index of the photons that heat i -> i+1 continuously (L: none)
    float invgap;     // 1 / (E_(i+1) - E_i) (0 for the top bin)
};

// Interpolation constants of a transition distance d = f - i: grid
// coordinate b_d = ln(r^d - 1) / dln(lambda) split as -floor and fraction.
struct alignas(8) DPar {
    int nib;          // -floor(b_d)
    float fb;         // b_d - floor(b_d), in [0, 1)
};

// Device tables of one registered grain (all owned by the context).
struct Grain {
    int n_bins = 0;
    double E_lo = 0, E_hi = 0, n_atoms = 0, theta = 0, longwave = 0, radius = 0;
    double* E = nullptr;       // [n]
    double* dE = nullptr;      // [n]
    double* T = nullptr;       // [n]
    double* cool = nullptr;    // [n]
    ColPar* colpar = nullptr;  // [n]
    DPar* dpar = nullptr;      // [n]   entry d = 1..n-1
    double* gam = nullptr;     // [n]   log2(dE_k) + 3 log2(lambda_0) - log2(h^2 c)
    double* invgap = nullptr;  // [n]   1 / (E_(i+1) - E_i)
    int* jstar = nullptr;      // [n]   first grid index of continuous (intrabin) photons, L = none
    int* jrep = nullptr;       // [n]   first grid index of representable photons from bin i
    double* cabs = nullptr;    // [L]
    float* Bt = nullptr;       // [n][Lp] C_abs B_lambda(T_i) [E_i >= hc/lambda] / s_lambda
    float* bscale = nullptr;   // [Lp]   s_lambda (0 where the column is empty)
    int nbp = 0;               // n rounded up to 64
    unsigned short* Bh = nullptr;   // [Lp][nbp] Bt transposed as BF16 hi terms (zero padded)
    unsigned short* Bl = nullptr;   // [Lp][nbp] and lo terms bf16(Bt - hi)
};

// Kernel-side view of a grain for the solver.
struct GrainView {
    const ColPar* colpar;
    const DPar* dpar;
    const double* gam;
    const double* invgap;
    const int* jstar;
    const int* jrep;
    const double* cabs;
    double rbin;      // r = E_(i+1) / E_i
    int nb;
    int pad;
};

// Launch configuration of one bin-count class of the solver (defaults, or the
// autotuner's choice).
constexpr int kClasses = 4;
constexpr int kClassHi[kClasses] = {1024, 512, 256, 128};   // class c holds kClassHi[c+1] < bins <= kClassHi[c]
struct ClassCfg {
    int kg = 2;          // row slots per straight-line group: 2 or 4
    int wide = 0;        // alternate lane layout: > 512 bins: 0 = 32 lanes x 32 slots with Cum in LDS,
                         // 1 = 64 x 16; 257..512 bins: 0 = 32 x 16, 1 = 16 x 32 with Cum in LDS;
                         // <= 128 bins: 0 = 16 x 8, 1 = 8 x 16
    int persistent = 0;  // 1 = persistent grid fed by an atomic item counter
};
// Classes with an alternate lane layout.
constexpr bool class_has_wide(int cls) { return cls == 0 || cls == 1 || cls == 3; }

// One grain slot of a batch for the grouped emission contraction.
struct ContractSlot {
    long long pt_off;         // first element of the slot's P~ rows [rows][nb] in the workspace
    const float* Bt;          // [nb][Lp]           (FP32 mode)
    const unsigned short* Bh; // [Lp][nbp] hi / lo  (split-BF16 mode)
    const unsigned short* Bl;
    const float* bscale;      // [Lp]
    int nb, nbp, rows, gslot;
    int tile0;                // first workgroup of the slot in the grid
    int rowmap_off;           // cell of row r: rowmap[rowmap_off + r]; -1: row r is cell r
};

struct Ctx {
    int device = 0;
    ClassCfg cfg[kClasses];
    int L = 0, Lp = 0;
    double lnlam0 = 0, dlnlam = 0;
    double* lam = nullptr;        // [L] device copy of the grid
    double* wtrap = nullptr;      // [L] 4 pi x trapezoid weights of the grid
    std::vector<double> lam_host;
    std::vector<Grain> grains;
    std::string err;
    // workspace (grown on demand)
    float* Pt = nullptr;          size_t Pt_cap = 0;       // scaled P rows
    float* pscale = nullptr;      size_t pscale_cap = 0;   // max P per pair
    float* diag_tmp = nullptr;    size_t diag_cap = 0;
    GrainView* views = nullptr;   size_t views_cap = 0;
    long long* offs = nullptr;    size_t offs_cap = 0;
    int2* items = nullptr;        size_t items_cap = 0;
    ContractSlot* cslots = nullptr; size_t cslots_cap = 0;
    unsigned* queue = nullptr;    // [kClasses] item counters of persistent launches
    double* sizew = nullptr;      size_t sizew_cap = 0;   // size-distribution weights
    unsigned* errword = nullptr;  // device: bit 0 set by kernels on non-finite input
    unsigned char* scratch = nullptr;   // device address of the library's fixed scratch array on this device
    int contract = 1;             // emission contraction: 0 FP32 products, 1 three BF16 products (hi/lo split)
    int contract_waves = 4;       // waves per contraction workgroup (split BF16): 4 or 8
    bool timing = false;
    bool timed = false;           // events of the last solve are recorded
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // eager solves: the classes as concurrent branches on these streams (made
    // on first use), each smaller class contracted on its branch from these
    // slots by class
    hipStream_t side[kClasses] = {};
    hipEvent_t sev[kClasses + 1] = {};
    ContractSlot* cslots_cls = nullptr; size_t cslots_cls_cap = 0;
};

// Gauss-Legendre rules used by the precompute kernels (nodes on [-1, 1]).
struct GLRule {
    int n;
    double x[24];
    double w[24];
};
GLRule gauss_legendre(int n);

// ---- launchers (host functions, defined in the .hip files) ----
hipError_t build_grain_tables(Ctx& c, Grain& g);                        // hsd_precompute.hip

struct SolveLaunch {
    const double* u;
    int n_cells, n_gslots;
    const GrainView* views;   // device [n_gslots]
    const long long* offs;    // device [n_gslots] element offset of each slot in Pt
    float* Pt;
    float* pscale;            // [n_cells * n_gslots]
    float* diag;              // [n_cells * n_gslots * 4] or null
    double* P64;              // [n_cells * nb] (single-slot P output) or null
    unsigned* errword;
    // optional pair lists: slot s solves the cells cellmap[seg_off[s] .. + seg_cnt[s]]
    // (its P~ rows in that order); null = every cell for every slot
    const int* cellmap = nullptr;
    const int* seg_off = nullptr;
    const int* seg_cnt = nullptr;
};
// Launch the fused rates -> B -> recursion kernel for every pair of the
// listed (slot, first cell) items of bin-count class cls, with the class's
// configuration in c.cfg.  A persistent configuration needs `queue`, one
// device counter that this call clears (with a kernel) before the launch.
hipError_t launch_solve(const Ctx& c, const SolveLaunch& a, int cls, const int2* items_dev, int n_items,
                        unsigned* queue, hipStream_t s);
int solve_cells_per_item(const ClassCfg& cfg, int cls);
// Workgroups of class cls's kernel (in the context's configuration) that fit
// on the device at once; the persistent grid size.  Queries the runtime on the
// first call per kernel only.
int solve_capacity(const Ctx& c, int cls);

hipError_t launch_from_rates(const Ctx& c, int nb, int n_pairs, const double* A, const double* cool,
                             double* P, hipStream_t s);

// Every slot of a batch in one launch: one workgroup per (slot, 64-row tile),
// looping over the wavelength tiles; with diag, the epilogue also sums the
// pair's emitted power 4 pi int j dlambda (FP64) and writes diag entry 1.
struct ContractLaunch {
    const ContractSlot* slots;   // device [n_slots]
    int n_slots, n_blocks;
    const float* Pt;             // workspace base
    const float* pscale;         // [cells * n_gslots]
    const int* rowmap;           // pair lists, or null
    float* j;                    // [cells][n_gslots][L]
    float* diag;                 // [cells][n_gslots][4] or null
    const double* wtrap;         // [L] 4 pi x trapezoid weight of each grid wavelength
    int L, Lp, n_gslots, mode;   // mode 0 FP32 products, 1 split BF16
    int waves;                   // split BF16: waves per workgroup, 4 or 8 (wavelength panels of 64 waves)
};
hipError_t launch_contract(const ContractLaunch& a, hipStream_t s);
// Host side: the slot descriptors of a batch (rows[g] P~ rows of slot g at
// offs[g]; lists: rowmap_off[g] or -1) and the grid size.
int contract_blocks(std::vector<ContractSlot>& slots);
// The table method (hsd_table.hip).
hipError_t launch_node_fields(const double* u_ref, double lo, double step, int n_nodes, int L, double* u_out,
                              hipStream_t s);
hipError_t launch_cell_energies(const double* u, const double* lam, int n_cells, int L, int G,
                                const double* const* cabs, double* energy, double* A, hipStream_t s);
hipError_t launch_table_logs(const float* j, const double* A, int n_nodes, int G, int L, float* table, hipStream_t s);
// Energy budget of a table (rho [G][n_nodes]: 4 pi int 2^y dlambda per node
// spectrum) and the cells' node-grid coordinates, for the HSD_CHECK_TABLE check.
hipError_t launch_budget_nodes(const float* table, int n_nodes, int G, int L, const double* lam, double* rho,
                               hipStream_t s);
hipError_t launch_node_coord(const double* energy, const double* ref_energy, int n_cells, double lo, double step,
                             int n_nodes, double* t, hipStream_t s);
hipError_t launch_table_eval(const double* energy, const double* ref_energy, const double* A, const float* table,
                             int n_nodes, double lo, double step, int n_cells, int G, int L, float* j, hipStream_t s);
// Exponentials per second that the device issues (hsd_measure.hip).
hipError_t measure_exp2(double* per_s);
// flags as hsd_size_convolve's: bit 0 lambda-weighted, bit 1 in eV.
hipError_t launch_sizedist(const float* j, const double* w, const double* lam, int n_cells, int G, int L, int flags,
                           double* out, hipStream_t s);

// ---- learned surrogate (hsd_surrogate.hip) ----
// Layers whose input operand enters the BF16 products as two terms, hi =
// bf16(x) and lo = bf16(x - hi) (about 16 significant bits): the normalised
// features (the network's input) and the last hidden activations.
constexpr int kSplitIn[4] = {1, 0, 0, 1};
// Normalisation scale of the energy-ratio output, in units of its standard
// deviation over the training set.
constexpr double kRatioScale = 10.0;
struct Sur {
    Ctx* c = nullptr;
    int L = 0;                 // wavelengths of the spectrum
    int n_out = 0;             // network outputs: L spectrum values, then the energy ratio
    int widths[5] = {33, 256, 256, 256, 0};
    long long n_params = 0;
    long long off_W[4] = {}, off_b[4] = {};
    float* w = nullptr;        // master weights
    float* g = nullptr;        // gradients
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    float* we = nullptr;       // moving average of the weights over the training steps
    long long t = 0;           // Adam steps taken
    float* xm = nullptr;       // [33] input means / stds
    float* xs = nullptr;
    float* ym = nullptr;       // [n_out] target means / stds
    float* ys = nullptr;
    float* wq = nullptr;       // [n_out] 4 pi x trapezoid weights (0 for the ratio output)
    float band_weight = 0.f;   // bw of the band-weighted loss (0: plain mean squared error)
    float* bw_l = nullptr;     // [L] trapezoid half-segment of each node to its left / right
    float* bw_r = nullptr;
    int* segband = nullptr;    // [L - 1] band of each grid segment
    int* bedge = nullptr;      // [33] first segment of each band, then L - 1
    bool have_norm = false;
    // training workspace (grown on demand)
    int cap_B = 0;
    float *Xb = nullptr, *Yb = nullptr, *Z[3] = {}, *H[3] = {}, *Yh = nullptr, *dY = nullptr, *dZ[2] = {};
    float* Wb = nullptr;       // [B][n_out] loss weights of the minibatch (band-weighted loss)
    long long* idx = nullptr;
    double* loss = nullptr;    // the minibatch loss, then the loss reduction's per-block partials
    int splits = 1;            // K splits of the weight-gradient products
    float* split_work = nullptr;
    unsigned short* wb = nullptr;   // BF16 weights for inference (W1 padded to 64 inputs)
    bool wb_fresh = false;
    bool train_graph = true;   // training steps replayed from one captured HIP graph (else eager launches)
    std::vector<float> loss_trace;
};

hipError_t sur_alloc(Sur& s);
void sur_free(Sur& s);
hipError_t sur_grow(Sur& s, int B);
hipError_t sur_bands(const Ctx& c, const double* u, int n_cells, float* bands, hipStream_t st);
hipError_t sur_wc(const Ctx& c, const double* const* cabs, int n_sel, double* wcT, hipStream_t st);
hipError_t sur_pairs(const Ctx& c, const double* u, const float* bands, const double* wcT, const float* loga,
                     long long row0, long long n_rows, int n_sel, float* X, double* A, unsigned short* xb,
                     const float* xm, const float* xs, hipStream_t st);
hipError_t sur_targets(const float* j, const double* A, const double* lam, long long n, int L, float* Y,
                       hipStream_t st);
hipError_t sur_colstats(const float* Xm, long long n, int w, std::vector<double>& mean, std::vector<double>& sd);
hipError_t sur_forward(Sur& s, int B, const float* Xb, hipStream_t st, bool keep_z);
hipError_t sur_backward(Sur& s, int B, const float* Xb, hipStream_t st);
hipError_t sur_loss(Sur& s, int B, hipStream_t st);
hipError_t sur_gather(Sur& s, const float* X, const float* Y, int B, hipStream_t st);
hipError_t sur_batch_idx(Sur& s, unsigned long long seed, long long step, int B, long long n, hipStream_t st,
                         const long long* ctr = nullptr);
hipError_t sur_seq_idx(Sur& s, long long first, int B, hipStream_t st);
hipError_t sur_adam(Sur& s, float lr, hipStream_t st, bool ema = false, float ema_decay = 0.f);
// Adam's bias-corrected step sizes (lr_t, eps_t) of step t (1-based).
float2 adam_step_sizes(float lr, long long t);
// Graph-replayable training step pieces: Adam with the step sizes of step
// *ctr at sched[*ctr - t0]; the step's end (loss into trace[*ctr - t0] when
// trace is given, then ++*ctr).
hipError_t sur_adam_sched(Sur& s, const float2* sched, const long long* ctr, long long t0, hipStream_t st, bool ema,
                          float ema_decay);
hipError_t sur_step_end(long long* ctr, long long t0, const double* loss, double* trace, hipStream_t st);
hipError_t sur_pack(Sur& s, hipStream_t st);
hipError_t sur_infer_rows(Sur& s, int M, const unsigned short* xb, const double* A, long long row0, int n_sel,
                          int n_slots, const int* sel, float* j, float* emit, float* rho, unsigned short* h0,
                          unsigned short* h1, hipStream_t st);
int sur_emit_parts(int n_out);
// rho: the network's ratios (HSD_CHECK_MODEL) or null; bud: the table budget
// [rows][bud_K] with bud_row per slot and cell_t per cell (HSD_CHECK_TABLE) or null.
hipError_t sur_diag(const double* A, const float* emit, int n_parts, const float* rho, const double* bud,
                    const int* bud_row, int bud_K, const double* cell_t, long long row0, long long n, int n_sel,
                    int n_slots, const int* sel, float tol, float* diag, unsigned* cnt, long long* list,
                    long long list_cap, hipStream_t st);
hipError_t sur_fb_scatter_list(const long long* list, long long n, int n_slots, const int* seg_off, unsigned* cursor,
                               int* cellmap, long long* pairs, hipStream_t st);
hipError_t sur_fb_scatter(const float* diag, long long n_pairs, int n_slots, const int* seg_off, unsigned* cursor,
                          int* cellmap, long long* pairs, hipStream_t st);

}  // namespace hsd
