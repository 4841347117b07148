/*
 * hsd.h -- C ABI of the MI355X stochastic-heating emissivity library.
 *
 * For every (cell radiation field, grain size) pair the library computes the
 * steady-state enthalpy-bin probabilities P_i of a radiatively heated grain and
 * its emission spectrum j_lambda, with the matrix formalism summarised in
 * Porter & Vladimirov, arXiv:1311.4627, Sec. 2 (Guhathakurta & Draine; Draine &
 * Li) in the "thermal continuous" approximation:
 *
 *   heating  A_fi = Omega(lambda_fi) lambda_fi^3 dE_f / (h^2 c), f > i,
 *            Omega = u_lambda C_abs interpolated log-log on the wavelength grid
 *            (Sec. 2.2, eq:heating, eq:interpolation), plus the continuous
 *            intrabin term of Draine & Li on A_(i+1)i;
 *   cooling  T_(f-1)f = [8 pi / (h^3 c^2)] int_0^{E_f} E^3 C_abs / (e^{E/kT_f} - 1) dE
 *            / (E_f - E_(f-1))   (Sec. 2.2, eq:cooling);
 *   B_fj = sum_{k>=f} A_kj (eq:bmatrix), X_0 = 1,
 *   X_f = sum_{j<f} B_fj X_j / T_(f-1)f (eq:xf), P = X / sum X (eq:renormalization);
 *   j_lambda = C_abs(lambda) sum_i P_i B_lambda(T_i) [E_i >= hc/lambda]
 *            (Sec. 2.3, eq:emission, eq:emission-lambda).
 *
 * Units are CGS throughout: wavelength cm, energy erg, cross-section cm^2,
 * field energy density u_lambda erg cm^-3 cm^-1, emissivity j_lambda
 * erg s^-1 sr^-1 cm^-1 per grain.
 *
 * Conventions shared by every entry point:
 *  - Every call returns an hsd_status; on failure hsd_last_error() holds a
 *    message.  No C++ exception crosses the ABI.
 *  - Pointers named *_dev are device pointers on the context's device (for
 *    instance the data_ptr() of a PyTorch tensor).  Pointers named *_host are
 *    host pointers.  The caller owns every buffer it passes; the library never
 *    frees or retains them past the call (asynchronous calls read and write
 *    them until the stream reaches the enqueued work).
 *  - The library owns its per-grain tables and workspaces; they persist, grow
 *    on demand and are released by hsd_destroy().
 *  - Asynchronous entry points take a hipStream_t as void*; NULL means the
 *    null stream.  Errors raised by device work surface at the next
 *    hsd_sync() (or the next synchronous call).
 *  - A context is not re-entrant: calls on one context must be serialised by
 *    the caller (the paper's library serialises concurrent calls the same
 *    way, appendix on usage in parallel platforms).  Separate contexts are
 *    independent.
 */
#ifndef HSD_H
#define HSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HSD_OK = 0,
    HSD_ERR_INVALID_ARG = -1,       /* null pointer, bad size, bad id */
    HSD_ERR_UNSUPPORTED_GRID = -2,  /* wavelength grid not log-uniform or too long */
    HSD_ERR_OOM = -3,               /* device allocation failed */
    HSD_ERR_HIP = -4,               /* a HIP runtime call failed */
    HSD_ERR_NONFINITE_INPUT = -5,   /* a field value was NaN, infinite or negative */
    HSD_ERR_STATE = -6              /* call not valid in the context's state */
} hsd_status;

typedef struct hsd_ctx hsd_ctx;
typedef struct hsd_plan hsd_plan;

/* One grain size of one composition (the paper's GrainModel row plus the
 * engine's enthalpy grid, appendix on the library interface).  There is no
 * flags field: the one switch such a row could carry, the continuous
 * (intrabin) heating term, is always on, and no other per-grain option
 * exists. */
typedef struct {
    double radius_cm;        /* grain radius: an input of the surrogate (the plain solve
                                takes the size from C_abs); > 0 for surrogate use */
    double n_atoms;          /* N: 3N Debye modes, real-valued                        */
    double theta_debye_K;    /* Debye temperature of the heat capacity               */
    int32_t n_bins;          /* M + 1 enthalpy bins; 16 <= n_bins <= 1024, multiple of 16 */
    double E_lo_erg;         /* E_0: lowest bin enthalpy, > 0                          */
    double E_hi_erg;         /* E_M: highest bin enthalpy, > E_lo; bins are log-uniform */
    const double* cabs_host; /* [n_lambda] C_abs on the context's wavelength grid, > 0 */
    double longwave_index;   /* p: C_abs ~ lambda^-p beyond the grid's long end (used by
                                the cooling integral only)                              */
} hsd_grain_desc;

/* Create a context on HIP device `device` for the wavelength grid
 * lambda_host[0..n_lambda-1] (cm, strictly increasing, log-uniform to 1e-9
 * relative, 16 <= n_lambda <= 1024).  Rates are evaluated at arbitrary
 * wavelengths by the closed-form grid index of a log-uniform grid; another
 * grid gives HSD_ERR_UNSUPPORTED_GRID.  *out receives the context. */
hsd_status hsd_create(int32_t device, const double* lambda_host, int32_t n_lambda, hsd_ctx** out);

/* Release every device allocation of the context and the context itself.
 * Waits for the context's outstanding work.  NULL is ignored. */
void hsd_destroy(hsd_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  The string belongs to
 * the context and stays valid until the next call on it. */
const char* hsd_last_error(const hsd_ctx* ctx);

/* Register a grain and build its device tables (Sec. 2.2: everything that does
 * not depend on the field is precomputed once): bin enthalpies and widths,
 * bin temperatures from the Debye heat capacity, cooling rates, the scaled
 * Planck table for the emission contraction, and the closed-form
 * interpolation tables for the heating rates.  Synchronous.  *grain_id
 * receives a small non-negative id. */
hsd_status hsd_add_grain(hsd_ctx* ctx, const hsd_grain_desc* desc, int32_t* grain_id);

/* Copy a grain's field-independent tables to host arrays of n_bins doubles
 * each (any pointer may be NULL): bin enthalpies E_i (erg), bin widths dE_i
 * (erg), bin temperatures T_i (K) and cooling rates T_(f-1)f (s^-1, entry 0 is
 * 0).  Synchronous. */
hsd_status hsd_grain_tables(hsd_ctx* ctx, int32_t grain_id, double* E_host, double* dE_host,
                            double* T_host, double* cool_host);

/* The plain solve (Sec. 2): for every cell c < n_cells and every listed grain
 * g, compute P and j_lambda.
 *   u_dev      [n_cells][n_lambda] double: field energy density per unit
 *              wavelength, finite and >= 0 (a violation is flagged per pair and
 *              reported as HSD_ERR_NONFINITE_INPUT by hsd_sync; the pair is
 *              solved with the bad values read as 0).
 *   grain_ids_host [n_grains] ids from hsd_add_grain (repeats allowed).
 *   j_dev      [n_cells][n_grains][n_lambda] float: emissivity per grain,
 *              erg s^-1 sr^-1 cm^-1.
 *   diag_dev   optional [n_cells][n_grains][4] float: absorbed power
 *              int c u C_abs dlambda, emitted power 4 pi int j dlambda (both
 *              erg s^-1 on the grid, trapezoid), the representable absorbed
 *              power A_rep, and the pair's flags as an exact small integer
 *              (bit 0: no heating term, P = delta_i0; bit 1: X was rescaled;
 *              bit 2: non-finite or negative field value).
 * Asynchronous on `stream`; grows the context's workspace if needed (that
 * growth allocates and synchronises). */
hsd_status hsd_solve(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                     const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream);

/* hsd_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels, arguments, results and asynchrony, but the solve's workspace
 * (grain views, work items, per-pair scales and the scaled-P rows: 256-byte
 * aligned pieces, 4 bytes per bin per pair for the rows) lives in a fixed
 * 64 MiB device array inside the library, one per GPU, held until the
 * process ends.  A batch that needs more than that fails with
 * HSD_ERR_INVALID_ARG (the message gives the bytes it needs; the batched
 * workload's 13,968 bins per cell allow about 1,100 cells per call).  The call
 * makes no hipMalloc / hipFree; it copies the batch's small description
 * (views, offsets, work items) host to device on `stream`.  Every context on
 * a GPU shares that GPU's array and it keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other threads or contexts)
 * race on it and must be serialised by the caller. */
hsd_status hsd_solve_noalloc(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                             const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream);

/* Same solve for one grain, returning the bin probabilities in double
 * precision instead of the spectrum: P_dev [n_cells][n_bins] double.
 * Asynchronous on `stream`. */
hsd_status hsd_solve_P(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t grain_id,
                       double* P_dev, void* stream);

/* The FP64 steps alone, on rates the caller supplies: B sums, the X
 * recursion with power-of-two rescaling and the renormalisation
 * (eq:bmatrix, eq:xf, eq:renormalization), for n_pairs independent systems.
 *   A_dev    [n_pairs][n_bins][n_bins] double, row-major: A[f][i] is the
 *            heating rate from bin i to bin f; only f > i is read.
 *   cool_dev [n_pairs][n_bins] double: cool[f] = T_(f-1)f > 0 for f >= 1.
 *   P_dev    [n_pairs][n_bins] double out.
 * n_bins: 16 <= n_bins <= 1024, multiple of 16.  Asynchronous on `stream`.
 * Needs no grain; any context works. */
hsd_status hsd_solve_from_rates(hsd_ctx* ctx, int32_t n_bins, int32_t n_pairs, const double* A_dev,
                                const double* cool_dev, double* P_dev, void* stream);

/* Wait for all device work of the context's device and report deferred
 * errors (including HSD_ERR_NONFINITE_INPUT raised by a previous hsd_solve). */
hsd_status hsd_sync(hsd_ctx* ctx);

/* Phase timing (profiling aid).  With enable != 0, every following hsd_solve
 * records HIP events on its stream around its three phases: the fused
 * rates/recursion kernels, the emission contraction, and the diagnostics.
 * The contraction's epilogue writes the emitted power, so the diagnostics
 * phase holds no launch of its own and reads (close to) 0 ms.
 * hsd_phase_ms waits for the last timed solve and writes the elapsed
 * milliseconds of the three phases to ms_host[0..2].  Timing adds no
 * synchronisation to hsd_solve itself. */
hsd_status hsd_set_timing(hsd_ctx* ctx, int32_t enable);
hsd_status hsd_phase_ms(hsd_ctx* ctx, double* ms_host);

/* ---- The table method (the yardstick of the learned surrogate) ----
 * The paper's introduction names precomputed emissivity tables as the cheap
 * alternative to the full solve that other codes use.  Here such a table
 * holds, per grain, the plain solve (hsd_solve) of one reference field shape
 * u_ref scaled to n_nodes field strengths U_k = 10^(log10U_lo + k (log10U_hi
 * - log10U_lo) / (n_nodes - 1)), stored as y_k(lambda) = log2(j / A), A the
 * pair's absorbed power (trapezoid of c u C_abs); a value without emission is
 * stored as -1e30.  A cell is looked up by U = int u dlambda / int u_ref
 * dlambda alone (clamped to the node range): its spectrum is
 * A_cell 2^((1 - w) y_k + w y_(k+1)), k and w from log10 U on the node grid
 * (zero where a node it draws on has no emission), so each looked-up
 * spectrum carries the cell's own absorbed power and the reference field's
 * shape.
 *   u_ref_dev  [n_lambda] double, the reference field at U = 1;
 *   table_dev  [n_grains][n_nodes][n_lambda] float (the caller's).
 * hsd_table_build solves n_nodes x n_grains pairs (grows the workspace,
 * synchronises once); hsd_table_eval writes j_dev [n_cells][n_grains][n_lambda]
 * like hsd_solve.  Both asynchronous on `stream`. */
hsd_status hsd_table_build(hsd_ctx* ctx, int32_t n_grains, const int32_t* grain_ids_host, const double* u_ref_dev,
                           int32_t n_nodes, double log10U_lo, double log10U_hi, float* table_dev, void* stream);
hsd_status hsd_table_eval(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                          const int32_t* grain_ids_host, const double* u_ref_dev, int32_t n_nodes, double log10U_lo,
                          double log10U_hi, const float* table_dev, float* j_dev, void* stream);

/* The energy budget of a table, as the reference of the surrogate's
 * HSD_CHECK_TABLE check: per grain, the emitted power per unit absorbed power
 * of each node spectrum, rho_k = 4 pi int 2^(y_k) dlambda (trapezoid on the
 * grid; FP64), and the reference field's energy int u_ref dlambda.  A pair's
 * budget is then A rho(t), rho interpolated linearly in the cell's node-grid
 * coordinate t (its log10 U, as hsd_table_eval looks it up): the power the
 * plain model's solves of the reference shape emit at the cell's field
 * strength, from plain solves alone and none of the network's outputs (the
 * energy balance of eq:steady-state as the discrete model realises it).
 *   table_dev, u_ref_dev, n_nodes, log10U_lo/hi: a table as hsd_table_build
 *   wrote it for grain_ids_host (n_grains distinct registered grains).
 * Replaces any budget set before; the check then covers these grains only.
 * Reads the table on `stream` and waits for it; the table may be freed
 * afterwards. */
hsd_status hsd_set_energy_budget(hsd_ctx* ctx, int32_t n_grains, const int32_t* grain_ids_host,
                                 const double* u_ref_dev, int32_t n_nodes, double log10U_lo, double log10U_hi,
                                 const float* table_dev, void* stream);

/* Measurement aid: the number of single-precision exponentials per second
 * the context's device issues (one per heating rate in the solver; the
 * benchmark quotes it beside the solver's roofline).  Runs a calibration
 * kernel of independent exponential chains on an internal stream, ten timed
 * launches after a warm-up.  Synchronous; allocates 2 MB for the duration. */
hsd_status hsd_measure_exp2(hsd_ctx* ctx, double* per_second_host);

/* The emissivity of a whole size distribution (Sec. 2.3, eq:convolution on
 * the discrete size grid): out[c][l] = sum_g w_g j[c][g][l], multiplied by
 * lambda_l when flags has HSD_SIZE_LAMBDA (lambda j_lambda = nu j_nu, the
 * form the paper's library returns) and divided by 1 eV in erg
 * (1.602176634e-12) when it has HSD_SIZE_EV.  The weights w_g are the
 * caller's quadrature of the size distribution, per H atom for the paper's
 * units: with both flags out is then in the paper's eV s^-1 sr^-1 per H
 * (erg s^-1 sr^-1 per H without HSD_SIZE_EV).
 *   j_dev        [n_cells][n_grains][n_lambda] float (as from hsd_solve)
 *   weights_host [n_grains] double, finite
 *   flags        0, or HSD_SIZE_LAMBDA and/or HSD_SIZE_EV (other bits: HSD_ERR_INVALID_ARG)
 *   out_dev      [n_cells][n_lambda] double
 * FP64 sums.  Waits for `stream` once (to reuse the weight buffer), then
 * enqueues on it. */
#define HSD_SIZE_LAMBDA 1
#define HSD_SIZE_EV 2
hsd_status hsd_size_convolve(hsd_ctx* ctx, int32_t n_cells, int32_t n_grains, const float* j_dev,
                             const double* weights_host, int32_t flags, double* out_dev, void* stream);

/* ---- Launch configuration (read and set by the autotuner) ----
 * The solver groups grains into four bin-count classes, each served by its
 * own kernel shape: class 0 holds 513..1024 bins, class 1 257..512, class 2
 * 129..256 and class 3 16..128.  Per class:
 *   kg          row slots evaluated per straight-line group: 2 or 4;
 *   wide        the alternate lane layout, classes 0, 1 and 3 (1 is refused
 *               for class 2).  Class 0: 0 = 32 lanes per pair with 32 row
 *               slots each and the absorbed-power table in LDS, 1 = 64 lanes
 *               with 16 slots; class 1: 0 = 32 lanes with 16 slots, 1 = 16
 *               lanes with 32 slots and the absorbed-power table in LDS;
 *               class 3: 0 = 16 lanes with 8 slots, 1 = 8 lanes with 16;
 *   persistent  0 = one workgroup per work item (items in an order that
 *               gives each XCD whole cell blocks), 1 = a grid of the
 *               workgroups that fit on the device at once, fed items longest
 *               first from an atomic counter.
 * kg and persistent change speed only: the results are the same bit for bit.
 * wide also changes the order of the FP64 sums, so results agree to rounding.
 * The defaults are kg 2, wide 0, persistent 0.  Synchronous; affects later
 * solves and later plans. */
typedef struct {
    int32_t kg;
    int32_t wide;
    int32_t persistent;
} hsd_class_cfg;
hsd_status hsd_get_class_cfg(hsd_ctx* ctx, int32_t cls, hsd_class_cfg* cfg_host);
hsd_status hsd_set_class_cfg(hsd_ctx* ctx, int32_t cls, const hsd_class_cfg* cfg_host);

/* Emission contraction (Sec. 2.3, eq:emission): j = (P~ B~) max P s_lambda,
 * a (cells x bins) . (bins x wavelengths) product per grain with both
 * operands in [0, 1] and FP32 accumulation, on the matrix cores in one of
 *   HSD_CONTRACT_FP32    FP32 products (v_mfma_f32_16x16x4_f32);
 *   HSD_CONTRACT_BF16X3  each operand x split as hi = bf16(x), lo =
 *                        bf16(x - hi), |x - hi - lo| <= 2^-16 |x|, and the
 *                        product taken as hi hi + hi lo + lo hi on BF16
 *                        matrix cores (v_mfma_f32_16x16x32_bf16): every term
 *                        within 3 2^-16 = 4.6e-5 of the exact product, and
 *                        since all terms are >= 0, so is each j value.
 * The default is HSD_CONTRACT_BF16X3.  Affects later solves and later plans. */
#define HSD_CONTRACT_FP32 0
#define HSD_CONTRACT_BF16X3 1
hsd_status hsd_set_contract(hsd_ctx* ctx, int32_t mode);
hsd_status hsd_get_contract(hsd_ctx* ctx, int32_t* mode_host);

/* Workgroup size of the split-BF16 contraction (a tuning choice, results
 * unchanged: every j value is the same sum in the same order; the emitted
 * power's FP64 sum is regrouped): 4 waves (the default) walk the padded
 * wavelengths in panels of 256 and read each grain's P~ rows once per panel,
 * 8 waves take panels of 512 and read them once, with one workgroup per
 * compute unit.  Other values fail with HSD_ERR_INVALID_ARG.  Affects later
 * solves and later plans. */
hsd_status hsd_set_contract_waves(hsd_ctx* ctx, int32_t waves);
hsd_status hsd_get_contract_waves(hsd_ctx* ctx, int32_t* waves_host);

/* ---- Autotuner ----
 * Time every configuration of every bin-count class that the listed grains
 * occupy, on the given batch, and keep the fastest per class in the context
 * (later solves and plans use it).  Each configuration runs the solver phase
 * (rates, sums, recursion, scaled-P writes; no contraction) `runs` times on an
 * internal stream; the first run is a warm-up and the mean of the others is
 * the score (the paper's benchmarks time 4 runs and average the last 3, Sec. 3).  The
 * paper picks its tile sizes by measurement in the same way (appendix on loop
 * tiling).  One record per configuration timed is written to
 * records_host[0..max_records-1]; *n_records receives the number timed.
 * Synchronous; grows the context's workspace. */
typedef struct {
    int32_t cls;             /* bin-count class; -1: a whole-plan record (hsd_autotune_plan's
                                starting point, or its contraction candidate) */
    hsd_class_cfg cfg;       /* configuration timed (zeros for cls = -1) */
    int32_t contract_waves;  /* contraction workgroup size in effect */
    int32_t n_grains;        /* grains of the batch in this class (all, for cls = -1) */
    double ms;               /* mean time of the timed runs: the solver phase (hsd_autotune)
                                or the whole plan replay (hsd_autotune_plan) */
} hsd_tune_record;
hsd_status hsd_autotune(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                        const int32_t* grain_ids_host, int32_t runs, hsd_tune_record* records_host,
                        int32_t max_records, int32_t* n_records);

/* Tuning for plans, timed as they run: every candidate is a concurrent plan
 * (HSD_PLAN_CONCURRENT) of the given batch — all occupied classes as
 * parallel graph branches with their contractions, into an internal j
 * buffer —
 * replayed `runs` times (first replay a warm-up, the mean of the others the
 * score).  Starting from the context's configuration with every class as an
 * ordinary grid (persistent = 0, as concurrent plans require), it tries, one
 * class at a time from the largest bin counts down, each other slot-group
 * size and lane layout with the other classes fixed and keeps any that is
 * faster, then the other contraction workgroup size
 * (hsd_set_contract_waves).  The winners stay in the context.  One record per
 * plan timed (the first, cls = -1, is the starting point).  Synchronous;
 * allocates a j buffer of n_cells x n_grains x n_lambda floats and one plan
 * workspace at a time.  On failure the context's configuration is restored. */
hsd_status hsd_autotune_plan(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                             const int32_t* grain_ids_host, int32_t runs, hsd_tune_record* records_host,
                             int32_t max_records, int32_t* n_records);

/* ---- Plans: a batch captured once as a HIP graph ----
 * The paper keeps its data resident on the coprocessor and reuses it across
 * calls (appendix on offload traffic reduction); a plan does the same for a
 * batch whose shape and buffers do not change: hsd_plan_create records every
 * launch of one hsd_solve of (n_cells, u_dev, grain_ids_host, j_dev, diag_dev)
 * - the solver classes (fields are read directly by the solver, no separate
 * ingest pass) and the contraction with the diagnostics - into one HIP graph,
 * with its own workspace, using the class configurations current at creation.
 * hsd_plan_launch replays it on `stream`; each replay computes exactly what
 * hsd_solve would on the buffers' contents at that time.
 *   flags  HSD_PLAN_TIMING: the solver and the contraction (with the
 *          diagnostics in its epilogue) are captured as graphs of their own,
 *          and hsd_plan_launch records HIP events around the two graph
 *          launches on `stream`; hsd_plan_phase_ms waits for the last launch
 *          and writes the milliseconds of the solver, the contraction and the
 *          diagnostics (always 0, as for hsd_phase_ms) to ms_host[0..2].
 *          HSD_PLAN_CONCURRENT: the solver classes run as parallel branches
 *          of the graph, so one class's tail overlaps the next class, and
 *          each class except the one with the most solver work (bins^2 x
 *          cells) is contracted on its own branch as soon as its solve ends;
 *          that class is contracted after the branches join.  With
 *          HSD_PLAN_TIMING the early contractions count in the solver's
 *          milliseconds.  The results are the same bit for bit as without
 *          the flag.  Every class must then be configured with persistent =
 *          0, else the call
 *          fails with HSD_ERR_INVALID_ARG (a persistent grid takes every
 *          workgroup slot of the device and would hold the other branches
 *          off it).
 * The buffers must stay allocated, and the grains registered, while the plan
 * lives.  A plan is used by one thread at a time; replays of one plan on
 * different streams must not overlap (they share its workspace).
 * hsd_plan_create allocates the workspace and synchronises; hsd_plan_launch
 * allocates nothing.  hsd_plan_destroy waits for the device and frees the
 * plan (NULL is ignored); destroy plans before their context. */
#define HSD_PLAN_TIMING 1
#define HSD_PLAN_CONCURRENT 2
hsd_status hsd_plan_create(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                           const int32_t* grain_ids_host, float* j_dev, float* diag_dev, int32_t flags,
                           hsd_plan** out);
hsd_status hsd_plan_launch(hsd_plan* plan, void* stream);
hsd_status hsd_plan_phase_ms(hsd_plan* plan, double* ms_host);
void hsd_plan_destroy(hsd_plan* plan);

/* ---- Learned surrogate ----
 * Not part of the paper's method: a learned approximation of it (the paper's
 * introduction names precomputed emissivity tables as the cheap alternative
 * to the full solve), with the plain solve as its fallback and its accuracy reference.
 * One network maps a (field, grain) pair to its spectrum:
 *   inputs   x [33]: log10 of the field's energy int u dlambda in 32 bands of
 *            the wavelength grid (band b spans the grid nodes
 *            floor(b (L-1) / 32) .. floor((b+1) (L-1) / 32), trapezoid rule),
 *            then log10 of the grain radius in cm;
 *   outputs  y [L + 1]: y_lambda = log10(j_lambda / A) for the L wavelengths,
 *            A = int c u C_abs dlambda the pair's absorbed power
 *            (trapezoid), then y_L = log10(E / A), E = 4 pi int j dlambda
 *            the emitted power on the grid: the discrete model's own energy
 *            budget, which misses 1 for coarse enthalpy bins (transitions
 *            whose photon energy lies beyond the grid's short end carry no
 *            rate);  training targets are log10(max(j, 1e-6 max j) / A) and
 *            log10(E / A) of the plain solve;
 *   network  33 -> 256 -> 256 -> 256 -> L + 1, GELU (x Phi(x)) after each
 *            hidden layer; inputs z-scored per column, targets centred per
 *            column, the L spectrum columns divided by one pooled standard
 *            deviation and the ratio column by ten times its own
 *            (statistics of the training set); every matrix product rounds its operands to
 *            bfloat16 (the inputs of the first and last layer as two terms,
 *            hi + lo) and accumulates in FP32; master weights FP32.
 * Parameters are one FP32 vector, layer by layer: W_l row-major [out][in],
 * then b_l (269,045 values for L = 500).  Rows of X_dev / Y_dev / A_dev are
 * pairs in the order r = cell * n_grains + g. */
typedef struct hsd_sur hsd_sur;
hsd_status hsd_sur_create(hsd_ctx* ctx, hsd_sur** out);   /* weights uninitialised: set them */
void hsd_sur_destroy(hsd_sur* sur);                       /* NULL is ignored; before the context */
hsd_status hsd_sur_n_params(hsd_sur* sur, int64_t* n_params_host);
/* Set (and reset the optimiser state) / read the FP32 parameter vector.  Synchronous. */
hsd_status hsd_sur_set_params(hsd_sur* sur, const float* params_host);
hsd_status hsd_sur_get_params(hsd_sur* sur, float* params_host);
/* Training loss.  band_weight = 0 (the default) is the mean squared error
 * over the normalised outputs.  With 0 < band_weight <= 1 each spectrum
 * element k of a training row is weighted by W_k = (1 - band_weight) +
 * band_weight L rho_k, where rho_k is element k's share of the bands the
 * accuracy metric counts: over the 32 bands (as for the inputs) whose
 * trapezoid integral of j = A 10^y holds at least 1e-3 of the row's total,
 * rho_k = sum_b j_k q_kb / J_b / n_bands, q_kb node k's trapezoid weight in
 * band b, J_b the band's integral (an error d in log10 j_k moves band b by
 * ln 10 d j_k q_kb / J_b); the ratio output keeps weight 1.  The loss is the
 * mean of W (yhat - y)^2.  Weights come from each row's raw targets.  Kept
 * in checkpoints. */
hsd_status hsd_sur_set_loss(hsd_sur* sur, float band_weight);
/* Column means and standard deviations (> 0) of raw inputs [33] and targets
 * [L + 1].  Synchronous. */
hsd_status hsd_sur_set_norm(hsd_sur* sur, const double* x_mean_host, const double* x_std_host,
                            const double* y_mean_host, const double* y_std_host);
hsd_status hsd_sur_get_norm(hsd_sur* sur, double* x_mean_host, double* x_std_host, double* y_mean_host,
                            double* y_std_host);
/* Raw inputs X_dev [n_cells * n_grains][33] (float) and absorbed powers
 * A_dev [n_cells * n_grains] (double) of every pair; either may be NULL.
 * Grains need radius_cm > 0.  Asynchronous on `stream`. */
hsd_status hsd_sur_features(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                            const int32_t* grain_ids_host, float* X_dev, double* A_dev, void* stream);
/* Raw targets Y_dev [n][L + 1] from spectra j_dev [n][L] and absorbed
 * powers A_dev [n].  Asynchronous on `stream`. */
hsd_status hsd_sur_targets(hsd_ctx* ctx, int64_t n, const float* j_dev, const double* A_dev, float* Y_dev,
                           void* stream);
/* Statistics of a training set (FP64 column sums on the device): input
 * column means and standard deviations, target column means, the pooled
 * standard deviation of the L spectrum columns (sqrt of their mean variance,
 * repeated) and ten times that of the ratio column (a smaller loss weight),
 * stored as by hsd_sur_set_norm.  Synchronous. */
hsd_status hsd_sur_fit_norm(hsd_sur* sur, int64_t n, const float* X_dev, const float* Y_dev);
/* Test hook: mean squared error over the n rows (normalised targets) and
 * its gradient with respect to the parameter vector (grad_host may be NULL),
 * without an update.  n <= 65536.  Synchronous. */
hsd_status hsd_sur_loss_grad(hsd_sur* sur, int32_t n, const float* X_dev, const float* Y_dev, double* loss_host,
                             float* grad_host);
/* Train: `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8) on minibatches of
 * `batch` rows drawn with replacement by a counter-based generator from
 * `seed`; learning rate warms up linearly over the first 2% of steps, then
 * decays as a cosine to 5% of `lr`.  loss_host (optional) receives each
 * step's minibatch loss.  Optimiser state carries over between calls until
 * hsd_sur_set_params.  On return the parameters are the exponential moving
 * average of the call's iterates (decay min(0.999, 1 - 20 / steps), started
 * from the parameters at the call).  Waits for the device's earlier work
 * first; synchronous.  The steps run as one captured HIP graph replayed
 * `steps` times (its per-step values, the minibatch counter and the step
 * sizes, are read from device memory), unless hsd_sur_set_train_graph(0)
 * asks for eager launches; both give the same bits. */
hsd_status hsd_sur_train(hsd_sur* sur, int64_t n, const float* X_dev, const float* Y_dev, int32_t steps,
                         int32_t batch, float lr, uint64_t seed, float* loss_host);
hsd_status hsd_sur_set_train_graph(hsd_sur* sur, int32_t enable);
/* Checkpoint and resume (the paper's library is configured once and reused
 * across runs, appendix on the library interface; a trained network is kept
 * the same way).  hsd_surrogate_save writes, synchronously, to the file
 * `path` (created or truncated):
 *   line 1   "HSDSUR 1"
 *   line 2   a one-line JSON header: "widths" (33, 256, 256, 256, L + 1),
 *            "n_params", "step" (Adam steps taken, which is also the position
 *            of the minibatch generator), "loss_band_weight" (the setting of
 *            hsd_sur_set_loss), "optimizer" (true when the Adam
 *            moments follow), "byte_order" "little", and "sections": name,
 *            element type "f32" and count of each array below, in order;
 *   then     the arrays, raw little-endian FP32, back to back: params
 *            [n_params] (layout of hsd_sur_set_params), x_mean [33], x_std
 *            [33], y_mean [L + 1], y_std [L + 1], and unless flags has
 *            HSD_SAVE_WEIGHTS_ONLY, adam_m [n_params] and adam_v [n_params].
 * The network needs its statistics (HSD_ERR_STATE otherwise).
 * hsd_surrogate_load reads such a file into a network of the same widths
 * (HSD_ERR_INVALID_ARG for another shape, a truncated or foreign file): the
 * parameters, the statistics, the loss setting, and either the saved Adam moments and step or,
 * for a weights-only file, zero moments and step 0.  A network resumed from a
 * checkpoint trains on exactly as the saved one would: hsd_sur_train calls
 * after hsd_surrogate_load give the same bits as the same calls made on the
 * network that was saved.  Both wait for the device; file errors give
 * HSD_ERR_INVALID_ARG with the reason in hsd_last_error. */
#define HSD_SAVE_WEIGHTS_ONLY 1
hsd_status hsd_surrogate_save(hsd_sur* sur, const char* path, int32_t flags);
hsd_status hsd_surrogate_load(hsd_sur* sur, const char* path);
/* Energy checks of hsd_solve_surrogate.  With E the surrogate's emitted
 * power (4 pi int j dlambda on the grid) and A the pair's absorbed power:
 *   HSD_CHECK_ABSORBED  flag the pair when |E / A - 1| > tol;
 *   HSD_CHECK_MODEL     flag it when |E / (rho A) - 1| > tol, rho = 10^y_L
 *                       the network's prediction of the plain model's own
 *                       ratio E / A: the spectrum must carry the power the
 *                       discrete model absorbs;
 *   HSD_CHECK_TABLE     flag it when |E / B - 1| > tol, B the table budget
 *                       of hsd_set_energy_budget (the plain model's emitted
 *                       power at the cell's field strength, for the
 *                       reference field shape): a reference that does not
 *                       come from the network.  Every grain of the batch
 *                       needs a budget (else HSD_ERR_STATE). */
#define HSD_CHECK_ABSORBED 0
#define HSD_CHECK_MODEL 1
#define HSD_CHECK_TABLE 2
/* Surrogate spectra of every (cell, grain) pair: j_dev as in hsd_solve;
 * diag_dev (optional) = (A, 4 pi int j dlambda, rho A, flags) with flags
 * bit 3 set (value from the surrogate) and bit 4 set where the
 * HSD_CHECK_MODEL test with tol = 0.01 fails.  Asynchronous on `stream`
 * (grows workspace). */
hsd_status hsd_sur_predict(hsd_sur* sur, int32_t n_cells, const double* u_dev, int32_t n_grains,
                           const int32_t* grain_ids_host, float* j_dev, float* diag_dev, void* stream);
/* The surrogate with the plain solve as fallback: every pair is first
 * evaluated by the network surs_host[g] of its grain (one network may serve
 * several grains); a pair that fails the energy check `check`
 * (HSD_CHECK_ABSORBED, HSD_CHECK_MODEL or HSD_CHECK_TABLE, relative
 * tolerance tol; the energy balance of eq:steady-state) is re-solved by the
 * plain path, in place.  j_dev and diag_dev as in hsd_solve; surrogate pairs
 * carry diag flag bit 3 and entry 2 = the power the check compares with (A,
 * rho A or B),
 * re-solved pairs carry the plain solve's diagnostics.  *n_fallback_host
 * receives the number of re-solved pairs.  Waits for the stream once (to
 * size the fallback). */
hsd_status hsd_solve_surrogate(hsd_ctx* ctx, int32_t n_cells, const double* u_dev, int32_t n_grains,
                               const int32_t* grain_ids_host, hsd_sur* const* surs_host, float tol, int32_t check,
                               float* j_dev, float* diag_dev, int64_t* n_fallback_host, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HSD_H */
