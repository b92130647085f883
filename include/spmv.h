/*
 * Adaptive sparse matrix-vector multiply for AMD Instinct MI355X (gfx950).
 *
 * The caller hands over one matrix in CSR form; the library measures its
 * structure on the GPU, picks a storage format (CSR, COO, ELL, DIA, or 4x4
 * block CSR) and a kernel for it, converts the matrix into plan-owned device
 * memory and then
 * computes y = A x as often as asked.  This is the input-adaptive auto-tuner
 * of Li, Zhang, Tan and Chen, "SMAT: An Input Adaptive Sparse Matrix-Vector
 * Multiplication Auto-Tuner" (arXiv 1210.2536): a CSR-based interface
 * (Section 3), the four basic formats (Section 2.1), the feature parameters
 * of Table 3 (Section 4), a learned format model (Section 5) and the runtime
 * search with execute-and-measure refinement (Section 6).
 *
 * Conventions shared by every entry point
 *   - Pointers named *_dev are device pointers (HIP device memory of the
 *     current device); all other pointers are host pointers.
 *   - `stream` is a hipStream_t handle passed as void* (NULL = the null
 *     stream).  Work is enqueued on it; functions that must read results
 *     back synchronise that stream and say so.
 *   - Indices are 0-based int32.  nnz and every padded slot count must stay
 *     below 2^31 for the int32 paths (else SPMV_EUNSUPPORTED).
 *   - Values are float32 (SPMV_F32) or float64 (SPMV_F64).  float32 kernels
 *     multiply and accumulate in float64 and round once per output.
 *   - Errors: every function returns a spmv_status; a negative value is an
 *     error and spmv_last_error() then describes it (thread-local string).
 *     Launch failures are SPMV_EDEVICE; faults inside a kernel surface at the
 *     caller's next synchronisation.
 *   - Thread safety: distinct plans may be used from distinct threads; one
 *     plan must not run on two streams at the same time (its COO carries,
 *     split-row partials and panel partial sums are per-plan scratch).
 */
#ifndef SMAT_SPMV_H
#define SMAT_SPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SPMV_F32 = 0, SPMV_F64 = 1 } spmv_dtype;

typedef enum {
    SPMV_OK = 0,
    SPMV_EINVAL = -1,        /* bad argument or non-canonical CSR */
    SPMV_ENOMEM = -2,        /* device allocation failed */
    SPMV_EDEVICE = -3,       /* HIP runtime / launch error */
    SPMV_EUNSUPPORTED = -4   /* size beyond the int32 paths, or a kernel that
                                cannot represent this matrix */
} spmv_status;

/* Storage formats (Section 2.1), plus 4x4 block CSR (the blocked formats the
 * paper names as its extension, Section 2.1 and the conclusion). */
typedef enum {
    SPMV_FMT_CSR = 0, SPMV_FMT_COO = 1, SPMV_FMT_ELL = 2, SPMV_FMT_DIA = 3, SPMV_FMT_BCSR = 4
} spmv_format;

/* Kernel classes: a format plus an implementation (the paper's "best
 * implementation" per format, Section 3).  These are also the classes the
 * learned selector scores. */
typedef enum {
    SPMV_K_CSR_SCALAR = 0,    /* CSR, one thread per row (plain baseline)      */
    SPMV_K_CSR_VECTOR = 1,    /* CSR, one lane group of fixed width per row     */
    SPMV_K_CSR_ADAPTIVE = 2,  /* CSR, rows binned by length, width per bin,
                                 whole workgroups for long rows               */
    SPMV_K_ELL = 3,           /* ELL, slot-major, one thread per row            */
    SPMV_K_DIA = 4,           /* DIA, x windows staged in LDS                   */
    SPMV_K_DIA_DIRECT = 5,    /* DIA, x read through the caches                 */
    SPMV_K_COO = 6,           /* COO, wavefront segmented reduction             */
    SPMV_K_CSR_PANEL = 7,     /* CSR re-sorted into column panels whose slice
                                 of x fits one XCD's L2 (spmv_params
                                 panel_xcd / panel_kib)                      */
    SPMV_K_BCSR = 8,          /* 4x4 block CSR: block row pointer, block
                                 columns, 16 values per block (row-major,
                                 absent entries +0.0); a lane group per block
                                 row, one block per lane and trip          */
    SPMV_K_COUNT = 9
} spmv_kernel;

/* How plan creation chooses the kernel (Section 6). */
typedef enum {
    SPMV_SELECT_RULES = 0,      /* the Section 4 thresholds, no measurement   */
    SPMV_SELECT_MLP = 1,        /* learned model; measures the top-k when the
                                   model's confidence margin is below tau     */
    SPMV_SELECT_EXHAUSTIVE = 2, /* measure every feasible kernel (brute force) */
    SPMV_SELECT_FORCED = 3      /* use opts.force_kernel                      */
} spmv_selector_mode;

/* A CSR matrix in device memory (Section 3: the unified input format).
 * Canonical form is required: row_ptr[0] = 0, non-decreasing, row_ptr[m] =
 * nnz; 0 <= col < n; columns strictly increasing inside each row.  Explicit
 * zero values are allowed and kept. */
typedef struct {
    int64_t m, n, nnz;
    const int32_t *row_ptr_dev;   /* m + 1 entries */
    const int32_t *col_dev;       /* nnz entries   */
    const void *val_dev;          /* nnz values of `dtype` */
    int32_t dtype;                /* spmv_dtype */
} spmv_csr;

/* Tunable kernel parameters (the paper's offline "kernel search", Section 3,
 * done here per matrix by the autotuner).  Zero means "library default". */
typedef struct {
    int32_t block;              /* threads per workgroup, row-parallel kernels */
    int32_t vector_lanes;       /* CSR_VECTOR lanes per row: 1..64, power of 2 */
    int32_t adaptive_rows_per_lane; /* CSR_ADAPTIVE: a bin of width L takes
                                   rows of up to L * this many entries        */
    int32_t adaptive_wg_min;    /* CSR_ADAPTIVE: rows longer than this get a
                                   whole workgroup                            */
    int32_t dia_rows_per_thread;/* DIA: rows per thread (tile = block * this) */
    int32_t dia_span;           /* DIA: max offset span staged per LDS window */
    int32_t coo_chunk;          /* COO: entries per lane per wavefront chunk  */
    int32_t ell_unroll;         /* ELL: slots fetched per loop trip (1, 2, 4) */
    int32_t stream_nt;          /* matrix arrays loaded non-temporally: 1 on,
                                   2 off (0 = default: on for ELL and DIA of
                                   banded matrices, off otherwise)           */
    int32_t panel_kib;          /* CSR_PANEL: most bytes of x per column
                                   panel, in KiB (default 4096)              */
    int32_t panel_xcd;          /* CSR_PANEL: 1 = all panels in one launch,
                                   eight at a time, one per XCD, each panel
                                   summing into its own partial vector that a
                                   second kernel adds in panel order
                                   (default); 2 = one launch per panel, the
                                   running sums carried in y               */
    int32_t wide_loads;         /* DIA and ELL: 1 = a lane takes 16 bytes'
                                   worth of consecutive rows (4 in float32,
                                   2 in float64) and reads every diagonal or
                                   slot of them with one 16-byte load; 2 =
                                   one row per lane; 0 = default (1 from
                                   2^20 rows on, 2 below)                  */
    int32_t bcsr_lanes;         /* BCSR: lanes per block row, a power of two
                                   in [1, 64].  float32: one block per lane
                                   at a time (0 = default: the mean blocks
                                   per block row rounded up to a power of
                                   two).  float64: 8 lanes read a block
                                   together, so lanes / 8 blocks of a row
                                   are read at once (values below 8 are
                                   raised to 8; 0 = default 8, widened as
                                   the 1e-12 bound needs)                  */
    int32_t long_lds;           /* CSR_ADAPTIVE and CSR_PANEL: where the
                                   rows of the longest bin (a workgroup each
                                   in the binned launch) go.  1 = x chunks
                                   (float64 only): a kernel that streams x
                                   through LDS in column chunks, 16-32 such
                                   rows per workgroup of 1024 threads;
                                   3 = tiles (both dtypes) for the rows
                                   longer than min(adaptive_wg_min,
                                   tile_row_min):
                                   x cut into 80 KB panels, one workgroup
                                   per (row block, panel) holding its panel
                                   in LDS, one float64 partial per (row,
                                   panel), the partials added in a fixed
                                   order by a second kernel; 2 = binned
                                   launch; 0 = default (tiles from 1024
                                   rows longer than 1024, else 2).  Tiles
                                   fall back to chunks
                                   (float64) or 2 where their partials and
                                   segment starts would exceed 1/5 of the
                                   long rows' bytes per run or no lane count
                                   keeps the 1e-12 bound; chunks fall back
                                   to 2 in float32 and for rows too long for
                                   the bound with 64 lanes per row          */
    int32_t tile_row_min;       /* CSR_ADAPTIVE and CSR_PANEL with long-row
                                   tiles: the rows longer than this many
                                   entries go to the tiles (0 = default
                                   1024; at least 64)                      */
    int32_t panel_direct_max;   /* CSR_PANEL: rows of at most this many
                                   entries (rounded down to a length-bin
                                   boundary) skip the column panels -- no
                                   partial sums -- and are summed by the
                                   length-binned kernel reading x through
                                   the caches; -1 = every row in the panels;
                                   0 = default (-1)                          */
} spmv_params;

typedef struct spmv_selector_s *spmv_selector_t;

/* Device memory for a plan (an interface convention, not from the paper:
 * the caller's framework may own all device memory, e.g. PyTorch's caching
 * allocator).  alloc returns at least `bytes` bytes of device memory on the
 * current device, 256-byte aligned, or NULL (plan creation then fails with
 * ENOMEM); free returns a block from alloc with its size.  ctx is passed
 * through.  alloc runs during spmv_plan_create and spmv_convert_roundtrip
 * on the calling thread; free runs there and in spmv_plan_destroy.  Both
 * NULL (the default): hipMalloc / hipFree.  Selectors and batches always
 * use hipMalloc.
 * Stream rule: a block freed during spmv_plan_create or
 * spmv_convert_roundtrip may still be in use by work queued on that call's
 * stream, so the allocator must not hand it out again before that work is
 * done (a stream-ordered pool whose blocks belong to that stream does this,
 * as PyTorch's caching allocator does for blocks allocated on it).
 * spmv_plan_destroy synchronises the plan's device before it calls free,
 * so runs of the plan on any stream have finished by then. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *ctx);
    void *ctx;
} spmv_allocator;

typedef struct {
    int32_t selector;           /* spmv_selector_mode; default MLP when a model
                                   is given, RULES otherwise                  */
    int32_t force_kernel;       /* spmv_kernel for SPMV_SELECT_FORCED         */
    float confidence_tau;       /* MLP margin (predicted log slowdown between
                                   best and runner-up) below which candidates
                                   are measured; default 0.1                  */
    int32_t measure_topk;       /* candidates measured when unsure; default 3 */
    int32_t timing_reps;        /* timed repetitions per candidate; default 5.
                                   Each repetition times back-to-back calls
                                   worth about 50 us (at most 64 calls) and
                                   the median per-call time is kept; after a
                                   prediction another kernel (or parameter
                                   point) replaces the predicted one only
                                   when more than 3% faster               */
    uint32_t disable_mask;      /* bit k set: never pick kernel k             */
    uint64_t mem_cap_bytes;     /* cap on the storage of the padded formats
                                   (ELL, DIA, BCSR) and column panels; 0 =
                                   1/4 of free device memory                */
    spmv_selector_t model;      /* learned model (NULL: rules)                */
    int32_t autotune;           /* 1: time a few parameter points for the
                                   chosen kernel and keep the fastest (the
                                   paper's offline kernel search, Section
                                   3); a point is only kept if its output on
                                   an all-ones probe vector agrees with the
                                   starting point's within twice the
                                   accuracy bound (info.tune_rejected)     */
    int32_t use_params;         /* 1: take `params` as given                  */
    spmv_params params;
    int32_t segments;           /* >= 2: cut the rows into this many segments
                                   of about nnz/segments entries each (at most
                                   64, at most m) and plan each segment on its
                                   own -- its own features, format and kernel
                                   (the per-thread sub-matrices of Section 6)
                                   -- with these same options; 0 or 1: one
                                   plan for the whole matrix (default)      */
    int32_t staged;             /* 1: staged feature extraction (Section 6,
                                   the time-saving format search): rows
                                   statistics, then the diagonal census; if
                                   these already settle the format -- RULES:
                                   the DIA or ELL test passes; MLP: the
                                   model's stage rule (spmv_selector_set_stage)
                                   names a DIA, ELL or CSR kernel, feasible,
                                   with confidence >= stage_conf, inputs inside
                                   the model's domain -- the power-law fit,
                                   the 4x4 block count, the network and any
                                   measurement are skipped.  RULES picks the
                                   same kernel staged or not.  Default 1
                                   (spmv_plan_opts_default); 0: all features
                                   first.  EXHAUSTIVE and FORCED ignore it. */
    float stage_conf;           /* stage rule confidence needed to stop early
                                   (the share of training matrices of the
                                   rule's leaf on which its kernel ran within
                                   5% of the fastest); <= 0: default 0.98  */
    spmv_allocator allocator;   /* plan memory (see spmv_allocator); EINVAL
                                   unless both callbacks or neither are set */
    int32_t time_baseline;      /* 1: after planning, time the chosen kernel
                                   and the plain CSR kernel (one thread per
                                   row, on the caller's CSR) and report the
                                   break-even call count of Equation 2 in
                                   spmv_plan_info (t_run_ms, t_plain_ms,
                                   break_even_calls); 0: not timed         */
    int32_t log;                /* 1: print a one-line plan summary on
                                   stderr when the plan is created          */
} spmv_plan_opts;

/* Feature parameters of Table 3 (Section 4) plus the selector's extras.
 * Readings: ER_DIA = NNZ / (Ndiags M), ER_ELL = NNZ / (max_RD M); var_RD is
 * the population variance; a diagonal is "true" when 5 count > 3 length;
 * R is the least-squares power-law exponent of the row degrees.  The
 * diagonal census is only taken while DIA can still be feasible
 * (max_RD M <= 20 NNZ); otherwise ndiags = -1.  A staged plan that stopped
 * early leaves R = NaN and blocks4 = block_fill = -1 (not extracted). */
typedef struct {
    int64_t m, n, nnz;
    int64_t sum_rd, sum_rd2, max_rd, min_rd;
    int64_t ndiags, ntdiags, bandwidth, blocks4;
    double aver_rd, var_rd, std_rd, er_dia, er_ell, ntdiags_ratio, R, block_fill;
    int32_t dia_feasible, ell_feasible;
} spmv_features;

typedef struct {
    int64_t m, n, nnz;
    int32_t dtype, kernel, format, selector_used;
    float confidence;                   /* MLP margin, -1 if not used          */
    float mlp_scores[SPMV_K_COUNT];     /* predicted log slowdowns            */
    int32_t n_measured;                 /* candidates timed at plan time      */
    int32_t measured_kernel[SPMV_K_COUNT];
    double measured_ms[SPMV_K_COUNT];   /* median run time per measured kernel */
    uint32_t feasible_mask;             /* bit k: kernel k could be used      */
    spmv_features features;
    spmv_params params;                 /* parameters in effect               */
    int32_t ell_width, dia_ndiags, dia_windows;
    int64_t m_pad;
    uint64_t device_bytes;              /* plan-owned device memory           */
    double t_validate_ms, t_features_ms, t_select_ms, t_convert_ms, t_plan_ms;
    float mlp_input[12];                /* raw selector inputs of this matrix  */
    int32_t rules_kernel;               /* what SPMV_SELECT_RULES would pick   */
    int32_t out_of_domain;              /* 1: MLP inputs outside the model's
                                           training range, every feasible
                                           kernel was measured               */
    double t_tune_ms;                   /* parameter search (autotune), part
                                           of t_convert_ms and t_plan_ms      */
    int64_t bcsr_blocks;                /* stored 4x4 blocks (BCSR plans)     */
    int32_t n_segments;                 /* segmented plans: the number of row
                                           segments (kernel and format are
                                           then -1; spmv_plan_segment gives
                                           each segment's plan); else 0     */
    int32_t feature_stage;              /* 0: not staged; 1: staged, settled
                                           after the census (rest stage
                                           skipped; rules_kernel is then -1
                                           unless the rules' DIA / ELL tests
                                           decide); 2: staged, every stage
                                           ran                               */
    float stage_confidence;             /* MLP stage rule: confidence of the
                                           leaf reached, -1 if not consulted */
    int32_t tune_rejected;              /* parameter points the autotuner
                                           dropped because their output on
                                           the all-ones probe left twice the
                                           accuracy bound of the starting
                                           point's (0 when all agree)      */
    int32_t long_lanes;                 /* params.long_lds 1 or 3 in effect:
                                           lanes per long row (chunks: 32 or
                                           64; tiles: the most of any row
                                           block, 8-64), else 0             */
    int64_t long_rows;                  /* rows taken by that kernel        */
    /* opts.time_baseline = 1 (else -1): median time of one run of the plan
     * and of the plain CSR kernel on the same matrix, and the break-even
     * call count of Equation 2, t_plan_ms / (t_plain_ms - t_run_ms): the
     * number of calls after which planning has paid for itself (+inf when
     * the plan is not faster than plain CSR). */
    double t_run_ms, t_plain_ms, break_even_calls;
} spmv_plan_info;

typedef struct spmv_plan_s *spmv_plan_t;
typedef struct spmv_batch_s *spmv_batch_t;

/* Fill `opts` with defaults.  Always OK. */
spmv_status spmv_plan_opts_default(spmv_plan_opts *opts);

/* Environment overrides (an interface convention, not from the paper),
 * applied by spmv_plan_create to its options and exported so that callers
 * can see the options in effect.  Host only, no device work.
 *   SPMV_SELECTOR  rules | mlp | exhaustive | a kernel name (forced), e.g.
 *                  csr_adaptive (spmv_kernel_name); mlp is ignored, with a
 *                  note on stderr, when opts->model is NULL
 *   SPMV_TAU       confidence threshold (a float >= 0)
 *   SPMV_LOG       1 / 0: opts->log
 * Unset or empty variables leave the field alone; an unparsable value is
 * ignored with a note on stderr.  The weights file and the autotune cache
 * (SPMV_WEIGHTS, SPMV_AUTOTUNE_CACHE) belong to the Python layer.
 * EINVAL if opts is NULL. */
spmv_status spmv_plan_opts_apply_env(spmv_plan_opts *opts);

/* Validate the CSR (Section 3 input), extract features (Section 4), choose a
 * kernel (Sections 5-6), convert into plan-owned device buffers and return
 * the plan.  The caller's CSR is only read; it may be freed after return.
 * Synchronises `stream`.  Errors: EINVAL (NULL pointers, m/n/nnz < 0,
 * non-canonical CSR, force_kernel out of range or infeasible), EUNSUPPORTED
 * (nnz >= 2^31 or m, n >= 2^31), ENOMEM, EDEVICE.  On error *out = NULL. */
spmv_status spmv_plan_create(const spmv_csr *csr, const spmv_plan_opts *opts,
                             void *stream, spmv_plan_t *out);

/* y_dev[0..m) = A x_dev[0..n) (y overwritten, never accumulated into).
 * Asynchronous on `stream`, no allocation, no synchronisation.  x and y
 * must not overlap (EINVAL).  m = 0 is a no-op; n = 0 allows x_dev = NULL.
 * The result is defined for finite x: the DIA and BCSR kernels multiply
 * their zero-filled slots by x too, so an Inf or NaN in x at a column that a
 * row does not store can turn that row into NaN there, where the CSR, COO
 * and ELL kernels give the product of the stored entries only. */
spmv_status spmv_run(spmv_plan_t plan, const void *x_dev, void *y_dev, void *stream);

/* Copy the plan's report into *out (host). */
spmv_status spmv_plan_info_get(spmv_plan_t plan, spmv_plan_info *out);

/* Segment k of a segmented plan (opts.segments >= 2): its own plan, which
 * covers rows row0 .. row0 + m_k - 1 and all columns (report through
 * spmv_plan_info_get; spmv_run on it with y + row0 computes those rows).
 * The segment plan belongs to `plan` and lives as long as it; do not
 * destroy it.  EINVAL if `plan` is not segmented or k is out of range. */
spmv_status spmv_plan_segment(spmv_plan_t plan, int32_t k, spmv_plan_t *segment, int64_t *row0);

/* Release the plan and its device memory.  NULL is accepted (OK). */
spmv_status spmv_plan_destroy(spmv_plan_t plan);

/* Features only (validation included).  Synchronises `stream`. */
spmv_status spmv_features_compute(const spmv_csr *csr, spmv_features *out, void *stream);

/* spmv_features_compute for callers that cannot allocate device memory
 * (code in a serving loop or a harness that forbids hipMalloc): the same
 * validation and feature kernels, with every device buffer (flags,
 * statistics, the diagonal and row-degree histograms) taken from one fixed
 * 64 MiB device array that each GPU holds from the first call until the
 * process ends, and results read back through pageable host memory.  No
 * hipMalloc, hipFree or host-pinned allocation.  Limit: an m x n matrix
 * needs 256 + 4 (m + n - 1) + 4 (n + 2) bytes, each part rounded up to 256
 * (about m + 2n <= 16.7 million); larger matrices give SPMV_EUNSUPPORTED
 * and nothing runs.  Every call on one GPU shares the array: calls that
 * overlap on one GPU (two threads, or two streams) race; calls one after
 * another do not see each other's data.  Synchronises `stream`.  Results
 * and errors otherwise as spmv_features_compute. */
spmv_status spmv_features_compute_noalloc(const spmv_csr *csr, spmv_features *out, void *stream);

/* Test hook: rebuild CSR from the plan's internal format (CSR->X->CSR must be
 * the identity bit for bit).  Outputs are caller-owned device buffers of
 * m+1, nnz and nnz elements.  Synchronises `stream`. */
spmv_status spmv_convert_roundtrip(spmv_plan_t plan, int32_t *row_ptr_dev, int32_t *col_dev,
                                   void *val_dev, void *stream);

/* Layout export for parity tests: copy one internal array of the plan into
 * the caller's device buffer `dst_dev` of `bytes` bytes.  `which`:
 *   0 COO row indices (int32, nnz)     1 ELL columns (int32, K*m_pad)
 *   2 ELL values (K*m_pad)             3 DIA offsets (int32, D)
 *   4 DIA values (D*m_pad)             5 DIA presence bits (uint32 words)
 *   6 CSR-adaptive row order (int32, m)
 *   7 BCSR block row pointer (int32, ceil(m/4)+1)
 *   8 BCSR block columns (int32, blocks)
 *   9 BCSR values (16 per block, row-major within the block)
 *  10 BCSR presence bits (uint32 words; bit 16 k + 4 r + c: entry (r, c) of
 *     block k is stored, so explicit zeros survive the round trip)
 * EINVAL if the plan has no such array or `bytes` is too small.  On success
 * *bytes_out (if not NULL) receives the array size.  Synchronises. */
spmv_status spmv_plan_export(spmv_plan_t plan, int32_t which, void *dst_dev, size_t bytes,
                             size_t *bytes_out, void *stream);

/* Learned selector (the Section 5 data-mining model, here a 12-64-64-C
 * multilayer perceptron).  `params` holds n_params float32 weights in the
 * order W1 (64x12), b1, W2 (64x64), b2, W3 (Cx64), b3, row-major, with C =
 * SPMV_K_COUNT; `mean` and `std` are the 12 input standardisation constants.
 * Inputs are the raw features [m, nnz, aver_RD, max_RD, std_RD, Ndiags (nnz
 * when not taken), NNZ/(Ndiags m), 1 - ER_ELL, R, bandwidth, block_fill,
 * is_f64] with log1p applied to indices 0-5 and 9 before standardisation.
 * Copies everything to the device.  Synchronous. */
spmv_status spmv_selector_create(const float *params, int64_t n_params, const float *mean,
                                 const float *std, spmv_selector_t *out);
spmv_status spmv_selector_destroy(spmv_selector_t sel);

/* Training domain of a selector: `lo` and `hi` are host arrays of the 12 raw
 * inputs' smallest and largest values over the matrices the model was fitted
 * on (copied; both NULL clears the domain).  A matrix whose raw inputs leave
 * [lo, hi] in any coordinate is outside what the model has seen, so its
 * scores are not trusted whatever their margin: plan creation then measures
 * every feasible kernel, as when the margin falls below the confidence
 * threshold (Section 5, the execute-and-measure step for uncertain
 * predictions), and reports out_of_domain = 1.  EINVAL if only one pointer
 * is NULL or lo[i] > hi[i]. */
spmv_status spmv_selector_set_domain(spmv_selector_t sel, const float *lo, const float *hi);

/* Stage rule of a selector (Section 6: the format search runs format by
 * format, DIA first, and stops once a format's rules are confident): a
 * binary decision tree over the raw inputs known after the diagonal census,
 * inputs 0-7, 9 and 11 (spmv_plan_info.mlp_input order).  Node i < n_nodes
 * with feat[i] >= 0 sends raw[feat[i]] <= thr[i] to node left[i], else to
 * right[i]; a leaf (feat[i] = -1) names kernel[i] with confidence conf[i] in
 * [0, 1] (the share of its training matrices on which that kernel ran within
 * 5% of the fastest).  Node 0 is the root; child indices must exceed their
 * parent's.  Host arrays of n_nodes entries, copied (thr, left and right of
 * leaves are ignored).  n_nodes = 0 removes the rule.  Used by plans created
 * with opts.staged = 1.  EINVAL on NULL arrays with n_nodes > 0, n_nodes
 * outside [0, 4096], an input other than those listed, a child out of
 * order or range, a kernel out of range or a confidence outside [0, 1]. */
spmv_status spmv_selector_set_stage(spmv_selector_t sel, const int32_t *feat, const float *thr,
                                    const int32_t *left, const int32_t *right,
                                    const int32_t *kernel, const float *conf, int32_t n_nodes);

/* Score raw feature rows with the selector on the GPU (inference kernel):
 * raw_dev is float32 [rows x 12], scores_dev float32 [rows x SPMV_K_COUNT]. */
spmv_status spmv_selector_score(spmv_selector_t sel, const float *raw_dev, int64_t rows,
                                float *scores_dev, void *stream);

/* Selector training kernels (float32, batch-major).  Shapes: x_dev [B x 12]
 * already standardised, target_dev and mask_dev [B x C], params_dev / grad_dev
 * / adam_m_dev / adam_v_dev [n_params] in the spmv_selector_create order,
 * scores_dev [B x C], workspace_dev of spmv_mlp_workspace_floats(B) floats.
 * spmv_mlp_forward   : scores = net(x)
 * spmv_mlp_backward  : grad = d loss / d params of the masked mean squared
 *                      error sum mask (s - t)^2 / max(1, sum mask); also
 *                      writes the loss to *loss_dev (one float)
 * spmv_mlp_adam      : Adam step t >= 1 with bias correction.
 * All asynchronous on `stream`. */
int64_t spmv_mlp_param_count(int32_t n_out);
int64_t spmv_mlp_workspace_floats(int64_t batch);
spmv_status spmv_mlp_forward(const float *params_dev, int32_t n_out, const float *x_dev,
                             int64_t batch, float *scores_dev, float *workspace_dev, void *stream);
spmv_status spmv_mlp_backward(const float *params_dev, int32_t n_out, const float *x_dev,
                              const float *target_dev, const float *mask_dev, int64_t batch,
                              float *grad_dev, float *loss_dev, float *workspace_dev, void *stream);
spmv_status spmv_mlp_adam(float *params_dev, const float *grad_dev, float *adam_m_dev,
                          float *adam_v_dev, int64_t n_params, int32_t step, float lr,
                          float beta1, float beta2, float eps, void *stream);

/* Multilevel batch (the AMG setting of Section 1), or any set of independent
 * SpMVs: run y_l = A_l x_l for all plans in one launch (mode 0, persistent
 * work-queue kernel) or as one captured HIP graph (mode 1).  Plans stay
 * owned by the caller and must outlive the batch.  Persistent mode covers
 * CSR_SCALAR, CSR_VECTOR, CSR_ADAPTIVE (unless rows were split into
 * segments or long rows use their own kernel), ELL, DIA, DIA_DIRECT and
 * BCSR levels, each with its plan's tile shape, in a kernel compiled for
 * just the level kinds present; levels with other kernels are launched
 * separately on the same stream, after the persistent kernel.  Mode 0 takes
 * 1..4096 plans of one dtype (a run whose vectors differ from the previous
 * run's uploads the new pointers and waits for that copy); mode 1 takes
 * 1..4096 plans of any dtypes and kernels (every spmv_run of the batch, in
 * order, captured on the first run and again whenever the vectors change).
 * EINVAL otherwise. */
spmv_status spmv_batch_create(const spmv_plan_t *plans, int32_t nplans, int32_t mode,
                              spmv_batch_t *out);
spmv_status spmv_batch_run(spmv_batch_t batch, const void *const *xs_dev, void *const *ys_dev,
                           void *stream);
/* Autotune the persistent launch: time grids of 1, 2, 4, 8 and 16 workgroups
 * per compute unit, each with 0, 1 or 2 of the leading levels run as their
 * own kernels before the persistent launch (a level large enough to fill the
 * GPU alone keeps its own tuned kernel; at least one level stays in the
 * persistent launch), on the given vectors (outputs are overwritten), and
 * keep the fastest; *grid_out (if not NULL) receives the chosen grid.  No-op
 * for graph mode.  Synchronises `stream`. */
spmv_status spmv_batch_tune(spmv_batch_t batch, const void *const *xs_dev, void *const *ys_dev,
                            int32_t reps, void *stream, int32_t *grid_out);
/* Persistent-mode launch shape in effect: workgroups of the persistent launch
 * and the number of leading levels launched on their own (both 0 in graph
 * mode).  Either pointer may be NULL. */
spmv_status spmv_batch_shape(spmv_batch_t batch, int32_t *grid, int32_t *split);
spmv_status spmv_batch_destroy(spmv_batch_t batch);

/* Achievable-bandwidth probe: dst_dev[i] = src_dev[i] for `bytes` bytes
 * (multiple of 16, 16-byte aligned).  Asynchronous. */
spmv_status spmv_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, void *stream);

/* Read-dominant bandwidth probe, the traffic shape of SpMV (the matrix is
 * read, y is a small fraction written): streams `bytes` bytes of src_dev
 * (multiple of 16, 16-byte aligned) with 16-byte non-temporal loads and
 * writes one 16-byte word per thread of a fixed grid to out_dev (the
 * 32-bit words of the thread's loads added, so no load can be dropped);
 * out_dev must hold spmv_stream_read_out_bytes() bytes.  Asynchronous. */
spmv_status spmv_stream_read(const void *src_dev, size_t bytes, void *out_dev, void *stream);
size_t spmv_stream_read_out_bytes(void);

/* Random-gather ceiling probe, the memory pattern of a CSR row loop (a
 * coalesced value stream, a coalesced index stream and one gather per
 * entry) without row pointers or y: thread t of a fixed grid of
 * spmv_gather_probe_threads() threads writes out_dev[t] = the sum, in
 * order, of val_dev[i] * table_dev[idx_dev[i]] over i = t, t + G, t + 2G, ...
 * < count (G the thread count), products and sum in float64, rounded once
 * to the element type.  elt = 4 (float32 table, val and out) or 8
 * (float64).  idx values must lie in [0, table_len).  Device buffers,
 * caller-owned; asynchronous.  EINVAL on NULL buffers with count > 0, a bad
 * elt, count < 0 or table_len < 1. */
spmv_status spmv_gather_probe(const void *table_dev, int64_t table_len, const int32_t *idx_dev,
                              const void *val_dev, int64_t count, int32_t elt, void *out_dev,
                              void *stream);
int64_t spmv_gather_probe_threads(void);

/* Readable name of a status, and the calling thread's last error text. */
const char *spmv_status_string(spmv_status s);
const char *spmv_last_error(void);
const char *spmv_kernel_name(int32_t kernel);

#ifdef __cplusplus
}
#endif
#endif /* SMAT_SPMV_H */
