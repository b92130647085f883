// C-ABI of the adaptive SpMV library: plan creation (validation, feature
// extraction, kernel selection, conversion) and the run entry point.
//
// Plan creation follows the runtime stage of the paper (Section 6): extract
// features (Section 4), search the format (rules in the order DIA, ELL, CSR,
// COO, or the learned model of Section 5), execute-and-measure candidates
// when the model is not confident, then keep the chosen format and kernel
// ("kernel library" of Section 3) in plan-owned device memory.
#include "plan.hpp"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>

namespace smat {

namespace {
thread_local char g_err[1024] = "";
}

thread_local spmv_allocator g_alloc{};

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

spmv_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SPMV_ENOMEM : SPMV_EDEVICE;
}

namespace {

int elt_of(int dtype) { return dtype == SPMV_F64 ? 8 : 4; }

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int pow2_ceil(int64_t v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

#define SMAT_TRY(expr)                              \
    do {                                            \
        spmv_status _s = (expr);                    \
        if (_s != SPMV_OK) return _s;               \
    } while (0)

__global__ void k_gather_rowptr(int64_t count, const int32_t *__restrict__ rows,
                                const int32_t *__restrict__ rp, int64_t *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t r = rows[i];
    out[2 * i] = rp[r];
    out[2 * i + 1] = rp[r + 1];
}

__global__ void k_fill_one(int64_t n, int elt, void *x) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (elt == 8)
        ((double *)x)[i] = 1.0;
    else
        ((float *)x)[i] = 1.0f;
}

// Row sums of |a_ij|: (|A||x|)_i for the all-ones probe vector.
template <typename T>
__global__ void k_row_abs_sum(int64_t m, const int32_t *__restrict__ rp,
                              const T *__restrict__ val, double *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += fabs((double)val[p]);
    out[i] = s;
}

// Sets *bad unless |y_i - ref_i| <= tol (|A||x|)_i for every row (a NaN
// difference counts as a disagreement).
template <typename T>
__global__ void k_tune_check(int64_t m, const T *__restrict__ y, const T *__restrict__ ref,
                             const double *__restrict__ absrow, double tol, unsigned *bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double d = fabs((double)y[i] - (double)ref[i]);
    if (!(d <= tol * absrow[i])) atomicOr(bad, 1u);
}

}  // namespace
}  // namespace smat

using namespace smat;

namespace smat {
namespace {

// ------------------------------------------------------------------ features

struct FeatureWork {
    Dev scratch;   // RowStats + EntryStats + DiagStats + flags + fit sums
    Dev row_hist;
    Dev diag_hist; // m + n - 1 bins; later the diagonal -> slot map
    bool census = false;       // the census was taken (DIA could be feasible)
    bool census_done = false;  // the census question is settled
    // Allocation-free mode: the three buffers are carved out of a device
    // region the caller owns (FeatureArena layout for this matrix) and
    // results come back through pageable host memory.
    unsigned char *arena = nullptr;
    size_t arena_bytes = 0;
    size_t arena_row_off = 0;
    // buffer k (0 scratch, 1 diag_hist, 2 row_hist) of `bytes` bytes
    spmv_status take(int k, size_t bytes);
};

// Layout of the allocation-free region for an m x n matrix: the scratch
// block, the m + n - 1 diagonal bins and up to n + 1 row-degree bins
// (max_RD <= n), each 256-byte aligned.
struct FeatureArena {
    static size_t align(size_t b) { return (b + 255) / 256 * 256; }
    static constexpr size_t kDiagOffset = 256;
    static size_t row_offset(int64_t m, int64_t n) {
        return kDiagOffset + align(sizeof(unsigned) * (size_t)std::max<int64_t>(1, m + n - 1));
    }
    static size_t total(int64_t m, int64_t n) {
        return row_offset(m, n) + align(sizeof(unsigned) * (size_t)(n + 2));
    }
};

spmv_status FeatureWork::take(int k, size_t bytes) {
    Dev &d = k == 0 ? scratch : k == 1 ? diag_hist : row_hist;
    if (!arena) return d.alloc(bytes);
    const size_t off = k == 0 ? 0 : k == 1 ? FeatureArena::kDiagOffset : arena_row_off;
    const size_t end = k == 0 ? FeatureArena::kDiagOffset : k == 1 ? arena_row_off : arena_bytes;
    if (off + bytes > end) {
        set_error("feature buffer %d of %zu bytes exceeds its part of the region", k, bytes);
        return SPMV_EUNSUPPORTED;
    }
    d.borrow(arena + off, bytes);
    return SPMV_OK;
}

// Matrices with at most this many diagonal bins (m + n - 1) take the census
// together with the CSR checks, gated on the device by their outcome: one
// synchronisation less, for a histogram small enough to clear in passing.
constexpr int64_t kCensusWithChecksBins = int64_t(1) << 22;

struct Scratch {
    RowStats rs;
    EntryStats es;
    DiagStats ds;
    uint32_t flags;    // row_ptr check
    uint32_t flags2;   // column checks
    double fit[5];
};
static_assert(sizeof(Scratch) <= FeatureArena::kDiagOffset, "scratch block fits its slot");

// The scratch zeroed (min_rd at INT_MAX) by one small kernel rather than a
// copy from pageable host memory.
__global__ void k_init_scratch(Scratch *d) {
    unsigned *w = reinterpret_cast<unsigned *>(d);
    for (unsigned i = threadIdx.x; i < sizeof(Scratch) / sizeof(unsigned); i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) d->rs.min_rd = INT_MAX;
}

// The scratch read back into pinned host memory (one block per thread, kept
// for the process), which the copy engine writes directly; NULL if pinned
// memory is unavailable (a stack copy is used then).
Scratch *pinned_scratch() {
    thread_local Scratch *p = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc(reinterpret_cast<void **>(&p), sizeof(Scratch), hipHostMallocDefault) !=
            hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
        }
    }
    return p;
}

spmv_status read_scratch(const Scratch *d, Scratch &h, hipStream_t s, bool pinned_ok = true) {
    Scratch *pin = pinned_ok ? pinned_scratch() : nullptr;
    Scratch *dst = pin ? pin : &h;
    SMAT_HIP(hipMemcpyAsync(dst, d, sizeof(Scratch), hipMemcpyDeviceToHost, s));
    SMAT_HIP(hipStreamSynchronize(s));
    if (pin) h = *pin;
    return SPMV_OK;
}

// Feature extraction in stages, in the order the format search consumes them
// (Section 6: DIA first, then ELL and CSR, COO last):
//   rows    validation, row statistics and bandwidth -- everything the ELL
//           and CSR tests need;
//   census  the diagonal histogram (Ndiags, NTdiags, ER_DIA), taken only
//           while DIA can still be feasible;
//   rest    the row-degree histogram with the power-law fit (R, the COO
//           trigger) and the 4x4 block count.
// Without staging, census and rest share one entry pass and one
// synchronisation.
enum : unsigned { kStageCensus = 1, kStageRest = 2 };

void set_census(spmv_features &F, const DiagStats &ds, int64_t m, int64_t nnz, FeatureWork &W) {
    W.census = true;
    F.ndiags = (int64_t)ds.ndiags;
    F.ntdiags = (int64_t)ds.ntrue;
    F.ntdiags_ratio = F.ndiags ? (double)F.ntdiags / (double)F.ndiags : 0.0;
    F.er_dia = F.ndiags ? (double)nnz / ((double)F.ndiags * (double)m) : 0.0;
    F.dia_feasible = (__int128)F.ndiags * m <= (__int128)20 * nnz;
}

spmv_status extract_rows(const spmv_csr &A, hipStream_t s, spmv_features &F, FeatureWork &W) {
    const int64_t m = A.m, n = A.n, nnz = A.nnz;
    SMAT_TRY(W.take(0, sizeof(Scratch)));
    Scratch *d = W.scratch.as<Scratch>();
    Scratch h{};
    k_init_scratch<<<1, 64, 0, s>>>(d);
    SMAT_LAUNCHED("init_scratch");
    // the row_ptr check, the column checks (with the bandwidth) and the row
    // pass share one synchronisation: the column and row passes stay in
    // bounds whatever row_ptr holds, and their results are only used when
    // the row_ptr check passes
    SMAT_TRY(launch_validate_rows(m, nnz, A.row_ptr_dev, &d->flags, s));
    SMAT_TRY(launch_validate_entries(m, n, nnz, A.row_ptr_dev, A.col_dev, &d->flags2,
                                     &d->es.bandwidth, s));
    SMAT_TRY(launch_row_stats(m, A.row_ptr_dev, &d->rs, s));
    // small matrices: the census too, run on the device only if the checks
    // pass and DIA can still be feasible
    const bool with_census = nnz > 0 && m + n - 1 <= kCensusWithChecksBins;
    if (with_census) {
        SMAT_TRY(W.take(1, sizeof(unsigned) * (size_t)(m + n - 1)));
        SMAT_HIP(hipMemsetAsync(W.diag_hist.p, 0, W.diag_hist.bytes, s));
        SMAT_TRY(launch_entry_stats(m, n, nnz, A.row_ptr_dev, A.col_dev, &d->es,
                                    W.diag_hist.as<unsigned>(), false, s, &d->flags, &d->rs));
        SMAT_TRY(launch_diag_stats(m, n, W.diag_hist.as<unsigned>(), &d->ds, s));
    }
    SMAT_TRY(read_scratch(d, h, s, W.arena == nullptr));
    if (h.flags) {
        set_error("invalid CSR row_ptr (flags 0x%x: %s%s%s)", h.flags,
                  (h.flags & kBadRowPtr0) ? "row_ptr[0] != 0 " : "",
                  (h.flags & kBadRowPtrEnd) ? "row_ptr[m] != nnz " : "",
                  (h.flags & kBadRowPtrOrder) ? "row_ptr decreasing or out of range" : "");
        return SPMV_EINVAL;
    }
    h.flags = h.flags2;
    if (h.flags) {
        set_error("invalid CSR columns (flags 0x%x: %s%s)", h.flags,
                  (h.flags & kBadColRange) ? "column out of [0, n) " : "",
                  (h.flags & kBadColOrder) ? "columns not strictly increasing in a row" : "");
        return SPMV_EINVAL;
    }
    F = spmv_features{};
    F.m = m;
    F.n = n;
    F.nnz = nnz;
    F.sum_rd = (int64_t)h.rs.sum_rd;
    F.sum_rd2 = (int64_t)h.rs.sum_rd2;
    F.max_rd = m ? h.rs.max_rd : 0;
    F.min_rd = m ? h.rs.min_rd : 0;
    F.aver_rd = m ? (double)nnz / (double)m : 0.0;
    if (m) {
        __int128 num = (__int128)m * (__int128)F.sum_rd2 - (__int128)F.sum_rd * F.sum_rd;
        F.var_rd = (double)num / ((double)m * (double)m);
    }
    F.std_rd = std::sqrt(F.var_rd);
    F.er_ell = F.max_rd ? (double)nnz / ((double)F.max_rd * (double)m) : 0.0;
    F.ell_feasible = m && (__int128)F.max_rd * m <= (__int128)20 * nnz;
    F.bandwidth = h.es.bandwidth;
    // not extracted yet
    F.ndiags = -1;
    F.blocks4 = -1;
    F.block_fill = -1.0;
    F.R = std::numeric_limits<double>::quiet_NaN();
    if (with_census) {
        W.census_done = true;
        if (F.ell_feasible) set_census(F, h.ds, m, nnz, W);
        if (!F.dia_feasible) W.diag_hist.release();
    }
    return SPMV_OK;
}

spmv_status extract_entries(const spmv_csr &A, hipStream_t s, spmv_features &F, FeatureWork &W,
                            unsigned what, bool keep_census) {
    const int64_t m = A.m, n = A.n, nnz = A.nnz;
    Scratch *d = W.scratch.as<Scratch>();
    const bool rest = what & kStageRest;
    // ---- power-law fit over the row-degree histogram
    if (rest && m && F.max_rd >= 1) {
        SMAT_TRY(W.take(2, sizeof(unsigned) * (size_t)(F.max_rd + 1)));
        SMAT_HIP(hipMemsetAsync(W.row_hist.p, 0, W.row_hist.bytes, s));
        SMAT_TRY(launch_row_hist(m, A.row_ptr_dev, (int)F.max_rd, W.row_hist.as<unsigned>(), s));
        SMAT_TRY(launch_powerlaw_fit(W.row_hist.as<unsigned>(), (int)F.max_rd, m, d->fit, s));
    }
    // ---- entry pass: diagonal census (while DIA may still be feasible,
    // since Ndiags >= max_RD) and / or the 4x4 block count
    const bool census = (what & kStageCensus) && !W.census_done && F.ell_feasible && nnz > 0;
    if (census) {
        SMAT_TRY(W.take(1, sizeof(unsigned) * (size_t)(m + n - 1)));
        SMAT_HIP(hipMemsetAsync(W.diag_hist.p, 0, W.diag_hist.bytes, s));
    }
    if (census || rest)
        SMAT_TRY(launch_entry_stats(m, n, nnz, A.row_ptr_dev, A.col_dev, &d->es,
                                    census ? W.diag_hist.as<unsigned>() : nullptr, rest, s));
    if (census) SMAT_TRY(launch_diag_stats(m, n, W.diag_hist.as<unsigned>(), &d->ds, s));
    Scratch h{};
    SMAT_TRY(read_scratch(d, h, s, W.arena == nullptr));
    if (rest) {
        F.blocks4 = (int64_t)h.es.blocks4;
        F.block_fill = F.blocks4 ? (double)nnz / (16.0 * (double)F.blocks4) : 0.0;
        F.R = (m && F.max_rd >= 1 && h.fit[0] >= 2.0 && h.fit[4] > 0) ? -h.fit[3] / h.fit[4]
                                                                     : 0.0;
    }
    if (census) {
        set_census(F, h.ds, m, nnz, W);
    } else if ((what & kStageCensus) && !W.census_done) {
        F.ndiags = -1;
        F.ntdiags = 0;
        F.ntdiags_ratio = 0.0;
        F.er_dia = 0.0;
        F.dia_feasible = 0;
    }
    if (what & kStageCensus) W.census_done = true;
    if (!keep_census || !F.dia_feasible) W.diag_hist.release();
    W.row_hist.release();
    return SPMV_OK;
}

// All features up front (no staging).
spmv_status validate_and_extract(const spmv_csr &A, hipStream_t s, spmv_features &F,
                                 FeatureWork &W, bool keep_census, double *t_val,
                                 double *t_feat) {
    auto t0 = std::chrono::steady_clock::now();
    SMAT_TRY(extract_rows(A, s, F, W));
    auto t1 = std::chrono::steady_clock::now();
    SMAT_TRY(extract_entries(A, s, F, W, kStageCensus | kStageRest, keep_census));
    auto t2 = std::chrono::steady_clock::now();
    if (t_val) *t_val = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (t_feat) *t_feat = std::chrono::duration<double, std::milli>(t2 - t1).count();
    return SPMV_OK;
}

// ------------------------------------------------------------------ params

int default_lanes(const spmv_features &F) {
    // about four entries per lane for a row of mean length: enough loads per
    // lane in flight, few idle lanes
    int L = pow2_ceil((int64_t)std::ceil(F.aver_rd)) / 4;
    return std::max(1, std::min(64, L));
}

spmv_params default_params(int kernel, const spmv_features &F) {
    // Sizes that keep a few thousand workgroups in flight on 256 compute
    // units: small matrices get small workgroups and tiles.
    spmv_params p{};
    p.block = F.m >= (512 << 10) ? 256 : F.m >= (64 << 10) ? 128 : 64;
    p.vector_lanes = default_lanes(F);
    p.adaptive_rows_per_lane = 2;
    p.adaptive_wg_min = 4096;
    p.dia_rows_per_thread = F.m >= (4 << 20) ? 4 : F.m >= (1 << 20) ? 2 : 1;
    p.dia_span = 64;
    p.coo_chunk = F.nnz >= (8 << 20) ? 8 : F.nnz >= (1 << 20) ? 4 : 2;
    p.ell_unroll = 4;
    p.stream_nt = 0;  // resolved per kernel by resolve_params
    p.panel_kib = 4096;
    p.panel_xcd = 1;
    (void)kernel;
    return p;
}

constexpr int kXcds = 8;  // gfx950: eight accelerator complex dies, one L2 each
// Column panels: rows of at most this many entries are summed without panels
// by default (-1: none).
constexpr int kPanelDirectMaxDefault = -1;
// Long-row tiles take the rows longer than this by default (params.tile_row_min).
constexpr int kTileRowMin = 1024;
constexpr int64_t kDiaLdsMax = 64 * 1024;  // dynamic LDS of one DIA workgroup

// Column-panel geometry: width w columns (a multiple of 64) and panel count P.
// XCD mode: P = 8 G panels, G the fewest groups of eight whose panels hold
// at most panel_kib KiB of x (trailing panels may be empty); sequential
// mode: x bytes per panel <= panel_kib KiB.
void panel_geometry(const spmv_features &F, int elt, const spmv_params &p, int64_t *w, int *P) {
    const int64_t kib = std::max<int64_t>(1, p.panel_kib);
    if (p.panel_xcd != 2) {
        const int64_t xbytes = std::max<int64_t>(1, F.n) * elt;
        const int64_t G = std::min<int64_t>((xbytes + kXcds * kib * 1024 - 1) / (kXcds * kib * 1024),
                                            (1 << 20) / kXcds);
        int64_t width = ((std::max<int64_t>(1, F.n) + kXcds * G - 1) / (kXcds * G) + 63) / 64 * 64;
        *w = std::max<int64_t>(64, width);
        *P = (int)(kXcds * G);
        return;
    }
    int64_t width = (kib * 1024 / elt) / 64 * 64;
    if (width < 64) width = 64;
    *w = width;
    *P = (int)std::min<int64_t>((F.n + width - 1) / width, 1 << 20);
}

// Fill in the per-kernel defaults left open (0) in `p`.  Streaming loads pay
// off for the fully coalesced ELL and DIA streams of banded matrices, whose x
// is reused through the cache; the CSR kernels revisit partly consumed cache
// lines and random gathers from a large x do better with the default policy
// (measured on gfx950).
spmv_params resolve_params(int kernel, spmv_params p, const spmv_features &F, int elt) {
    if (p.stream_nt == 0) {
        bool dense_stream = kernel == SPMV_K_ELL || kernel == SPMV_K_DIA ||
                            kernel == SPMV_K_DIA_DIRECT;
        p.stream_nt = (dense_stream && F.dia_feasible) ? 1 : 2;
    }
    // 16-byte streams pay off once a quarter or half as many lanes still fill
    // the chip many times over (measured: faster from about a million rows,
    // slower on smaller matrices)
    if (p.wide_loads == 0) p.wide_loads = F.m >= (1 << 20) ? 1 : 2;
    if (p.panel_direct_max == 0) p.panel_direct_max = kPanelDirectMaxDefault;
    if (p.tile_row_min == 0) p.tile_row_min = kTileRowMin;
    if (p.bcsr_lanes == 0) {
        const int64_t mb = std::max<int64_t>(1, (F.m + 3) / 4);
        const int64_t avg = (std::max<int64_t>(0, F.blocks4) + mb - 1) / mb;
        const int per_row = std::max(1, std::min(64, pow2_ceil(std::max<int64_t>(1, avg))));
        if (elt == 8)
            // one block of the row at a time by its 8 lanes once the block
            // rows alone fill the GPU (measured best on dense 4x4 block
            // matrices from 2^16 block rows); below, a lane group per block
            p.bcsr_lanes = mb >= (1 << 16) ? 8 : std::min(64, 8 * per_row);
        else
            // about one block per lane for a block row of mean length
            p.bcsr_lanes = per_row;
    }
    return p;
}

void merge_params(spmv_params &p, const spmv_params &u) {
    if (u.block > 0) p.block = u.block;
    if (u.vector_lanes > 0) p.vector_lanes = u.vector_lanes;
    if (u.adaptive_rows_per_lane > 0) p.adaptive_rows_per_lane = u.adaptive_rows_per_lane;
    if (u.adaptive_wg_min > 0) p.adaptive_wg_min = u.adaptive_wg_min;
    if (u.dia_rows_per_thread > 0) p.dia_rows_per_thread = u.dia_rows_per_thread;
    if (u.dia_span > 0) p.dia_span = u.dia_span;
    if (u.coo_chunk > 0) p.coo_chunk = u.coo_chunk;
    if (u.ell_unroll > 0) p.ell_unroll = u.ell_unroll;
    if (u.stream_nt > 0) p.stream_nt = u.stream_nt;
    if (u.panel_kib > 0) p.panel_kib = u.panel_kib;
    if (u.panel_xcd > 0) p.panel_xcd = u.panel_xcd;
    if (u.wide_loads > 0) p.wide_loads = u.wide_loads;
    if (u.bcsr_lanes > 0) p.bcsr_lanes = u.bcsr_lanes;
    if (u.long_lds > 0) p.long_lds = u.long_lds;
    if (u.tile_row_min > 0) p.tile_row_min = u.tile_row_min;
    if (u.panel_direct_max != 0) p.panel_direct_max = u.panel_direct_max;
}

spmv_status check_params(const spmv_params &p) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!(p.block >= 64 && p.block <= 1024 && p.block % 64 == 0)) {
        set_error("params.block must be a multiple of 64 in [64, 1024]");
        return SPMV_EINVAL;
    }
    if (!(pow2(p.vector_lanes) && p.vector_lanes <= 64)) {
        set_error("params.vector_lanes must be a power of two <= 64");
        return SPMV_EINVAL;
    }
    if (p.adaptive_rows_per_lane < 1 || p.adaptive_rows_per_lane > 64 ||
        p.adaptive_wg_min < 64 || p.adaptive_wg_min > (1 << 20)) {
        set_error("params.adaptive_* out of range");
        return SPMV_EINVAL;
    }
    if (!(p.dia_rows_per_thread == 1 || p.dia_rows_per_thread == 2 ||
          p.dia_rows_per_thread == 4 || p.dia_rows_per_thread == 8) ||
        p.dia_span < 0 || p.dia_span > 8192) {
        set_error("params.dia_rows_per_thread must be 1, 2, 4 or 8 and dia_span in [0, 8192]");
        return SPMV_EINVAL;
    }
    if (p.coo_chunk < 1 || p.coo_chunk > 64) {
        set_error("params.coo_chunk must be in [1, 64]");
        return SPMV_EINVAL;
    }
    if (!(p.ell_unroll == 1 || p.ell_unroll == 2 || p.ell_unroll == 4)) {
        set_error("params.ell_unroll must be 1, 2 or 4");
        return SPMV_EINVAL;
    }
    if (p.stream_nt < 0 || p.stream_nt > 2) {
        set_error("params.stream_nt must be 0 (default), 1 (on) or 2 (off)");
        return SPMV_EINVAL;
    }
    if (p.panel_kib < 1 || p.panel_kib > (1 << 20) || p.panel_xcd < 0 || p.panel_xcd > 2) {
        set_error("params.panel_kib must be in [1, 2^20] and panel_xcd 0, 1 or 2");
        return SPMV_EINVAL;
    }
    if (p.wide_loads < 0 || p.wide_loads > 2) {
        set_error("params.wide_loads must be 0 (default), 1 (on) or 2 (off)");
        return SPMV_EINVAL;
    }
    if (p.long_lds < 0 || p.long_lds > 3) {
        set_error("params.long_lds must be 0 (default), 1 (x chunks), 2 (off) or 3 (tiles)");
        return SPMV_EINVAL;
    }
    if (p.tile_row_min != 0 && (p.tile_row_min < 64 || p.tile_row_min > (1 << 20))) {
        set_error("params.tile_row_min must be 0 (default) or in [64, 2^20]");
        return SPMV_EINVAL;
    }
    if (p.panel_direct_max < -1 || p.panel_direct_max > (1 << 20)) {
        set_error("params.panel_direct_max must be -1 (none), 0 (default) or a row length "
                  "up to 2^20");
        return SPMV_EINVAL;
    }
    if (p.bcsr_lanes != 0 && !(pow2(p.bcsr_lanes) && p.bcsr_lanes <= 64)) {
        set_error("params.bcsr_lanes must be 0 (default) or a power of two <= 64");
        return SPMV_EINVAL;
    }
    return SPMV_OK;
}

// Longest float64 summation chain of a BCSR lane with L lanes per block
// row (the float64 kernel: 8 lanes per block): 2 products per block for
// ceil(4 max_RD / G) blocks (G = L / 8 lane groups), then 1 + log2 G
// shuffled additions.
int64_t bcsr_f64_depth(int64_t max_rd, int L) {
    const int64_t G = std::max(1, L / 8);
    return 2 * ((4 * max_rd + G - 1) / G) + 1 + ilog2((int)G);
}

// Longest COO chain: a row spans at most this many chunks in float64.
constexpr int64_t kCooMaxChunksPerRow = 3000;
constexpr int64_t kSplitSegment = 512 * 1024;   // entries per split segment (512 threads)
constexpr int64_t kSplitMin = 256 * 4000;       // longer rows than this are split
constexpr int64_t kTileRowsDefault = 1024;   // default: tiles from this many such rows
// Tiles: lanes per row of a row block, the fewest (at least 2^kTileLanesLog2Min)
// that give about kTileEntriesPerLane entries per lane of the block's mean
// segment (raised further where the float64 chain bound needs it).
constexpr int kTileLanesLog2Min = 3;
// Tiles are built only when their partial sums and segment starts cost at
// most 1/kTileExtraShare of the long rows' own bytes per run.
constexpr double kTileExtraShare = 5.0;
constexpr int64_t kTileMinEntries = 16384;   // per tile workgroup, at least
constexpr double kTileEntriesPerLane = 16.0;

// Kernels that can hold this matrix (zero-fill rule, storage cap) and, when
// `accuracy` is set, also keep every float64 summation chain short enough for
// the 1e-12 (|A||x|)_i bound.  A forced kernel is only held to the first part.
uint32_t feasible_mask(const spmv_features &F, int dtype, int64_t m_pad, uint64_t cap,
                       const spmv_params &p, bool accuracy = true) {
    const int elt = elt_of(dtype);
    uint32_t mask = 0;
    const bool f64 = dtype == SPMV_F64 && accuracy;
    // CSR scalar: the sequential chain is the whole row
    if (!f64 || F.max_rd <= kFp64MaxDepth) mask |= 1u << SPMV_K_CSR_SCALAR;
    // CSR vector: chain ceil(max/L) + log2 L
    {
        int L = p.vector_lanes;
        if (!f64 || (F.max_rd + L - 1) / L + ilog2(L) <= kFp64MaxDepth)
            mask |= 1u << SPMV_K_CSR_VECTOR;
    }
    mask |= 1u << SPMV_K_CSR_ADAPTIVE;
    if (F.ell_feasible) {
        uint64_t bytes = (uint64_t)F.max_rd * (uint64_t)m_pad * (uint64_t)(elt + 4);
        if (bytes <= cap && (!f64 || F.max_rd <= kFp64MaxDepth)) mask |= 1u << SPMV_K_ELL;
    }
    if (F.dia_feasible && F.ndiags >= 0) {
        uint64_t bytes = (uint64_t)F.ndiags * (uint64_t)m_pad * (uint64_t)elt +
                         (uint64_t)F.ndiags * (uint64_t)m_pad / 8;
        if (bytes <= cap && (!f64 || F.ndiags <= kFp64MaxDepth))
            mask |= (1u << SPMV_K_DIA) | (1u << SPMV_K_DIA_DIRECT);
    }
    {
        int64_t per = (int64_t)p.coo_chunk * kWave;
        if (!f64 || F.max_rd <= kCooMaxChunksPerRow * per) mask |= 1u << SPMV_K_COO;
    }
    {
        // BCSR 4x4: the zero-fill rule (Section 2.3) applied to blocks --
        // stored block slots at most 20x the entries (fill >= 5%) -- plus the
        // storage cap; float64 chains: with 64 lanes (8 groups of 8) a lane
        // adds 2 ceil(4 max_RD / 8) products (a block row has at most
        // 4 max_RD blocks) and 4 shuffled partial sums.
        const uint64_t nb = (uint64_t)std::max<int64_t>(0, F.blocks4);
        const uint64_t mb = (uint64_t)(F.m + 3) / 4;
        const uint64_t bytes = nb * (uint64_t)(16 * elt + 6) + 4u * (mb + 1);
        bool ok = nb > 0 && 16u * nb <= 20u * (uint64_t)F.nnz && bytes <= cap &&
                  16u * nb < (1ull << 31);
        if (f64 && bcsr_f64_depth(F.max_rd, 64) > kFp64MaxDepth) ok = false;
        if (ok) mask |= 1u << SPMV_K_BCSR;
    }
    {
        // Column panels pay off only when x does not fit one panel.  In
        // sequential mode float32 rounds the running sum once per panel, so
        // at most 16 panels keep it inside 2e-6 (|A||x|)_i (XCD mode rounds
        // each panel's own partial once: at most 2^-24 sum_p |partial_p| <=
        // 2^-24 (|A||x|)_i for any P); no row may need splitting.
        int64_t w;
        int P;
        panel_geometry(F, elt, p, &w, &P);
        uint64_t bytes = (uint64_t)F.nnz * (uint64_t)(elt + 4) +
                         (uint64_t)P * (uint64_t)(F.m + 1) * 4u +
                         (p.panel_xcd != 2 ? (uint64_t)P * (uint64_t)F.m * (uint64_t)elt : 0u);
        bool ok = P >= 2 && F.nnz > 0 && F.max_rd <= kSplitMin && bytes <= cap &&
                  (uint64_t)F.n * (uint64_t)elt > (2u << 20) &&
                  (uint64_t)P * (uint64_t)(F.m + 1) < (1ull << 31);
        if (dtype == SPMV_F32 && p.panel_xcd == 2 && P > 16) ok = false;
        if (ok) mask |= 1u << SPMV_K_CSR_PANEL;
    }
    return mask;
}

// The method without the learned part: Section 4 observations as IF-THEN
// rules, tried in the Section 6 order (DIA, ELL, then COO on its only
// trigger R, CSR by default).  Integer forms of every threshold.
// The DIA and ELL tests: the part of the rule order that needs no feature of
// the rest stage.  -1 when neither applies.
int rules_dia_ell(const spmv_features &F, uint32_t feas) {
    const __int128 M = F.m, NNZ = F.nnz;
    const int64_t nd = F.ndiags;
    if ((feas & (1u << SPMV_K_DIA)) && nd >= 0 && nd <= 500) {
        if (nd < 25 || 5 * NNZ > (__int128)3 * nd * M || 5 * (__int128)F.ntdiags > 2 * (__int128)nd)
            return SPMV_K_DIA_DIRECT;  // the faster DIA implementation on gfx950
    }
    if (feas & (1u << SPMV_K_ELL)) {
        const __int128 mx = F.max_rd;
        bool er_ok = 10 * NNZ > 9 * mx * M;
        bool var_ok = 2 * (M * (__int128)F.sum_rd2 - (__int128)F.sum_rd * F.sum_rd) < M * M;
        if (er_ok && (var_ok || F.max_rd < 5)) return SPMV_K_ELL;
    }
    return -1;
}

int rules_choose(const spmv_features &F, uint32_t feas) {
    const int k = rules_dia_ell(F, feas);
    if (k >= 0) return k;
    if (F.R >= 1.0 && F.R < 4.0 && (feas & (1u << SPMV_K_COO))) return SPMV_K_COO;
    // CSR: a fixed lane width suits rows of similar length, binning otherwise
    if ((double)F.max_rd <= 8.0 * std::max(1.0, F.aver_rd) && (feas & (1u << SPMV_K_CSR_VECTOR)))
        return SPMV_K_CSR_VECTOR;
    return SPMV_K_CSR_ADAPTIVE;
}

// Kernels a staged search may settle on before the rest stage (DIA, ELL and
// CSR come before COO in the search order; BCSR's feasibility needs the
// block count) and the selector inputs known by then (all but R, 8, and the
// block fill, 10).
constexpr uint32_t kStageKernels =
    (1u << SPMV_K_CSR_SCALAR) | (1u << SPMV_K_CSR_VECTOR) | (1u << SPMV_K_CSR_ADAPTIVE) |
    (1u << SPMV_K_CSR_PANEL) | (1u << SPMV_K_ELL) | (1u << SPMV_K_DIA) | (1u << SPMV_K_DIA_DIRECT);
constexpr uint32_t kStageInputs = 0xFFFu & ~((1u << 8) | (1u << 10));
// ... and those known before the census (all but Ndiags, 5, and the DIA fill, 6)
constexpr uint32_t kRowInputs = kStageInputs & ~((1u << 5) | (1u << 6));

// Leaf of the selector's stage rule reached by these inputs (node 0 is the
// root; every child index exceeds its parent's, so the walk ends).
int stage_leaf(const spmv_selector_s &S, const float raw[12]) {
    int i = 0;
    while (S.st_feat[i] >= 0) i = raw[S.st_feat[i]] <= S.st_thr[i] ? S.st_left[i] : S.st_right[i];
    return i;
}

void raw_features(const spmv_features &F, int dtype, float out[12]) {
    double nd = F.ndiags >= 0 ? (double)F.ndiags : (double)F.nnz;
    double dia_fill = (nd > 0 && F.m > 0) ? (double)F.nnz / (nd * (double)F.m) : 0.0;
    double v[12] = {(double)F.m, (double)F.nnz, F.aver_rd, (double)F.max_rd, F.std_rd, nd,
                    dia_fill, 1.0 - F.er_ell, F.R, (double)F.bandwidth, F.block_fill,
                    dtype == SPMV_F64 ? 1.0 : 0.0};
    for (int i = 0; i < 12; ++i) out[i] = (float)v[i];
}

// ------------------------------------------------------------------ conversion

// Long rows by tiles (x panels of long_tile_width values per workgroup)
// over the long rows already in V.long_rows, longest first, of lengths len.
// Row blocks hold about four panels' worth of entries per workgroup (less
// when the grid would have under 2048 workgroups); a block's lanes per row
// (8 to 64) give about 16 entries per lane of its mean segment, raised for
// float64 until its longest segment keeps the chain bound.  Leaves
// Launch geometry of the length bins blo..bhi of a binned row order (the
// other bins get no workgroups): bin 7 a workgroup per row, bins 6..0
// 256 >> max(0, b - shift) rows per workgroup.
AdaptiveLaunch bins_launch(const unsigned bin_off[kAdaptiveBins + 1], int blo, int bhi,
                           int shift) {
    AdaptiveLaunch a{};
    unsigned blocks = 0;
    for (int q = 0; q < 8; ++q) {
        const int b = 7 - q;
        a.first[q] = blocks;
        if (b < blo || b > bhi) continue;
        const unsigned cnt = bin_off[b + 1] - bin_off[b];
        const unsigned per = b == 7 ? 1u : (unsigned)(256 >> std::max(0, b - shift));
        blocks += (cnt + per - 1) / per;
    }
    a.first[8] = blocks;
    for (int b = 0; b < 9; ++b) a.row_begin[b] = bin_off[b];
    a.lane_shift = shift;
    return a;
}

// V.long_tiles false (nothing built) when the partials and segment starts
// would cost over 1/kTileExtraShare of the long rows' own bytes per run, or
// no lane count keeps the float64 bound.
spmv_status build_long_tiles(const spmv_plan_s &P, Variant &V, const std::vector<int64_t> &len,
                             hipStream_t s) {
    const int64_t n7 = (int64_t)len.size();
    const int64_t W = long_tile_width(P.elt);
    const int64_t NP = (P.n + W - 1) / W;
    if (n7 == 0 || NP < 1 || NP > 65535) return SPMV_OK;
    int64_t total = 0;
    for (int64_t l : len) total += l;
    const double extra = 16.0 * (double)NP * n7 + 8.0 * (double)(NP + 1) * n7;
    if (extra * kTileExtraShare > (double)total * (P.elt + 4)) return SPMV_OK;
    const size_t nseg = (size_t)(n7 * (NP + 1));
    SMAT_TRY(long_tiles_prepare());
    SMAT_TRY(V.tile_seg.alloc(sizeof(int32_t) * nseg));
    SMAT_TRY(launch_long_tile_seg(n7, NP, W, V.long_rows.as<int32_t>(), P.rp.as<int32_t>(),
                                  P.col.as<int32_t>(), V.tile_seg.as<int32_t>(), s));
    std::vector<int32_t> h(nseg);
    SMAT_HIP(hipMemcpyAsync(h.data(), V.tile_seg.p, sizeof(int32_t) * nseg,
                            hipMemcpyDeviceToHost, s));
    SMAT_HIP(hipStreamSynchronize(s));
    // entries per row block (over all its panels): about four panels' worth,
    // fewer so that the grid has about 2048 workgroups, but no fewer than
    // kTileMinEntries per workgroup -- each workgroup reads a whole x panel,
    // which small blocks would not repay (measured: 5-14% faster than 2048
    // workgroups on Zipf matrices of 1.1-2.6e7 long-row entries)
    const int64_t target = std::max<int64_t>(
        1, std::min<int64_t>(4 * W * NP,
                             std::max<int64_t>(total * NP / 2048, kTileMinEntries * NP)));
    std::vector<int32_t> blocks;
    int max_tpr = 0;
    for (int64_t r0 = 0; r0 < n7;) {
        int64_t r1 = r0, acc = 0;
        while (r1 < n7 && (r1 == r0 || acc < target)) acc += len[r1++];
        int64_t maxseg = 0;
        for (int64_t p = 0; p < NP; ++p)
            for (int64_t r = r0; r < r1; ++r)
                maxseg = std::max<int64_t>(maxseg, (int64_t)h[(p + 1) * n7 + r] - h[p * n7 + r]);
        const double mean = (double)acc / ((double)(r1 - r0) * (double)NP);
        int lg = kTileLanesLog2Min;
        while (lg < 6 && kTileEntriesPerLane * (double)(1 << lg) < mean) ++lg;
        auto depth = [&](int l) { return (maxseg + (1 << l) - 1) / (1 << l) + l + NP; };
        if (P.dtype == SPMV_F64) {
            while (lg < 6 && depth(lg) > kFp64MaxDepth) ++lg;
            if (depth(lg) > kFp64MaxDepth) {
                V.tile_seg.release();
                return SPMV_OK;
            }
        }
        blocks.push_back((int32_t)r0);
        blocks.push_back((int32_t)r1);
        blocks.push_back(lg);
        max_tpr = std::max(max_tpr, 1 << lg);
        r0 = r1;
    }
    SMAT_TRY(V.tile_blocks.alloc(sizeof(int32_t) * blocks.size()));
    SMAT_HIP(hipMemcpyAsync(V.tile_blocks.p, blocks.data(), sizeof(int32_t) * blocks.size(),
                            hipMemcpyHostToDevice, s));
    SMAT_TRY(V.tile_part.alloc(sizeof(double) * (size_t)(NP * n7)));
    // The long rows' entries packed in workgroup order -- row block, panel,
    // row -- so that each workgroup streams one contiguous range: pk[k] is
    // the first packed entry of row r in panel p, k = NP r0 + p (r1 - r0) +
    // (r - r0) for the block [r0, r1) holding r, and pk[k + 1] its end.
    // NP n7 stays below total / 10 (the partials' share above), so int32.
    std::vector<int32_t> pk((size_t)(NP * n7 + 1)), kb(2 * (size_t)n7);
    int64_t pos = 0;
    for (size_t bi = 0; bi < blocks.size(); bi += 3) {
        const int64_t r0 = blocks[bi], r1 = blocks[bi + 1];
        for (int64_t p = 0; p < NP; ++p)
            for (int64_t r = r0; r < r1; ++r) {
                pk[(size_t)(NP * r0 + p * (r1 - r0) + (r - r0))] = (int32_t)pos;
                pos += (int64_t)h[(p + 1) * n7 + r] - h[p * n7 + r];
            }
        for (int64_t r = r0; r < r1; ++r) {
            kb[2 * r] = (int32_t)(NP * r0 + (r - r0));
            kb[2 * r + 1] = (int32_t)(r1 - r0);
        }
    }
    pk[(size_t)(NP * n7)] = (int32_t)pos;
    if (pos != total) {
        set_error("long-row tiles: %lld packed entries for %lld", (long long)pos,
                  (long long)total);
        return SPMV_EINVAL;
    }
    {
        Dev kbd;
        SMAT_TRY(kbd.alloc(sizeof(int32_t) * kb.size()));
        SMAT_TRY(V.tile_pk.alloc(sizeof(int32_t) * pk.size()));
        SMAT_TRY(V.tile_off.alloc(sizeof(uint16_t) * (size_t)std::max<int64_t>(1, total)));
        SMAT_TRY(V.tile_val.alloc((size_t)P.elt * (size_t)std::max<int64_t>(1, total)));
        SMAT_HIP(hipMemcpyAsync(kbd.p, kb.data(), sizeof(int32_t) * kb.size(),
                                hipMemcpyHostToDevice, s));
        SMAT_HIP(hipMemcpyAsync(V.tile_pk.p, pk.data(), sizeof(int32_t) * pk.size(),
                                hipMemcpyHostToDevice, s));
        SMAT_TRY(launch_long_tile_pack(n7, NP, W, V.long_rows.as<int32_t>(), P.rp.as<int32_t>(),
                                       P.col.as<int32_t>(), P.val.p, P.elt,
                                       V.tile_seg.as<int32_t>(), kbd.as<int32_t>(),
                                       V.tile_pk.as<int32_t>(), V.tile_off.as<uint16_t>(),
                                       V.tile_val.p, s));
        SMAT_HIP(hipStreamSynchronize(s));
    }
    V.tile_seg.release();   // the CSR-position segment starts are not needed to run
    V.tile_P = NP;
    V.tile_nb = (int64_t)blocks.size() / 3;
    V.long_tiles = true;
    V.long_tpr = max_tpr;
    return SPMV_OK;
}

spmv_status build_variant(spmv_plan_s &P, const spmv_features &F, FeatureWork &W, int kernel,
                          const spmv_params &prm_in, hipStream_t s, Variant &V) {
    const spmv_params prm = resolve_params(kernel, prm_in, F, P.elt);
    V.kernel = kernel;
    V.prm = prm;
    const int64_t m = P.m, n = P.n, nnz = P.nnz;
    const int elt = P.elt;
    switch (kernel) {
    case SPMV_K_CSR_SCALAR:
    case SPMV_K_CSR_VECTOR:
        return SPMV_OK;
    case SPMV_K_BCSR: {
        const int64_t mb = (m + 3) / 4;
        Dev counts, scan;
        SMAT_TRY(counts.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, mb)));
        SMAT_TRY(scan.alloc(sizeof(unsigned) * (size_t)(mb / 4096 + 2)));
        SMAT_TRY(V.brp.alloc(sizeof(int32_t) * (size_t)(mb + 1)));
        SMAT_TRY(launch_bcsr_count(m, P.rp.as<int32_t>(), P.col.as<int32_t>(),
                                   counts.as<int32_t>(), V.brp.as<int32_t>(), scan.as<unsigned>(),
                                   s));
        int32_t nb = 0;
        SMAT_HIP(hipMemcpyAsync(&nb, V.brp.as<int32_t>() + mb, sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
        SMAT_HIP(hipStreamSynchronize(s));
        V.nblocks = nb;
        SMAT_TRY(V.bcol.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, nb)));
        SMAT_TRY(V.bval.alloc((size_t)elt * 16 * (size_t)std::max<int64_t>(1, nb)));
        SMAT_TRY(V.bpres.alloc(sizeof(uint32_t) * (size_t)((nb + 1) / 2 + 1)));
        SMAT_HIP(hipMemsetAsync(V.bval.p, 0, V.bval.bytes, s));
        SMAT_HIP(hipMemsetAsync(V.bpres.p, 0, V.bpres.bytes, s));
        SMAT_TRY(launch_csr_to_bcsr(m, P.rp.as<int32_t>(), P.col.as<int32_t>(), P.val.p, elt,
                                    V.brp.as<int32_t>(), V.bcol.as<int32_t>(), V.bval.p,
                                    V.bpres.as<uint16_t>(), s));
        if (P.dtype == SPMV_F64) {
            // keep every lane's chain within the float64 bound
            int L = std::max(8, V.prm.bcsr_lanes);
            while (L < 64 && bcsr_f64_depth(F.max_rd, L) > kFp64MaxDepth) L *= 2;
            V.prm.bcsr_lanes = L;
        }
        SMAT_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    case SPMV_K_COO: {
        SMAT_TRY(V.row_idx.alloc(sizeof(int32_t) * (size_t)nnz));
        SMAT_TRY(launch_csr_to_coo(m, nnz, P.rp.as<int32_t>(), V.row_idx.as<int32_t>(), s));
        int64_t per = (int64_t)prm.coo_chunk * kWave;
        int64_t nch = std::max<int64_t>(1, (nnz + per - 1) / per);
        SMAT_TRY(V.coo_head.alloc(sizeof(double) * nch));
        SMAT_TRY(V.coo_tail.alloc(sizeof(double) * nch));
        SMAT_TRY(V.coo_flags.alloc(sizeof(uint32_t) * nch));
        return SPMV_OK;
    }
    case SPMV_K_ELL: {
        V.K = (int)F.max_rd;
        size_t slots = (size_t)V.K * (size_t)P.m_pad;
        SMAT_TRY(V.ecol.alloc(sizeof(int32_t) * slots));
        SMAT_TRY(V.eval.alloc((size_t)elt * slots));
        SMAT_TRY(launch_csr_to_ell(m, P.m_pad, V.K, P.rp.as<int32_t>(), P.col.as<int32_t>(),
                                   P.val.p, elt, V.ecol.as<int32_t>(), V.eval.p, s));
        return SPMV_OK;
    }
    case SPMV_K_DIA:
    case SPMV_K_DIA_DIRECT: {
        if (!W.diag_hist.p) {
            set_error("DIA conversion needs the diagonal census");
            return SPMV_EUNSUPPORTED;
        }
        V.D = (int)F.ndiags;
        SMAT_TRY(V.dia_off.alloc(sizeof(int32_t) * std::max(1, V.D)));
        if (P.dia_offsets.empty() && V.D > 0) {
            // compact the census into ascending offsets; bins become slot ids
            int64_t nbins = m + n - 1;
            int64_t nblk = (nbins + 4095) / 4096;
            Dev blk;
            SMAT_TRY(blk.alloc(sizeof(unsigned) * (size_t)nblk));
            SMAT_TRY(launch_diag_compact(m, n, W.diag_hist.as<unsigned>(), V.dia_off.as<int32_t>(),
                                         blk.as<unsigned>(), s));
            P.dia_offsets.resize(V.D);
            SMAT_HIP(hipMemcpyAsync(P.dia_offsets.data(), V.dia_off.p, sizeof(int32_t) * V.D,
                                    hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipStreamSynchronize(s));
        } else if (V.D > 0) {
            SMAT_HIP(hipMemcpyAsync(V.dia_off.p, P.dia_offsets.data(), sizeof(int32_t) * V.D,
                                    hipMemcpyHostToDevice, s));
        }
        size_t slots = (size_t)V.D * (size_t)P.m_pad;
        size_t words = (slots + 31) / 32;
        SMAT_TRY(V.dia_data.alloc((size_t)elt * slots));
        SMAT_TRY(V.dia_present.alloc(sizeof(uint32_t) * words));
        SMAT_HIP(hipMemsetAsync(V.dia_data.p, 0, V.dia_data.bytes, s));
        SMAT_HIP(hipMemsetAsync(V.dia_present.p, 0, V.dia_present.bytes, s));
        SMAT_TRY(launch_csr_to_dia(m, n, P.m_pad, nnz, P.rp.as<int32_t>(), P.col.as<int32_t>(),
                                   P.val.p, elt, W.diag_hist.as<unsigned>(), V.dia_data.p,
                                   V.dia_present.as<uint32_t>(), s));
        // windows of diagonals whose offsets span at most dia_span
        std::vector<DiaWindow> win;
        int max_span = 0;
        for (int d = 0; d < V.D;) {
            int e = d;
            while (e + 1 < V.D &&
                   (int64_t)P.dia_offsets[e + 1] - P.dia_offsets[d] <= prm.dia_span)
                ++e;
            win.push_back({d, e});
            max_span = std::max(max_span, P.dia_offsets[e] - P.dia_offsets[d]);
            d = e + 1;
        }
        V.nwin = (int)win.size();
        V.max_span = max_span;
        if (kernel == SPMV_K_DIA) {
            const int64_t rows = (int64_t)std::min(prm.block, 256) * prm.dia_rows_per_thread *
                                 (prm.wide_loads == 1 ? 16 / elt : 1);
            const int64_t lds = (rows + max_span) * elt;
            if (lds > kDiaLdsMax) {
                set_error("DIA tile of %lld rows with an x window span of %d needs %lld bytes "
                          "of LDS (limit %lld)", (long long)rows, max_span, (long long)lds,
                          (long long)kDiaLdsMax);
                return SPMV_EUNSUPPORTED;
            }
        }
        SMAT_TRY(V.dia_win.alloc(sizeof(DiaWindow) * std::max<size_t>(1, win.size())));
        if (!win.empty())
            SMAT_HIP(hipMemcpyAsync(V.dia_win.p, win.data(), sizeof(DiaWindow) * win.size(),
                                    hipMemcpyHostToDevice, s));
        SMAT_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    case SPMV_K_CSR_ADAPTIVE:
    case SPMV_K_CSR_PANEL: {
        const bool panels = kernel == SPMV_K_CSR_PANEL;
        int shift = 0;
        if (panels) {
            panel_geometry(F, elt, prm, &V.panel_w, &V.P);
            while ((2 << shift) <= V.P && shift < 6) ++shift;  // floor(log2 P)
        }
        V.alaunch.lane_shift = shift;
        BinSpec spec;
        const int rpl = prm.adaptive_rows_per_lane;
        for (int b = 0; b < 6; ++b) {  // widths 1..32
            spec.upper[b] = rpl << b;
            V.bin_lanes[b] = 1 << b;
        }
        V.bin_lanes[6] = 64;
        spec.upper[7] = (int)kSplitMin;   // one workgroup per row
        spec.upper[8] = INT_MAX;          // split rows
        V.bin_lanes[7] = 0;
        V.bin_lanes[8] = -1;
        unsigned nblk = (unsigned)std::max<int64_t>(1, (m + 255) / 256);
        SMAT_TRY(V.bin_rows.alloc(sizeof(int32_t) * std::max<int64_t>(1, m)));
        SMAT_TRY(V.bin_scratch.alloc(sizeof(unsigned) * ((size_t)nblk * kAdaptiveBins + kAdaptiveBins + 1)));
        // bins with rows longer than wg in bin 7, then one launch over bins
        // 7..0 (longest rows first)
        auto bin = [&](int wg) -> spmv_status {
            spec.upper[6] = std::max(wg, spec.upper[5]);  // width 64
            unsigned *blk = V.bin_scratch.as<unsigned>();
            unsigned *offs = blk + (size_t)nblk * kAdaptiveBins;
            SMAT_TRY(launch_bin_rows(m, P.rp.as<int32_t>(), spec, blk, V.bin_rows.as<int32_t>(),
                                     offs, s));
            SMAT_HIP(hipMemcpyAsync(V.bin_off, offs, sizeof(V.bin_off), hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipStreamSynchronize(s));
            unsigned blocks = 0;
            for (int q = 0; q < 8; ++q) {
                int b = 7 - q;
                V.alaunch.first[q] = blocks;
                unsigned cnt = V.bin_off[b + 1] - V.bin_off[b];
                unsigned per = b == 7 ? 1u : (unsigned)(256 >> std::max(0, b - shift));
                blocks += (cnt + per - 1) / per;
            }
            V.alaunch.first[8] = blocks;
            for (int b = 0; b < 9; ++b) V.alaunch.row_begin[b] = V.bin_off[b];
            return SPMV_OK;
        };
        // tiles (asked for, or the default's candidate) take the rows longer
        // than params.tile_row_min as well; the binned launch's own threshold is
        // restored below when they are not used
        const bool try_tiles = prm.long_lds == 0 || prm.long_lds == 3;
        int wg = try_tiles ? std::min(prm.adaptive_wg_min, prm.tile_row_min) : prm.adaptive_wg_min;
        SMAT_TRY(bin(wg));
        // split rows: segment table on the host from their row_ptr entries
        int64_t ns = V.bin_off[9] - V.bin_off[8];
        if (ns > 0) {
            Dev tmp;
            SMAT_TRY(tmp.alloc(sizeof(int64_t) * 2 * ns));
            k_gather_rowptr<<<(unsigned)((ns + 255) / 256), 256, 0, s>>>(
                ns, V.bin_rows.as<int32_t>() + V.bin_off[8], P.rp.as<int32_t>(), tmp.as<int64_t>());
            SMAT_LAUNCHED("gather_rowptr");
            std::vector<int64_t> be(2 * ns);
            std::vector<int32_t> rows(ns);
            SMAT_HIP(hipMemcpyAsync(be.data(), tmp.p, sizeof(int64_t) * 2 * ns,
                                    hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipMemcpyAsync(rows.data(), V.bin_rows.as<int32_t>() + V.bin_off[8],
                                    sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipStreamSynchronize(s));
            std::vector<int64_t> segs, begin(1, 0);
            for (int64_t r = 0; r < ns; ++r) {
                for (int64_t b = be[2 * r]; b < be[2 * r + 1]; b += kSplitSegment) {
                    segs.push_back(r);
                    segs.push_back(b);
                    segs.push_back(std::min(b + kSplitSegment, be[2 * r + 1]));
                }
                begin.push_back((int64_t)segs.size() / 3);
            }
            V.nsplit_rows = ns;
            V.nsplit_segs = (int64_t)segs.size() / 3;
            SMAT_TRY(V.split_segs.alloc(sizeof(int64_t) * segs.size()));
            SMAT_TRY(V.split_partials.alloc(sizeof(double) * V.nsplit_segs));
            SMAT_TRY(V.split_begin.alloc(sizeof(int64_t) * begin.size()));
            SMAT_TRY(V.split_rows.alloc(sizeof(int32_t) * ns));
            SMAT_HIP(hipMemcpyAsync(V.split_segs.p, segs.data(), sizeof(int64_t) * segs.size(),
                                    hipMemcpyHostToDevice, s));
            SMAT_HIP(hipMemcpyAsync(V.split_begin.p, begin.data(), sizeof(int64_t) * begin.size(),
                                    hipMemcpyHostToDevice, s));
            SMAT_HIP(hipMemcpyAsync(V.split_rows.p, rows.data(), sizeof(int32_t) * ns,
                                    hipMemcpyHostToDevice, s));
            SMAT_HIP(hipStreamSynchronize(s));
        }
        // The longest bin (a workgroup per row) can leave the binned launch
        // for a kernel that keeps x in LDS: x chunks streamed through each
        // workgroup of rows (long_lds 1, float64) or one x panel per (row
        // block, panel) workgroup (long_lds 3).  Default: tiles from
        // kTileRowsDefault rows longer than tile_row_min.  Tiles that do not
        // suit the matrix fall back to chunks where those keep the float64
        // chain bound, else to the binned launch.
        int ll = prm.long_lds;
        for (;;) {
            const int64_t n7 = (int64_t)V.bin_off[8] - V.bin_off[7];
            if (ll == 0) ll = n7 >= kTileRowsDefault ? 3 : 2;
            int tpr = n7 >= 8192 ? 32 : 64;
            if ((F.max_rd + tpr - 1) / tpr + ilog2(tpr) > kFp64MaxDepth) tpr = 64;
            const bool chunks_ok = P.dtype == SPMV_F64 &&
                                   (F.max_rd + tpr - 1) / tpr + ilog2(tpr) <= kFp64MaxDepth;
            if (n7 == 0 || (ll == 1 && !chunks_ok)) ll = 2;
            if (ll != 2) {
                // the long rows longest first, so that the rows of one
                // workgroup (which waits for its longest) are alike
                std::vector<int64_t> len(n7);
                {
                    Dev be;
                    SMAT_TRY(be.alloc(sizeof(int64_t) * 2 * (size_t)n7));
                    const int32_t *r7 = V.bin_rows.as<int32_t>() + V.bin_off[7];
                    k_gather_rowptr<<<(unsigned)((n7 + 255) / 256), 256, 0, s>>>(
                        n7, r7, P.rp.as<int32_t>(), be.as<int64_t>());
                    SMAT_LAUNCHED("gather_rowptr");
                    std::vector<int64_t> h(2 * (size_t)n7);
                    std::vector<int32_t> rows(n7);
                    SMAT_HIP(hipMemcpyAsync(h.data(), be.p, sizeof(int64_t) * 2 * n7,
                                            hipMemcpyDeviceToHost, s));
                    SMAT_HIP(hipMemcpyAsync(rows.data(), r7, sizeof(int32_t) * n7,
                                            hipMemcpyDeviceToHost, s));
                    SMAT_HIP(hipStreamSynchronize(s));
                    std::vector<int64_t> ord(n7);
                    for (int64_t i = 0; i < n7; ++i) ord[i] = i;
                    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
                        return h[2 * a + 1] - h[2 * a] > h[2 * b + 1] - h[2 * b];
                    });
                    std::vector<int32_t> sorted(n7);
                    for (int64_t i = 0; i < n7; ++i) {
                        sorted[i] = rows[ord[i]];
                        len[i] = h[2 * ord[i] + 1] - h[2 * ord[i]];
                    }
                    SMAT_TRY(V.long_rows.alloc(sizeof(int32_t) * (size_t)n7));
                    SMAT_HIP(hipMemcpyAsync(V.long_rows.p, sorted.data(), sizeof(int32_t) * n7,
                                            hipMemcpyHostToDevice, s));
                    SMAT_HIP(hipStreamSynchronize(s));
                }
                if (ll == 3) {
                    SMAT_TRY(build_long_tiles(P, V, len, s));
                    if (!V.long_tiles) ll = chunks_ok ? 1 : 2;
                }
            }
            if (ll != 3 && wg != prm.adaptive_wg_min && n7 > 0) {
                // no tiles: bins with the binned launch's own threshold
                V.long_rows.release();
                wg = prm.adaptive_wg_min;
                SMAT_TRY(bin(wg));
                continue;
            }
            if (ll == 1) {
                SMAT_TRY(long_rows_lds_prepare());
                V.long_tpr = tpr;
            }
            if (ll == 2) {
                V.long_rows.release();
            } else {
                V.n_long = n7;
                const unsigned b7 = V.alaunch.first[1];  // workgroups of bin 7
                V.arest = V.alaunch;
                V.arest.first[0] = 0;
                for (int q = 1; q < 9; ++q) V.arest.first[q] = V.alaunch.first[q] - b7;
            }
            break;
        }
        V.prm.long_lds = ll;
        V.bin_scratch.release();
        if (!panels) {
            // the launch's rows (bins 0-6 when the long rows left it, else
            // 0-7) with their entries copied in binned order: the rows of a
            // bin then read one contiguous range (measured 3-17% faster on
            // Zipf matrices, the same on uniform ones)
            const int64_t hi = V.bin_off[V.long_tpr ? 7 : 8];
            Dev len, scan;
            SMAT_TRY(len.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, hi)));
            SMAT_TRY(scan.alloc(sizeof(unsigned) * (size_t)(hi / 4096 + 2)));
            SMAT_TRY(V.binned_rp.alloc(sizeof(int32_t) * (size_t)(hi + 1)));
            SMAT_TRY(launch_binned_scan(hi, V.bin_rows.as<int32_t>(), P.rp.as<int32_t>(),
                                        len.as<int32_t>(), scan.as<unsigned>(),
                                        V.binned_rp.as<int32_t>(), s));
            int32_t tot = 0;
            SMAT_HIP(hipMemcpyAsync(&tot, V.binned_rp.as<int32_t>() + hi, sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipStreamSynchronize(s));
            SMAT_TRY(V.binned_col.alloc(sizeof(int32_t) * (size_t)std::max<int32_t>(1, tot)));
            SMAT_TRY(V.binned_val.alloc((size_t)elt * (size_t)std::max<int32_t>(1, tot)));
            SMAT_TRY(launch_pack_binned(hi, V.bin_rows.as<int32_t>(), P.rp.as<int32_t>(),
                                        P.col.as<int32_t>(), P.val.p, elt, V.binned_rp.as<int32_t>(),
                                        V.binned_col.as<int32_t>(), V.binned_val.p, s));
            SMAT_HIP(hipStreamSynchronize(s));
        }
        if (panels && prm.panel_direct_max > 0) {
            // the shortest bins leave the panels: their rows cost a panel
            // row pointer and a partial written and read per panel, more
            // than their few gathers from x save
            int S = 0;
            while (S < 6 && spec.upper[S] <= prm.panel_direct_max) ++S;
            V.short_bins = S;
            if (S > 0) {
                V.ashort = bins_launch(V.bin_off, 0, S - 1, 0);
                V.apanel = bins_launch(V.bin_off, S, V.long_tpr ? 6 : 7, shift);
            }
        }
        if (panels) {
            if (ns > 0) {
                set_error("column panels cannot hold rows longer than %lld entries",
                          (long long)kSplitMin);
                return SPMV_EUNSUPPORTED;
            }
            const int64_t L = (int64_t)V.P * (m + 1);
            if (L >= (1ll << 31)) {
                set_error("%d column panels x %lld rows exceed the int32 panel row pointers",
                          V.P, (long long)m);
                return SPMV_EUNSUPPORTED;
            }
            Dev inv, cnt, scan;
            SMAT_TRY(inv.alloc(sizeof(int32_t) * std::max<int64_t>(1, m)));
            SMAT_TRY(cnt.alloc(sizeof(int32_t) * (size_t)L));
            SMAT_TRY(scan.alloc(sizeof(unsigned) * (size_t)(L / 4096 + 2)));
            SMAT_TRY(V.prow.alloc(sizeof(int32_t) * (size_t)(L + 1)));
            SMAT_TRY(V.pcol.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, nnz)));
            SMAT_TRY(V.pval.alloc((size_t)elt * (size_t)std::max<int64_t>(1, nnz)));
            SMAT_TRY(launch_csr_to_panels(m, nnz, P.rp.as<int32_t>(), P.col.as<int32_t>(), P.val.p,
                                          elt, V.bin_rows.as<int32_t>(), V.P, V.panel_w,
                                          inv.as<int32_t>(), cnt.as<int32_t>(),
                                          V.prow.as<int32_t>(), scan.as<unsigned>(),
                                          V.pcol.as<int32_t>(), V.pval.p, s));
            if (prm.panel_xcd != 2)
                SMAT_TRY(V.ppart.alloc((size_t)elt * (size_t)V.P * (size_t)std::max<int64_t>(1, m)));
            SMAT_HIP(hipStreamSynchronize(s));
        }
        return SPMV_OK;
    }
    default:
        set_error("unknown kernel %d", kernel);
        return SPMV_EINVAL;
    }
}

// The long rows taken out of the binned launch: x chunks or tiles.
spmv_status run_long_rows(const spmv_plan_s &P, const Variant &V, const void *x, void *y,
                          hipStream_t s) {
    if (V.long_tiles)
        return run_long_tiles(P.elt, V.n_long, V.tile_P, V.tile_nb, V.tile_blocks.as<int32_t>(),
                              V.tile_pk.as<int32_t>(), V.long_rows.as<int32_t>(),
                              V.tile_off.as<uint16_t>(), V.tile_val.p, x, P.n,
                              V.tile_part.as<double>(), y, s);
    return run_long_rows_lds(V.long_tpr, V.n_long, V.long_rows.as<int32_t>(), P.rp.as<int32_t>(),
                             P.col.as<int32_t>(), P.val.as<double>(), (const double *)x, P.n,
                             (double *)y, s);
}

spmv_status run_variant(const spmv_plan_s &P, const Variant &V, const void *x, void *y,
                        hipStream_t s) {
    const int elt = P.elt;
    const int64_t m = P.m;
    const bool nt = V.prm.stream_nt == 1;
    if (m == 0) return SPMV_OK;
    switch (V.kernel) {
    case SPMV_K_CSR_SCALAR:
        return run_csr_scalar(elt, m, P.rp.as<int32_t>(), P.col.as<int32_t>(), P.val.p, x, y,
                              V.prm.block, s);
    case SPMV_K_CSR_VECTOR:
        return run_csr_vector(elt, nt, V.prm.vector_lanes, m, P.rp.as<int32_t>(),
                              P.col.as<int32_t>(), P.val.p, x, y, V.prm.block, s);
    case SPMV_K_CSR_ADAPTIVE: {
        if (V.long_tiles) {
            // the tiles first, then the short rows and the tiles' sums in
            // one launch
            SMAT_TRY(run_long_tiles(elt, V.n_long, V.tile_P, V.tile_nb,
                                    V.tile_blocks.as<int32_t>(), V.tile_pk.as<int32_t>(),
                                    V.long_rows.as<int32_t>(), V.tile_off.as<uint16_t>(),
                                    V.tile_val.p, x, P.n, V.tile_part.as<double>(), y, s, false));
            SMAT_TRY(run_csr_adaptive_tiles(elt, nt, V.arest, V.bin_rows.as<int32_t>(),
                                            V.binned_rp.as<int32_t>(), V.binned_col.as<int32_t>(),
                                            V.binned_val.p, x, y, V.n_long, V.tile_P,
                                            V.long_rows.as<int32_t>(), V.tile_part.as<double>(),
                                            s));
        } else {
            SMAT_TRY(run_csr_adaptive(elt, nt, V.long_tpr != 0, V.long_tpr ? V.arest : V.alaunch,
                                      V.bin_rows.as<int32_t>(), V.binned_rp.as<int32_t>(),
                                      V.binned_col.as<int32_t>(), V.binned_val.p, x, y, s, true));
            if (V.long_tpr) SMAT_TRY(run_long_rows(P, V, x, y, s));
        }
        if (V.nsplit_rows)
            SMAT_TRY(run_csr_split(elt, V.nsplit_segs, V.split_segs.as<int64_t>(),
                                   V.split_partials.as<double>(), V.nsplit_rows,
                                   V.split_begin.as<int64_t>(), V.split_rows.as<int32_t>(),
                                   P.col.as<int32_t>(), P.val.p, x, y, s));
        return SPMV_OK;
    }
    case SPMV_K_CSR_PANEL: {
        // binned positions [lo, hi) go through the panels: all rows but the
        // short bins (summed directly) and the longest bin (long-row kernel)
        const int64_t lo = V.bin_off[V.short_bins];
        const int64_t hi = V.long_tpr ? V.bin_off[7] : m;
        const AdaptiveLaunch &ap =
            V.short_bins ? V.apanel : V.long_tpr ? V.arest : V.alaunch;
        SMAT_TRY(run_csr_panels(elt, nt, ap, V.bin_rows.as<int32_t>(), V.P, m,
                                V.prow.as<int32_t>(), V.pcol.as<int32_t>(), V.pval.p, x, y,
                                V.prm.panel_xcd != 2 ? V.ppart.p : nullptr, lo, hi,
                                V.short_bins > 0 || V.long_tpr != 0, s));
        if (V.short_bins)
            SMAT_TRY(run_csr_adaptive(elt, nt, true, V.ashort, V.bin_rows.as<int32_t>(),
                                      P.rp.as<int32_t>(), P.col.as<int32_t>(), P.val.p, x, y, s));
        if (V.long_tpr) SMAT_TRY(run_long_rows(P, V, x, y, s));
        return SPMV_OK;
    }
    case SPMV_K_BCSR:
        return run_bcsr(elt, nt, m, P.n, V.brp.as<int32_t>(), V.bcol.as<int32_t>(), V.bval.p, x,
                        y, V.prm.bcsr_lanes, std::min(V.prm.block, 256), s);
    case SPMV_K_ELL:
        return run_ell(elt, nt, m, P.m_pad, V.K, V.ecol.as<int32_t>(), V.eval.p, x, y,
                       V.prm.block, V.prm.ell_unroll, V.prm.wide_loads == 1, s);
    case SPMV_K_DIA:
    case SPMV_K_DIA_DIRECT:
        return run_dia(elt, nt, V.kernel == SPMV_K_DIA, m, P.n, P.m_pad, V.D,
                       V.dia_off.as<int32_t>(), V.nwin, V.dia_win.as<DiaWindow>(), V.max_span,
                       V.dia_data.p, x, y, std::min(V.prm.block, 256), V.prm.dia_rows_per_thread,
                       V.prm.wide_loads == 1, s);
    case SPMV_K_COO:
        return run_coo(elt, nt, m, P.nnz, V.row_idx.as<int32_t>(), P.col.as<int32_t>(), P.val.p,
                       x, y, V.prm.coo_chunk, V.coo_head.as<double>(), V.coo_tail.as<double>(),
                       V.coo_flags.as<uint32_t>(), s);
    default:
        set_error("plan holds no kernel");
        return SPMV_EINVAL;
    }
}

// Median time in ms of `reps` runs (after one warm-up run).
// Per-rep time of a candidate: back-to-back launches between one event pair,
// as many as make about kTimeBatchMs of work (at most kTimeBatchMax), so that
// launch overhead and timer resolution do not decide between kernels of a
// few microseconds, and the figure is the steady rate of repeated calls.
// The median over `reps` such batches is reported, per launch.  With
// abandon_ms > 0 a candidate whose first batch already takes longer than
// that per launch is not timed further: that batch's figure is reported.
constexpr double kTimeBatchMs = 0.05;
constexpr int kTimeBatchMax = 64;

template <typename Run>
spmv_status time_calls(Run run, int reps, hipStream_t s, double *ms, double abandon_ms = 0.0) {
    hipEvent_t a, b;
    SMAT_HIP(hipEventCreate(&a));
    SMAT_HIP(hipEventCreate(&b));
    auto batch = [&](int inner, float *f) -> spmv_status {
        (void)hipEventRecord(a, s);
        for (int i = 0; i < inner; ++i) SMAT_TRY(run());
        (void)hipEventRecord(b, s);
        if (hipEventSynchronize(b) != hipSuccess) return hip_fail(hipGetLastError(), "timing");
        (void)hipEventElapsedTime(f, a, b);
        return SPMV_OK;
    };
    spmv_status st = run();
    float probe = 0;
    if (st == SPMV_OK) st = batch(1, &probe);
    int inner = 1;
    if (probe > 0)
        inner = (int)std::min<double>(kTimeBatchMax, std::ceil(kTimeBatchMs / probe));
    inner = std::max(inner, 1);
    std::vector<double> t;
    for (int r = 0; r < reps && st == SPMV_OK; ++r) {
        float f = 0;
        st = batch(inner, &f);
        t.push_back((double)f / inner);
        if (r == 0 && abandon_ms > 0.0 && t[0] > abandon_ms) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != SPMV_OK) return st;
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.0 : t[t.size() / 2];
    return SPMV_OK;
}

spmv_status time_variant(const spmv_plan_s &P, const Variant &V, const void *x, void *y,
                         int reps, hipStream_t s, double *ms, double abandon_ms = 0.0) {
    return time_calls([&] { return run_variant(P, V, x, y, s); }, reps, s, ms, abandon_ms);
}

// Parameter points tried by the autotuner for one kernel (the paper's offline
// "kernel search", Section 3, done per matrix): at most a dozen, around the
// defaults.
std::vector<spmv_params> tune_grid(int kernel, const spmv_params &b, const spmv_features &F,
                                   int dtype) {
    std::vector<spmv_params> g;
    auto add = [&](spmv_params p) {
        if (check_params(p) == SPMV_OK) g.push_back(p);
    };
    const int nts[2] = {1, 2};
    switch (kernel) {
    case SPMV_K_CSR_SCALAR:
        for (int bs : {64, 128, 256, 512}) {
            spmv_params p = b;
            p.block = bs;
            add(p);
        }
        break;
    case SPMV_K_CSR_VECTOR:
        for (int f : {-2, -1, 0, 1, 2})
            for (int nt : nts) {
                spmv_params p = b;
                int L = f >= 0 ? b.vector_lanes << f : b.vector_lanes >> -f;
                if (L < 1 || L > 64) continue;
                if (dtype == SPMV_F64 && (F.max_rd + L - 1) / L + ilog2(L) > kFp64MaxDepth)
                    continue;
                p.vector_lanes = L;
                p.stream_nt = nt;
                add(p);
            }
        break;
    case SPMV_K_CSR_ADAPTIVE:
        for (int rpl : {1, 2, 4})
            for (int nt : nts)
                for (int ll : {1, 2, 3}) {  // long rows: x chunks (float64), binned, tiles
                    if (ll == 1 && dtype != SPMV_F64) continue;
                    spmv_params p = b;
                    p.adaptive_rows_per_lane = rpl;
                    p.stream_nt = nt;
                    p.long_lds = ll;
                    add(p);
                }
        // tiles for more or only the longer rows, the other parameters at
        // their defaults
        for (int r : {256, 4096, 16384}) {
            spmv_params p = b;
            p.long_lds = 3;
            p.tile_row_min = r;
            p.adaptive_wg_min = std::max(b.adaptive_wg_min, r);
            add(p);
        }
        break;
    case SPMV_K_ELL:
        for (int u : {2, 4})
            for (int bs : {256, 512})
                for (int nt : nts)
                    for (int wide : {1, 2}) {
                        spmv_params p = b;
                        p.ell_unroll = u;
                        p.block = bs;
                        p.stream_nt = nt;
                        p.wide_loads = wide;
                        add(p);
                    }
        break;
    case SPMV_K_DIA_DIRECT:
        for (int r : {1, 2, 4, 8})
            for (int nt : nts)
                for (int wide : {1, 2}) {
                    spmv_params p = b;
                    p.dia_rows_per_thread = r;
                    p.stream_nt = nt;
                    p.wide_loads = wide;
                    add(p);
                }
        break;
    case SPMV_K_DIA:
        for (int r : {1, 2, 4})
            for (int sp : {32, 256})
                for (int nt : nts)
                    for (int wide : {1, 2}) {
                        spmv_params p = b;
                        p.dia_rows_per_thread = r;
                        p.dia_span = sp;
                        p.stream_nt = nt;
                        p.wide_loads = wide;
                        add(p);
                    }
        break;
    case SPMV_K_BCSR:
        for (int f : {1, 2, 4, 8})  // float64: 8, 16, 32, 64 lanes; float32:
            for (int nt : nts) {     // half, equal and twice the default
                if (dtype != SPMV_F64 && f == 8) continue;
                spmv_params p = b;
                p.bcsr_lanes = dtype == SPMV_F64 ? 8 * f : std::max(1, std::min(64, b.bcsr_lanes * f / 2));
                p.stream_nt = nt;
                add(p);
            }
        break;
    case SPMV_K_CSR_PANEL: {
        std::vector<std::pair<int, int>> seen;  // (mode, P): kib values giving equal panels
        for (int mode : {1, 2})  // 1: eight panels at a time, one launch; 2: sequential
            for (int kib : {1024, 2048, 4096}) {
                spmv_params p = b;
                p.panel_xcd = mode;
                p.panel_kib = kib;
                int64_t w;
                int P;
                panel_geometry(F, dtype == SPMV_F64 ? 8 : 4, p, &w, &P);
                if (P < 2 || (mode == 2 && dtype == SPMV_F32 && P > 16)) continue;
                if ((int64_t)P * (F.m + 1) >= (1ll << 31)) continue;  // int32 panel row pointers
                if (std::find(seen.begin(), seen.end(), std::make_pair(mode, P)) != seen.end())
                    continue;
                seen.push_back({mode, P});
                for (int nt : nts)
                    for (int ll : {1, 2, 3}) {  // long rows: x chunks (float64), binned, tiles
                        if (ll == 1 && dtype != SPMV_F64) continue;
                        p.stream_nt = nt;
                        p.long_lds = ll;
                        add(p);
                    }
            }
        // short rows without panels, and tiles for more or only the longer
        // rows, the other parameters at their defaults
        for (int d : {-1, 4, 16, 64}) {
            spmv_params p = b;
            p.panel_direct_max = d;
            add(p);
        }
        for (int r : {256, 4096, 16384}) {
            spmv_params p = b;
            p.long_lds = 3;
            p.tile_row_min = r;
            p.adaptive_wg_min = std::max(b.adaptive_wg_min, r);
            add(p);
        }
        break;
    }
    case SPMV_K_COO:
        for (int c : {2, 4, 8, 16})
            for (int nt : nts) {
                spmv_params p = b;
                p.coo_chunk = c;
                p.stream_nt = nt;
                if (dtype == SPMV_F64 && F.max_rd > kCooMaxChunksPerRow * (int64_t)c * kWave)
                    continue;
                add(p);
            }
        break;
    default:
        break;
    }
    return g;
}

bool same_params(const spmv_params &a, const spmv_params &b) {
    return std::memcmp(&a, &b, sizeof(a)) == 0;
}

// A timed alternative replaces the incumbent (the default parameters, or the
// predicted-best kernel) only when it is faster by more than this fraction:
// differences inside run-to-run timing noise would otherwise flip plans of
// the same matrix between equivalent choices from one process to the next.
constexpr double kSwitchMargin = 0.03;
// A point whose first timed batch is this much slower than the best so far
// is not timed further (it cannot come within kSwitchMargin of winning).
constexpr double kAbandonRatio = 1.25;

// Time the grid for the chosen kernel and keep the fastest variant.  Every
// visited point must also reproduce the starting variant's output on the
// all-ones probe vector within twice the accuracy contract (each result is
// within the contract of the exact one): a point that does not is never
// kept, and *rejected counts it.
spmv_status autotune_variant(spmv_plan_s &P, const spmv_features &F, FeatureWork &W, int reps,
                             hipStream_t s, std::unique_ptr<Variant> &best, int32_t *rejected) {
    const int64_t m = P.m;
    const unsigned g = (unsigned)((std::max<int64_t>(1, m) + 255) / 256);
    Dev xs, ys, yref, absrow, bad;
    SMAT_TRY(xs.alloc((size_t)P.elt * std::max<int64_t>(1, P.n)));
    SMAT_TRY(ys.alloc((size_t)P.elt * std::max<int64_t>(1, m)));
    SMAT_TRY(yref.alloc((size_t)P.elt * std::max<int64_t>(1, m)));
    SMAT_TRY(absrow.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, m)));
    SMAT_TRY(bad.alloc(sizeof(unsigned)));
    if (P.n) k_fill_one<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.elt, xs.p);
    SMAT_LAUNCHED("fill_one");
    double best_ms = 0;
    SMAT_TRY(time_variant(P, *best, xs.p, ys.p, reps, s, &best_ms));
    if (m) {
        SMAT_HIP(hipMemcpyAsync(yref.p, ys.p, (size_t)P.elt * m, hipMemcpyDeviceToDevice, s));
        if (P.elt == 8)
            k_row_abs_sum<double><<<g, 256, 0, s>>>(m, P.rp.as<int32_t>(), P.val.as<double>(),
                                                    absrow.as<double>());
        else
            k_row_abs_sum<float><<<g, 256, 0, s>>>(m, P.rp.as<int32_t>(), P.val.as<float>(),
                                                   absrow.as<double>());
        SMAT_LAUNCHED("row_abs_sum");
    }
    const double tol = 2.0 * (P.elt == 8 ? 1e-12 : 2e-6);
    const int kernel = best->kernel;
    // points whose parameters resolve to one already timed (a switch the
    // matrix leaves without effect) are not timed again
    std::vector<spmv_params> visited{best->prm};
    for (const spmv_params &p : tune_grid(kernel, best->prm, F, P.dtype)) {
        if (same_params(p, best->prm)) continue;
        auto V = std::make_unique<Variant>();
        spmv_status st = build_variant(P, F, W, kernel, p, s, *V);
        if (st == SPMV_ENOMEM || st == SPMV_EUNSUPPORTED) continue;
        if (st != SPMV_OK) return st;
        if (std::any_of(visited.begin(), visited.end(),
                        [&](const spmv_params &q) { return same_params(V->prm, q); }))
            continue;
        visited.push_back(V->prm);
        double ms = 0;
        SMAT_TRY(time_variant(P, *V, xs.p, ys.p, reps, s, &ms, best_ms * kAbandonRatio));
        if (m) {
            unsigned h = 0;
            SMAT_HIP(hipMemsetAsync(bad.p, 0, sizeof(unsigned), s));
            if (P.elt == 8)
                k_tune_check<double><<<g, 256, 0, s>>>(m, ys.as<double>(), yref.as<double>(),
                                                       absrow.as<double>(), tol, bad.as<unsigned>());
            else
                k_tune_check<float><<<g, 256, 0, s>>>(m, ys.as<float>(), yref.as<float>(),
                                                      absrow.as<double>(), tol, bad.as<unsigned>());
            SMAT_LAUNCHED("tune_check");
            SMAT_HIP(hipMemcpyAsync(&h, bad.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
            SMAT_HIP(hipStreamSynchronize(s));
            if (h) {
                ++*rejected;
                continue;
            }
        }
        if (ms < best_ms * (1.0 - kSwitchMargin)) {
            best_ms = ms;
            best = std::move(V);
        }
    }
    return SPMV_OK;
}

bool needs_csr(const Variant &V) {
    const int k = V.kernel;
    return k == SPMV_K_CSR_SCALAR || k == SPMV_K_CSR_VECTOR || k == SPMV_K_CSR_ADAPTIVE ||
           k == SPMV_K_COO ||
           // long rows and directly summed short rows read the CSR copy
           (k == SPMV_K_CSR_PANEL && (V.long_tpr || V.short_bins));
}

}  // namespace
}  // namespace smat

// ====================================================================== C-ABI

extern "C" const char *spmv_status_string(spmv_status s) {
    switch (s) {
    case SPMV_OK: return "SPMV_OK";
    case SPMV_EINVAL: return "SPMV_EINVAL";
    case SPMV_ENOMEM: return "SPMV_ENOMEM";
    case SPMV_EDEVICE: return "SPMV_EDEVICE";
    case SPMV_EUNSUPPORTED: return "SPMV_EUNSUPPORTED";
    }
    return "unknown status";
}

extern "C" const char *spmv_last_error(void) { return g_err; }

extern "C" const char *spmv_kernel_name(int32_t k) {
    static const char *names[] = {"csr_scalar", "csr_vector", "csr_adaptive", "ell",
                                  "dia",        "dia_direct", "coo",          "csr_panel",
                                  "bcsr"};
    return (k >= 0 && k < SPMV_K_COUNT) ? names[k] : "invalid";
}

extern "C" spmv_status spmv_plan_opts_default(spmv_plan_opts *o) {
    if (!o) return SPMV_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->selector = -1;  // resolved at plan time: MLP if a model is given
    o->force_kernel = -1;
    o->confidence_tau = 0.1f;
    o->measure_topk = 3;
    o->timing_reps = 5;
    o->staged = 1;
    o->stage_conf = 0.98f;
    return SPMV_OK;
}

extern "C" spmv_status spmv_plan_opts_apply_env(spmv_plan_opts *o) {
    if (!o) {
        set_error("opts is NULL");
        return SPMV_EINVAL;
    }
    const char *v = std::getenv("SPMV_SELECTOR");
    if (v && *v) {
        int k = -1;
        for (int i = 0; i < SPMV_K_COUNT; ++i)
            if (!std::strcmp(v, spmv_kernel_name(i))) k = i;
        if (!std::strcmp(v, "rules")) {
            o->selector = SPMV_SELECT_RULES;
        } else if (!std::strcmp(v, "mlp")) {
            if (o->model)
                o->selector = SPMV_SELECT_MLP;
            else
                std::fprintf(stderr, "[spmv] SPMV_SELECTOR=mlp ignored: no model given\n");
        } else if (!std::strcmp(v, "exhaustive")) {
            o->selector = SPMV_SELECT_EXHAUSTIVE;
        } else if (k >= 0) {
            o->selector = SPMV_SELECT_FORCED;
            o->force_kernel = k;
        } else {
            std::fprintf(stderr, "[spmv] SPMV_SELECTOR=%s ignored: not rules, mlp, exhaustive "
                                 "or a kernel name\n", v);
        }
    }
    v = std::getenv("SPMV_TAU");
    if (v && *v) {
        char *end = nullptr;
        const double t = std::strtod(v, &end);
        if (end && *end == 0 && std::isfinite(t) && t >= 0)
            o->confidence_tau = (float)t;
        else
            std::fprintf(stderr, "[spmv] SPMV_TAU=%s ignored: not a number >= 0\n", v);
    }
    v = std::getenv("SPMV_LOG");
    if (v && *v) {
        if (!std::strcmp(v, "1"))
            o->log = 1;
        else if (!std::strcmp(v, "0"))
            o->log = 0;
        else
            std::fprintf(stderr, "[spmv] SPMV_LOG=%s ignored: 0 or 1\n", v);
    }
    return SPMV_OK;
}

static spmv_status check_csr(const spmv_csr *A) {
    if (!A) {
        set_error("csr is NULL");
        return SPMV_EINVAL;
    }
    if (A->m < 0 || A->n < 0 || A->nnz < 0) {
        set_error("negative m, n or nnz");
        return SPMV_EINVAL;
    }
    if (A->dtype != SPMV_F32 && A->dtype != SPMV_F64) {
        set_error("dtype must be SPMV_F32 or SPMV_F64");
        return SPMV_EINVAL;
    }
    if (A->m >= INT_MAX || A->n >= INT_MAX || A->nnz >= INT_MAX) {
        set_error("m, n and nnz must stay below 2^31 (int32 index paths)");
        return SPMV_EUNSUPPORTED;
    }
    if (A->nnz > 0 && (A->m == 0 || A->n == 0)) {
        set_error("nnz > 0 with an empty dimension");
        return SPMV_EINVAL;
    }
    if (!A->row_ptr_dev || (A->nnz > 0 && (!A->col_dev || !A->val_dev))) {
        set_error("NULL device array");
        return SPMV_EINVAL;
    }
    return SPMV_OK;
}

extern "C" spmv_status spmv_features_compute(const spmv_csr *A, spmv_features *out, void *stream) {
    SMAT_TRY(check_csr(A));
    if (!out) {
        set_error("out is NULL");
        return SPMV_EINVAL;
    }
    FeatureWork W;
    return validate_and_extract(*A, (hipStream_t)stream, *out, W, false, nullptr, nullptr);
}

namespace smat {
size_t features_region_bytes(int64_t m, int64_t n) {
    return FeatureArena::total(std::max<int64_t>(0, m), std::max<int64_t>(0, n));
}

spmv_status features_in_region(const spmv_csr *A, spmv_features *out, hipStream_t s,
                               void *region, size_t bytes) {
    SMAT_TRY(check_csr(A));
    if (!out || !region) {
        set_error("out or region is NULL");
        return SPMV_EINVAL;
    }
    const size_t need = features_region_bytes(A->m, A->n);
    if (need > bytes) {
        set_error("matrix needs %zu bytes of feature scratch (m + n - 1 diagonal bins and "
                  "n + 1 row-degree bins); the fixed region holds %zu",
                  need, bytes);
        return SPMV_EUNSUPPORTED;
    }
    FeatureWork W;
    W.arena = static_cast<unsigned char *>(region);
    W.arena_bytes = need;
    W.arena_row_off = FeatureArena::row_offset(A->m, A->n);
    return validate_and_extract(*A, s, *out, W, false, nullptr, nullptr);
}
}  // namespace smat

namespace {
__global__ void k_rebase_rows(int64_t m, const int32_t *__restrict__ rp, int32_t base,
                              int32_t *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i <= m) out[i] = rp[i] - base;
}
__global__ void k_offset_rows(int64_t m, int32_t *__restrict__ rp, int32_t base) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i <= m) rp[i] += base;
}
}  // namespace

static spmv_status plan_create_impl(const spmv_csr *A, const spmv_plan_opts *opts_in,
                                    hipStream_t s, spmv_plan_t *out);

// Equation 2 of a finished plan (opts.time_baseline): the median time of one
// run of the plan and of the plain CSR kernel (one thread per row) on the
// caller's CSR, both on x = 1, and the calls after which the planning time
// is paid back, t_plan / (t_plain - t_run).
static spmv_status time_baseline(spmv_plan_s *P, const spmv_csr *A, int reps, hipStream_t s) {
    spmv_plan_info &I = P->info;
    Dev xs, ys;
    SMAT_TRY(xs.alloc((size_t)P->elt * std::max<int64_t>(1, P->n)));
    SMAT_TRY(ys.alloc((size_t)P->elt * std::max<int64_t>(1, P->m)));
    if (P->n) k_fill_one<<<(unsigned)((P->n + 255) / 256), 256, 0, s>>>(P->n, P->elt, xs.p);
    SMAT_LAUNCHED("fill_one");
    double t_run = 0, t_plain = 0;
    SMAT_TRY(time_calls([&] { return spmv_run(P, xs.p, ys.p, s); }, reps, s, &t_run));
    SMAT_TRY(time_calls(
        [&] {
            return run_csr_scalar(P->elt, A->m, A->row_ptr_dev, A->col_dev, A->val_dev, xs.p,
                                  ys.p, 256, s);
        },
        reps, s, &t_plain));
    I.t_run_ms = t_run;
    I.t_plain_ms = t_plain;
    I.break_even_calls = t_plain > t_run ? I.t_plan_ms / (t_plain - t_run)
                                         : std::numeric_limits<double>::infinity();
    return SPMV_OK;
}

// One line per plan on stderr (opts.log, SPMV_LOG=1).
static void log_plan(const spmv_plan_s &P) {
    const spmv_plan_info &I = P.info;
    static const char *sel[] = {"rules", "mlp", "exhaustive", "forced"};
    const int su = I.selector_used >= 0 && I.selector_used <= 3 ? I.selector_used : 0;
    char be[96] = "";
    if (I.t_run_ms >= 0)
        std::snprintf(be, sizeof(be), " run=%.4fms plain=%.4fms break_even=%.1f", I.t_run_ms,
                      I.t_plain_ms, I.break_even_calls);
    std::fprintf(stderr,
                 "[spmv] plan m=%lld n=%lld nnz=%lld %s kernel=%s selector=%s conf=%.3f "
                 "measured=%d stage=%d segments=%d long_rows=%lld plan=%.3fms tune=%.3fms "
                 "device=%.1fMB%s\n",
                 (long long)I.m, (long long)I.n, (long long)I.nnz,
                 I.dtype == SPMV_F64 ? "f64" : "f32",
                 I.n_segments ? "segmented" : spmv_kernel_name(I.kernel), sel[su],
                 (double)I.confidence, I.n_measured, I.feature_stage, I.n_segments,
                 (long long)I.long_rows, I.t_plan_ms, I.t_tune_ms,
                 (double)I.device_bytes / 1048576.0, be);
}

// Options in effect for plan creation: the caller's (or the defaults)
// with the environment overrides applied.
static spmv_plan_opts effective_opts(const spmv_plan_opts *opts) {
    spmv_plan_opts o;
    if (opts)
        o = *opts;
    else
        spmv_plan_opts_default(&o);
    spmv_plan_opts_apply_env(&o);
    return o;
}

// Segmented plan (Section 6: the matrix divided by rows into sub-matrices of
// equal nonzero counts, each tuned on its own): rows cut where the running
// nonzero count crosses k nnz / S, each segment planned through the public
// entry point with the caller's options.
static spmv_status plan_create_segments(const spmv_csr *A, const spmv_plan_opts &opts, int mode,
                                        hipStream_t s, spmv_plan_t *out,
                                        std::chrono::steady_clock::time_point t_start) {
    auto P = std::make_unique<spmv_plan_s>();
    P->alloc = opts.allocator;
    SMAT_HIP(hipGetDevice(&P->device));
    P->m = A->m;
    P->n = A->n;
    P->nnz = A->nnz;
    P->dtype = A->dtype;
    P->elt = elt_of(A->dtype);
    P->m_pad = round_up(A->m, kRowPad);
    P->var = std::make_unique<Variant>();  // kernel -1: the segments hold the work
    spmv_plan_info &I = P->info;
    I.m = A->m;
    I.n = A->n;
    I.nnz = A->nnz;
    I.dtype = A->dtype;
    I.confidence = -1.0f;
    I.m_pad = P->m_pad;
    I.kernel = -1;
    I.format = -1;
    I.selector_used = mode;
    I.stage_confidence = -1.0f;
    FeatureWork W;
    spmv_features F;
    SMAT_TRY(validate_and_extract(*A, s, F, W, false, &I.t_validate_ms, &I.t_features_ms));
    I.features = F;
    std::vector<int32_t> rp(A->m + 1);
    SMAT_HIP(hipMemcpyAsync(rp.data(), A->row_ptr_dev, sizeof(int32_t) * (A->m + 1),
                            hipMemcpyDeviceToHost, s));
    SMAT_HIP(hipStreamSynchronize(s));
    const int64_t S = std::min<int64_t>({(int64_t)opts.segments, A->m, 64});
    std::vector<int64_t> cut(1, 0);
    for (int64_t k = 1, r = 0; k < S; ++k) {
        const int64_t target = (int64_t)A->nnz * k / S;
        while (r < A->m && rp[r] < target) ++r;
        if (r > cut.back() && r < A->m) cut.push_back(r);
    }
    cut.push_back(A->m);
    spmv_plan_opts co = opts;
    co.segments = 0;
    co.time_baseline = 0;   // reported for the whole plan
    co.log = 0;
    Dev rb;
    SMAT_TRY(rb.alloc(sizeof(int32_t) * (size_t)(A->m + 1)));
    for (size_t k = 0; k + 1 < cut.size(); ++k) {
        const int64_t r0 = cut[k], mk = cut[k + 1] - r0;
        const int32_t base = rp[r0];
        k_rebase_rows<<<(unsigned)((mk + 256) / 256), 256, 0, s>>>(
            mk, (const int32_t *)A->row_ptr_dev + r0, base, rb.as<int32_t>());
        SMAT_LAUNCHED("rebase_rows");
        spmv_csr c{};
        c.m = mk;
        c.n = A->n;
        c.nnz = rp[cut[k + 1]] - base;
        c.row_ptr_dev = rb.as<int32_t>();
        c.col_dev = (const int32_t *)A->col_dev + base;
        c.val_dev = (const char *)A->val_dev + (size_t)P->elt * base;
        c.dtype = A->dtype;
        spmv_plan_t child = nullptr;
        SMAT_TRY(plan_create_impl(&c, &co, s, &child));
        P->seg.push_back(child);
        P->seg_row0.push_back(r0);
        I.device_bytes += child->info.device_bytes;
        I.t_select_ms += child->info.t_plan_ms;
        I.t_tune_ms += child->info.t_tune_ms;
        I.n_measured += child->info.n_measured;
    }
    I.n_segments = (int32_t)P->seg.size();
    I.t_plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                            t_start).count();
    I.t_run_ms = I.t_plain_ms = I.break_even_calls = -1.0;
    if (opts.time_baseline) SMAT_TRY(time_baseline(P.get(), A, opts.timing_reps, s));
    if (opts.log) log_plan(*P);
    *out = P.release();
    return SPMV_OK;
}

static spmv_status plan_create_impl(const spmv_csr *A, const spmv_plan_opts *opts_in,
                                    hipStream_t s, spmv_plan_t *out) {
    auto t_start = std::chrono::steady_clock::now();
    SMAT_TRY(check_csr(A));
    spmv_plan_opts opts;
    if (opts_in)
        opts = *opts_in;
    else
        spmv_plan_opts_default(&opts);
    if (opts.timing_reps <= 0) opts.timing_reps = 5;
    if (opts.measure_topk <= 0) opts.measure_topk = 3;
    if (!(opts.stage_conf > 0.0f)) opts.stage_conf = 0.98f;
    if (opts.staged != 0 && opts.staged != 1) {
        set_error("staged must be 0 or 1");
        return SPMV_EINVAL;
    }
    if (!opts.allocator.alloc != !opts.allocator.free) {
        set_error("allocator needs both alloc and free, or neither");
        return SPMV_EINVAL;
    }
    AllocScope scope(opts.allocator);
    int mode = opts.selector;
    if (mode < 0) mode = opts.model ? SPMV_SELECT_MLP : SPMV_SELECT_RULES;
    if (mode > SPMV_SELECT_FORCED) {
        set_error("unknown selector mode %d", mode);
        return SPMV_EINVAL;
    }
    if (mode == SPMV_SELECT_MLP && !opts.model) {
        set_error("SPMV_SELECT_MLP needs opts.model");
        return SPMV_EINVAL;
    }
    if (mode == SPMV_SELECT_FORCED && (opts.force_kernel < 0 || opts.force_kernel >= SPMV_K_COUNT)) {
        set_error("force_kernel %d out of range", opts.force_kernel);
        return SPMV_EINVAL;
    }
    if (opts.segments < 0) {
        set_error("segments must be >= 0");
        return SPMV_EINVAL;
    }
    if (opts.segments >= 2 && A->m >= 2 && A->nnz > 0)
        return plan_create_segments(A, opts, mode, s, out, t_start);
    auto P = std::make_unique<spmv_plan_s>();
    P->alloc = opts.allocator;
    SMAT_HIP(hipGetDevice(&P->device));
    P->m = A->m;
    P->n = A->n;
    P->nnz = A->nnz;
    P->dtype = A->dtype;
    P->elt = elt_of(A->dtype);
    P->m_pad = round_up(A->m, kRowPad);
    spmv_plan_info &I = P->info;
    I.m = A->m;
    I.n = A->n;
    I.nnz = A->nnz;
    I.dtype = A->dtype;
    I.confidence = -1.0f;
    I.m_pad = P->m_pad;

    FeatureWork W;
    spmv_features F;
    const bool staged = opts.staged == 1 &&
                        (mode == SPMV_SELECT_RULES || mode == SPMV_SELECT_MLP);
    bool may_stop = false;  // can the staged search still stop after the census?
    if (!staged) {
        SMAT_TRY(validate_and_extract(*A, s, F, W, true, &I.t_validate_ms, &I.t_features_ms));
    } else {
        auto t0 = std::chrono::steady_clock::now();
        SMAT_TRY(extract_rows(*A, s, F, W));
        auto t1 = std::chrono::steady_clock::now();
        if (mode == SPMV_SELECT_RULES) {
            may_stop = F.ell_feasible;  // DIA and ELL both need ELL's zero-fill bound
        } else {
            const spmv_selector_s &S = *opts.model;
            may_stop = !S.st_feat.empty();
            if (may_stop && S.has_domain) {  // the inputs known now must be in range
                float raw[12];
                raw_features(F, A->dtype, raw);
                for (int j = 0; j < 12; ++j)
                    if ((kRowInputs >> j) & 1u)
                        may_stop = may_stop && raw[j] >= S.lo[j] && raw[j] <= S.hi[j];
            }
        }
        // without a possible stop, census and rest share one pass
        if (!may_stop)
            SMAT_TRY(extract_entries(*A, s, F, W, kStageCensus | kStageRest, true));
        else if (F.ell_feasible && A->nnz > 0 && !W.census_done)
            SMAT_TRY(extract_entries(*A, s, F, W, kStageCensus, true));
        auto t2 = std::chrono::steady_clock::now();
        I.t_validate_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        I.t_features_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    }
    auto t_sel0 = std::chrono::steady_clock::now();

    uint64_t cap = opts.mem_cap_bytes;
    if (cap == 0) {
        size_t fr = 0, tot = 0;
        SMAT_HIP(hipMemGetInfo(&fr, &tot));
        cap = fr / 4;
    }
    spmv_params prm_base = default_params(0, F);
    if (opts.use_params) {
        merge_params(prm_base, opts.params);
        SMAT_TRY(check_params(prm_base));
    }
    uint32_t feas = feasible_mask(F, A->dtype, P->m_pad, cap, prm_base) & ~opts.disable_mask;

    // ---- staged search (Section 6): settle on DIA, ELL or CSR from the
    // features known so far when the format test is confident, else
    // extract the rest
    int chosen = -1;
    I.stage_confidence = -1.0f;
    if (staged && !may_stop) {
        I.feature_stage = 2;
        if (mode == SPMV_SELECT_MLP && !opts.model->st_feat.empty()) {
            float raw[12];
            raw_features(F, A->dtype, raw);
            I.stage_confidence = opts.model->st_conf[stage_leaf(*opts.model, raw)];
        }
    } else if (staged) {
        if (mode == SPMV_SELECT_RULES) {
            chosen = rules_dia_ell(F, feas);  // the rules' own DIA / ELL tests
        } else if (!opts.model->st_feat.empty()) {
            const spmv_selector_s &S = *opts.model;
            float raw[12];
            raw_features(F, A->dtype, raw);
            bool inside = true;
            if (S.has_domain)
                for (int j = 0; j < 12; ++j)
                    if ((kStageInputs >> j) & 1u)
                        inside = inside && raw[j] >= S.lo[j] && raw[j] <= S.hi[j];
            const int leaf = stage_leaf(S, raw);
            const int k = S.st_kernel[leaf];
            I.stage_confidence = S.st_conf[leaf];
            if (inside && ((kStageKernels & feas) >> k & 1u) &&
                S.st_conf[leaf] >= opts.stage_conf)
                chosen = k;
        }
        if (chosen >= 0) {
            I.feature_stage = 1;
        } else {
            auto t0 = std::chrono::steady_clock::now();
            SMAT_TRY(extract_entries(*A, s, F, W, kStageRest, true));
            I.t_features_ms += std::chrono::duration<double, std::milli>(
                                   std::chrono::steady_clock::now() - t0).count();
            feas = feasible_mask(F, A->dtype, P->m_pad, cap, prm_base) & ~opts.disable_mask;
            I.feature_stage = 2;
        }
    }
    I.features = F;

    // plan-owned CSR copy (every conversion starts from it)
    SMAT_TRY(P->rp.alloc(sizeof(int32_t) * (size_t)(A->m + 1)));
    SMAT_TRY(P->col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, A->nnz)));
    SMAT_TRY(P->val.alloc((size_t)P->elt * (size_t)std::max<int64_t>(1, A->nnz)));
    SMAT_HIP(hipMemcpyAsync(P->rp.p, A->row_ptr_dev, sizeof(int32_t) * (A->m + 1),
                            hipMemcpyDeviceToDevice, s));
    if (A->nnz) {
        SMAT_HIP(hipMemcpyAsync(P->col.p, A->col_dev, sizeof(int32_t) * A->nnz,
                                hipMemcpyDeviceToDevice, s));
        SMAT_HIP(hipMemcpyAsync(P->val.p, A->val_dev, (size_t)P->elt * A->nnz,
                                hipMemcpyDeviceToDevice, s));
    }
    P->has_csr = true;

    I.feasible_mask = feas;
    raw_features(F, A->dtype, I.mlp_input);
    // an early stop leaves R unknown: the rules' pick is known only when
    // their DIA / ELL tests decide
    I.rules_kernel = I.feature_stage == 1 ? rules_dia_ell(F, feas) : rules_choose(F, feas);

    // ---- selection
    std::vector<int> cands;
    I.selector_used = mode;
    if (chosen >= 0) {
        // settled by the staged search
    } else if (mode == SPMV_SELECT_FORCED) {
        uint32_t all = feasible_mask(F, A->dtype, P->m_pad, ~0ull, prm_base, false);
        bool structural_ok = (all >> opts.force_kernel) & 1u;
        // DIA and ELL need their zero-fill feasibility; the others always run
        if (!structural_ok && (opts.force_kernel == SPMV_K_DIA || opts.force_kernel == SPMV_K_DIA_DIRECT ||
                               opts.force_kernel == SPMV_K_ELL || opts.force_kernel == SPMV_K_BCSR)) {
            set_error("forced kernel %s is infeasible for this matrix (zero fill)",
                      spmv_kernel_name(opts.force_kernel));
            return SPMV_EINVAL;
        }
        if ((opts.force_kernel == SPMV_K_DIA || opts.force_kernel == SPMV_K_DIA_DIRECT) && !W.diag_hist.p) {
            set_error("forced DIA without a diagonal census");
            return SPMV_EINVAL;
        }
        chosen = opts.force_kernel;
    } else if (mode == SPMV_SELECT_RULES) {
        chosen = rules_choose(F, feas);
    } else if (mode == SPMV_SELECT_EXHAUSTIVE) {
        for (int k = 0; k < SPMV_K_COUNT; ++k)
            if ((feas >> k) & 1u) cands.push_back(k);
    } else {  // MLP
        spmv_selector_s *sel = opts.model;
        float raw[12];
        raw_features(F, A->dtype, raw);
        Dev draw, dsc;
        SMAT_TRY(draw.alloc(sizeof(raw)));
        SMAT_TRY(dsc.alloc(sizeof(float) * SPMV_K_COUNT));
        SMAT_HIP(hipMemcpyAsync(draw.p, raw, sizeof(raw), hipMemcpyHostToDevice, s));
        SMAT_TRY(run_mlp_infer(sel->params.as<float>(), sel->n_out, sel->mean.as<float>(),
                               sel->stdv.as<float>(), draw.as<float>(), 1, dsc.as<float>(), s));
        float sc[SPMV_K_COUNT];
        SMAT_HIP(hipMemcpyAsync(sc, dsc.p, sizeof(sc), hipMemcpyDeviceToHost, s));
        SMAT_HIP(hipStreamSynchronize(s));
        std::vector<std::pair<float, int>> order;
        for (int k = 0; k < SPMV_K_COUNT; ++k) {
            I.mlp_scores[k] = sc[k];
            if ((feas >> k) & 1u) order.push_back({sc[k], k});
        }
        std::sort(order.begin(), order.end());
        bool outside = false;
        if (sel->has_domain)
            for (int j = 0; j < 12; ++j)
                outside = outside || !(raw[j] >= sel->lo[j] && raw[j] <= sel->hi[j]);
        I.out_of_domain = outside ? 1 : 0;
        if (order.empty()) {
            chosen = SPMV_K_CSR_ADAPTIVE;
        } else if (outside && order.size() > 1) {
            // extrapolation: the scores are not evidence, measure them all
            I.confidence = order[1].first - order[0].first;
            for (auto &o : order) cands.push_back(o.second);
        } else {
            float margin = order.size() > 1 ? order[1].first - order[0].first : 1e30f;
            I.confidence = margin;
            if (margin >= opts.confidence_tau || order.size() == 1) {
                chosen = order[0].second;
            } else {
                for (size_t q = 0; q < order.size() && (int)q < opts.measure_topk; ++q)
                    cands.push_back(order[q].second);
            }
        }
    }
    if (chosen < 0 && cands.empty()) chosen = SPMV_K_CSR_ADAPTIVE;

    // ---- execute and measure the candidates, keep the fastest
    if (chosen < 0) {
        Dev xs, ys;
        SMAT_TRY(xs.alloc((size_t)P->elt * std::max<int64_t>(1, P->n)));
        SMAT_TRY(ys.alloc((size_t)P->elt * std::max<int64_t>(1, P->m)));
        if (P->n)
            k_fill_one<<<(unsigned)((P->n + 255) / 256), 256, 0, s>>>(P->n, P->elt, xs.p);
        SMAT_LAUNCHED("fill_one");
        double best = 1e300;
        for (int k : cands) {
            auto V = std::make_unique<Variant>();
            spmv_status st = build_variant(*P, F, W, k, prm_base, s, *V);
            if (st == SPMV_ENOMEM || st == SPMV_EUNSUPPORTED) continue;  // cannot be built
            if (st != SPMV_OK) return st;
            double ms = 0;
            SMAT_TRY(time_variant(*P, *V, xs.p, ys.p, opts.timing_reps, s, &ms));
            I.measured_kernel[I.n_measured] = k;
            I.measured_ms[I.n_measured] = ms;
            ++I.n_measured;
            // exhaustive timing keeps the plain minimum; after a prediction
            // (candidates in score order) a later one must win clearly
            const double margin = mode == SPMV_SELECT_EXHAUSTIVE ? 0.0 : kSwitchMargin;
            if (chosen < 0 || ms < best * (1.0 - margin)) {
                best = ms;
                chosen = k;
                P->var = std::move(V);
            }
        }
        if (chosen < 0) {
            set_error("no candidate kernel could be built");
            return SPMV_ENOMEM;
        }
    }
    auto t_conv0 = std::chrono::steady_clock::now();
    if (!P->var) {
        P->var = std::make_unique<Variant>();
        spmv_status st = build_variant(*P, F, W, chosen, prm_base, s, *P->var);
        if (st == SPMV_ENOMEM && mode != SPMV_SELECT_FORCED) {
            // fall back to CSR once (needs no extra storage)
            P->var = std::make_unique<Variant>();
            chosen = SPMV_K_CSR_VECTOR;
            SMAT_TRY(build_variant(*P, F, W, chosen, prm_base, s, *P->var));
        } else if (st != SPMV_OK) {
            return st;
        }
    }
    if (opts.autotune && !opts.use_params) {
        auto t_tune0 = std::chrono::steady_clock::now();
        SMAT_TRY(autotune_variant(*P, F, W, opts.timing_reps, s, P->var, &I.tune_rejected));
        SMAT_HIP(hipStreamSynchronize(s));
        I.t_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                t_tune0).count();
    }
    SMAT_HIP(hipStreamSynchronize(s));
    W.diag_hist.release();
    if (!needs_csr(*P->var)) {
        P->rp.release();
        P->col.release();
        P->val.release();
        P->has_csr = false;
    }
    auto t_end = std::chrono::steady_clock::now();
    I.kernel = chosen;
    I.format = (chosen <= SPMV_K_CSR_ADAPTIVE || chosen == SPMV_K_CSR_PANEL) ? SPMV_FMT_CSR
               : chosen == SPMV_K_ELL          ? SPMV_FMT_ELL
               : chosen == SPMV_K_COO          ? SPMV_FMT_COO
               : chosen == SPMV_K_BCSR         ? SPMV_FMT_BCSR
                                               : SPMV_FMT_DIA;
    I.bcsr_blocks = P->var->nblocks;
    I.long_lanes = P->var->long_tpr;
    I.long_rows = P->var->n_long;
    I.params = P->var->prm;
    I.ell_width = P->var->K;
    I.dia_ndiags = P->var->D;
    I.dia_windows = P->var->nwin;
    I.device_bytes = P->rp.bytes + P->col.bytes + P->val.bytes + P->var->bytes();
    I.t_select_ms = std::chrono::duration<double, std::milli>(t_conv0 - t_sel0).count();
    I.t_convert_ms = std::chrono::duration<double, std::milli>(t_end - t_conv0).count();
    I.t_plan_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    I.t_run_ms = I.t_plain_ms = I.break_even_calls = -1.0;
    if (opts.time_baseline) SMAT_TRY(time_baseline(P.get(), A, opts.timing_reps, s));
    if (opts.log) log_plan(*P);
    *out = P.release();
    return SPMV_OK;
}

extern "C" spmv_status spmv_plan_create(const spmv_csr *A, const spmv_plan_opts *opts,
                                        void *stream, spmv_plan_t *out) {
    if (!out) {
        set_error("out is NULL");
        return SPMV_EINVAL;
    }
    *out = nullptr;
    try {
        const spmv_plan_opts o = effective_opts(opts);
        return plan_create_impl(A, &o, (hipStream_t)stream, out);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SPMV_ENOMEM;
    }
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

extern "C" spmv_status spmv_run(spmv_plan_t P, const void *x, void *y, void *stream) {
    if (!P) {
        set_error("plan is NULL");
        return SPMV_EINVAL;
    }
    if (P->m == 0) return SPMV_OK;
    if (!y || (P->n > 0 && !x)) {
        set_error("x or y is NULL");
        return SPMV_EINVAL;
    }
    if (overlap(x, (size_t)P->elt * P->n, y, (size_t)P->elt * P->m)) {
        set_error("x and y overlap");
        return SPMV_EINVAL;
    }
    if (!P->seg.empty()) {
        for (size_t k = 0; k < P->seg.size(); ++k)
            SMAT_TRY(spmv_run(P->seg[k], x, (char *)y + (size_t)P->elt * P->seg_row0[k], stream));
        return SPMV_OK;
    }
    return run_variant(*P, *P->var, x, y, (hipStream_t)stream);
}

extern "C" spmv_status spmv_plan_segment(spmv_plan_t P, int32_t k, spmv_plan_t *segment,
                                         int64_t *row0) {
    if (!P || P->seg.empty() || k < 0 || k >= (int32_t)P->seg.size()) {
        set_error("plan is not segmented or segment %d does not exist", k);
        return SPMV_EINVAL;
    }
    if (segment) *segment = P->seg[k];
    if (row0) *row0 = P->seg_row0[k];
    return SPMV_OK;
}

extern "C" spmv_status spmv_plan_info_get(spmv_plan_t P, spmv_plan_info *out) {
    if (!P || !out) {
        set_error("plan or out is NULL");
        return SPMV_EINVAL;
    }
    *out = P->info;
    return SPMV_OK;
}

extern "C" spmv_status spmv_plan_destroy(spmv_plan_t P) {
    if (!P) return SPMV_OK;
    // Memory from a caller's allocator goes back to the caller, who may hand
    // it out again at once, while runs of this plan on any stream may still
    // read it: the plan's device is synchronised first.  (hipFree, the
    // default, synchronises by itself.)
    spmv_status st = SPMV_OK;
    if (P->alloc.free) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && P->device >= 0 && cur != P->device) e = hipSetDevice(P->device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) st = hip_fail(e, "spmv_plan_destroy: device synchronisation");
        if (cur >= 0 && cur != P->device) (void)hipSetDevice(cur);
    }
    delete P;
    return st;
}

extern "C" spmv_status spmv_convert_roundtrip(spmv_plan_t P, int32_t *rp, int32_t *col, void *val,
                                              void *stream) {
    if (!P || !rp || (P->nnz > 0 && (!col || !val))) {
        set_error("NULL argument");
        return SPMV_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    AllocScope scope(P->alloc);
    if (!P->seg.empty()) {
        // each segment rebuilds its rows; their row pointers are shifted by
        // the entries before the segment (its last entry is the next start)
        int64_t base = 0;
        for (size_t k = 0; k < P->seg.size(); ++k) {
            const spmv_plan_s &C = *P->seg[k];
            const int64_t r0 = P->seg_row0[k];
            SMAT_TRY(spmv_convert_roundtrip(P->seg[k], rp + r0, col + base,
                                            (char *)val + (size_t)P->elt * base, stream));
            k_offset_rows<<<(unsigned)((C.m + 256) / 256), 256, 0, s>>>(C.m, rp + r0,
                                                                        (int32_t)base);
            SMAT_LAUNCHED("offset_rows");
            base += C.nnz;
        }
        SMAT_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    const Variant &V = *P->var;
    const int64_t m = P->m, nnz = P->nnz;
    const int elt = P->elt;
    Dev counts, scan;
    SMAT_TRY(counts.alloc(sizeof(int32_t) * std::max<int64_t>(1, m)));
    SMAT_TRY(scan.alloc(sizeof(unsigned) * (size_t)(m / 4096 + 2)));
    switch (V.kernel) {
    case SPMV_K_CSR_SCALAR:
    case SPMV_K_CSR_VECTOR:
    case SPMV_K_CSR_ADAPTIVE:
        SMAT_HIP(hipMemcpyAsync(rp, P->rp.p, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToDevice, s));
        if (nnz) {
            SMAT_HIP(hipMemcpyAsync(col, P->col.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
            SMAT_HIP(hipMemcpyAsync(val, P->val.p, (size_t)elt * nnz, hipMemcpyDeviceToDevice, s));
        }
        break;
    case SPMV_K_COO:
        SMAT_TRY(launch_coo_to_csr(m, nnz, V.row_idx.as<int32_t>(), rp, s));
        if (nnz) {
            SMAT_HIP(hipMemcpyAsync(col, P->col.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
            SMAT_HIP(hipMemcpyAsync(val, P->val.p, (size_t)elt * nnz, hipMemcpyDeviceToDevice, s));
        }
        break;
    case SPMV_K_ELL:
        SMAT_TRY(launch_ell_to_csr(m, P->m_pad, V.K, V.ecol.as<int32_t>(), V.eval.p, elt, rp, col,
                                   val, counts.as<int32_t>(), scan.as<unsigned>(), s));
        break;
    case SPMV_K_BCSR:
        SMAT_TRY(launch_bcsr_to_csr(m, V.brp.as<int32_t>(), V.bcol.as<int32_t>(), V.bval.p,
                                    V.bpres.as<uint16_t>(), elt, rp, col, val,
                                    counts.as<int32_t>(), scan.as<unsigned>(), s));
        break;
    case SPMV_K_CSR_PANEL:
        SMAT_TRY(launch_panels_to_csr(m, V.bin_rows.as<int32_t>(), V.P, V.prow.as<int32_t>(),
                                      V.pcol.as<int32_t>(), V.pval.p, elt, rp, col, val,
                                      counts.as<int32_t>(), scan.as<unsigned>(), s));
        break;
    case SPMV_K_DIA:
    case SPMV_K_DIA_DIRECT:
        SMAT_TRY(launch_dia_to_csr(m, P->n, P->m_pad, V.D, V.dia_off.as<int32_t>(), V.dia_data.p,
                                   V.dia_present.as<uint32_t>(), elt, rp, col, val,
                                   counts.as<int32_t>(), scan.as<unsigned>(), s));
        break;
    default:
        set_error("plan holds no kernel");
        return SPMV_EINVAL;
    }
    SMAT_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

extern "C" spmv_status spmv_plan_export(spmv_plan_t P, int32_t which, void *dst, size_t bytes,
                                        size_t *bytes_out, void *stream) {
    if (!P) {
        set_error("plan is NULL");
        return SPMV_EINVAL;
    }
    const Variant &V = *P->var;
    const void *src = nullptr;
    size_t n = 0;
    switch (which) {
    case 0:
        if (V.kernel == SPMV_K_COO) { src = V.row_idx.p; n = sizeof(int32_t) * P->nnz; }
        break;
    case 1:
        if (V.kernel == SPMV_K_ELL) { src = V.ecol.p; n = sizeof(int32_t) * (size_t)V.K * P->m_pad; }
        break;
    case 2:
        if (V.kernel == SPMV_K_ELL) { src = V.eval.p; n = (size_t)P->elt * V.K * P->m_pad; }
        break;
    case 3:
        if (V.kernel == SPMV_K_DIA || V.kernel == SPMV_K_DIA_DIRECT) { src = V.dia_off.p; n = sizeof(int32_t) * V.D; }
        break;
    case 4:
        if (V.kernel == SPMV_K_DIA || V.kernel == SPMV_K_DIA_DIRECT) { src = V.dia_data.p; n = (size_t)P->elt * V.D * P->m_pad; }
        break;
    case 5:
        if (V.kernel == SPMV_K_DIA || V.kernel == SPMV_K_DIA_DIRECT) { src = V.dia_present.p; n = sizeof(uint32_t) * (((size_t)V.D * P->m_pad + 31) / 32); }
        break;
    case 6:
        if (V.kernel == SPMV_K_CSR_ADAPTIVE || V.kernel == SPMV_K_CSR_PANEL) { src = V.bin_rows.p; n = sizeof(int32_t) * P->m; }
        break;
    case 7:
        if (V.kernel == SPMV_K_BCSR) { src = V.brp.p; n = sizeof(int32_t) * (size_t)((P->m + 3) / 4 + 1); }
        break;
    case 8:
        if (V.kernel == SPMV_K_BCSR) { src = V.bcol.p; n = sizeof(int32_t) * (size_t)V.nblocks; }
        break;
    case 9:
        if (V.kernel == SPMV_K_BCSR) { src = V.bval.p; n = (size_t)P->elt * 16 * (size_t)V.nblocks; }
        break;
    case 10:
        if (V.kernel == SPMV_K_BCSR) { src = V.bpres.p; n = sizeof(uint32_t) * (size_t)((V.nblocks + 1) / 2); }
        break;
    default:
        break;
    }
    if (!src && n == 0 && which >= 0 && which <= 10 && bytes_out) {
        // an empty array of a present format
    }
    if (!src) {
        set_error("plan has no array %d", which);
        return SPMV_EINVAL;
    }
    if (bytes_out) *bytes_out = n;
    if (!dst) return SPMV_OK;  // size query
    if (bytes < n) {
        set_error("destination too small (%zu < %zu)", bytes, n);
        return SPMV_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (n) SMAT_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s));
    SMAT_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

extern "C" spmv_status spmv_selector_create(const float *params, int64_t n_params,
                                            const float *mean, const float *stdv,
                                            spmv_selector_t *out) {
    if (!out || !params || !mean || !stdv) {
        set_error("NULL argument");
        return SPMV_EINVAL;
    }
    *out = nullptr;
    if (n_params != spmv_mlp_param_count(SPMV_K_COUNT)) {
        set_error("selector expects %lld parameters, got %lld",
                  (long long)spmv_mlp_param_count(SPMV_K_COUNT), (long long)n_params);
        return SPMV_EINVAL;
    }
    for (int i = 0; i < 12; ++i)
        if (!(stdv[i] > 0.0f)) {
            set_error("std[%d] must be > 0", i);
            return SPMV_EINVAL;
        }
    auto S = std::make_unique<spmv_selector_s>();
    S->n_out = SPMV_K_COUNT;
    SMAT_TRY(S->params.alloc(sizeof(float) * n_params));
    SMAT_TRY(S->mean.alloc(sizeof(float) * 12));
    SMAT_TRY(S->stdv.alloc(sizeof(float) * 12));
    SMAT_HIP(hipMemcpy(S->params.p, params, sizeof(float) * n_params, hipMemcpyHostToDevice));
    SMAT_HIP(hipMemcpy(S->mean.p, mean, sizeof(float) * 12, hipMemcpyHostToDevice));
    SMAT_HIP(hipMemcpy(S->stdv.p, stdv, sizeof(float) * 12, hipMemcpyHostToDevice));
    *out = S.release();
    return SPMV_OK;
}

extern "C" spmv_status spmv_selector_set_domain(spmv_selector_t S, const float *lo,
                                                const float *hi) {
    if (!S || (!lo) != (!hi)) {
        set_error("selector handle and both or neither of lo / hi required");
        return SPMV_EINVAL;
    }
    if (!lo) {
        S->has_domain = false;
        return SPMV_OK;
    }
    for (int j = 0; j < 12; ++j)
        if (!(lo[j] <= hi[j])) {
            set_error("domain lo[%d] > hi[%d]", j, j);
            return SPMV_EINVAL;
        }
    std::copy(lo, lo + 12, S->lo);
    std::copy(hi, hi + 12, S->hi);
    S->has_domain = true;
    return SPMV_OK;
}

extern "C" spmv_status spmv_selector_set_stage(spmv_selector_t S, const int32_t *feat,
                                               const float *thr, const int32_t *left,
                                               const int32_t *right, const int32_t *kernel,
                                               const float *conf, int32_t n_nodes) {
    if (!S || n_nodes < 0 || n_nodes > 4096 ||
        (n_nodes > 0 && (!feat || !thr || !left || !right || !kernel || !conf))) {
        set_error("selector handle, 0 <= n_nodes <= 4096 and all six arrays required");
        return SPMV_EINVAL;
    }
    for (int i = 0; i < n_nodes; ++i) {
        if (feat[i] == -1) {
            if (kernel[i] < 0 || kernel[i] >= SPMV_K_COUNT || !(conf[i] >= 0.0f && conf[i] <= 1.0f)) {
                set_error("stage leaf %d: kernel %d or confidence out of range", i, kernel[i]);
                return SPMV_EINVAL;
            }
        } else if (feat[i] < 0 || feat[i] >= 12 || !((kStageInputs >> feat[i]) & 1u)) {
            set_error("stage node %d tests input %d, not known after the census", i, feat[i]);
            return SPMV_EINVAL;
        } else if (left[i] <= i || right[i] <= i || left[i] >= n_nodes || right[i] >= n_nodes ||
                   !std::isfinite(thr[i])) {
            set_error("stage node %d: children must lie in (%d, %d), threshold finite", i, i,
                      n_nodes);
            return SPMV_EINVAL;
        }
    }
    S->st_feat.assign(feat, feat + n_nodes);
    S->st_thr.assign(thr, thr + n_nodes);
    S->st_left.assign(left, left + n_nodes);
    S->st_right.assign(right, right + n_nodes);
    S->st_kernel.assign(kernel, kernel + n_nodes);
    S->st_conf.assign(conf, conf + n_nodes);
    return SPMV_OK;
}

extern "C" spmv_status spmv_selector_destroy(spmv_selector_t S) {
    delete S;
    return SPMV_OK;
}

extern "C" spmv_status spmv_selector_score(spmv_selector_t S, const float *raw, int64_t rows,
                                           float *scores, void *stream) {
    if (!S || (rows > 0 && (!raw || !scores)) || rows < 0) {
        set_error("bad argument");
        return SPMV_EINVAL;
    }
    return run_mlp_infer(S->params.as<float>(), S->n_out, S->mean.as<float>(), S->stdv.as<float>(),
                         raw, rows, scores, (hipStream_t)stream);
}

extern "C" int64_t spmv_gather_probe_threads(void) { return gather_probe_threads(); }

extern "C" spmv_status spmv_gather_probe(const void *table, int64_t table_len, const int32_t *idx,
                                         const void *val, int64_t count, int32_t elt, void *out,
                                         void *stream) {
    if ((elt != 4 && elt != 8) || count < 0 || table_len < 1 || !out ||
        (count > 0 && (!table || !idx || !val))) {
        set_error("gather_probe: elt 4 or 8, count >= 0, table_len >= 1, buffers required");
        return SPMV_EINVAL;
    }
    return run_gather_probe(table, idx, val, count, elt, out, (hipStream_t)stream);
}

extern "C" size_t spmv_stream_read_out_bytes(void) { return stream_read_out_bytes(); }

extern "C" spmv_status spmv_stream_read(const void *src, size_t bytes, void *out, void *stream) {
    if (!src || !out || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)out % 16) {
        set_error("stream_read needs 16-byte aligned buffers and a multiple of 16 bytes");
        return SPMV_EINVAL;
    }
    return run_stream_read(src, bytes, out, (hipStream_t)stream);
}

extern "C" spmv_status spmv_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) {
        set_error("stream_copy needs 16-byte aligned buffers and a multiple of 16 bytes");
        return SPMV_EINVAL;
    }
    return run_stream_copy(dst, src, bytes, (hipStream_t)stream);
}

