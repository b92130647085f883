// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spmv.h"

namespace smat {

constexpr int kWave = 64;           // gfx9 wavefront width
constexpr int kRowPad = 64;         // ELL / DIA slot stride is m rounded up to this
constexpr int kFp64MaxDepth = 4096; // longest sequential float64 summation chain
constexpr int kAdaptiveBins = 9;    // widths 1..64 (7 bins) + workgroup + split

void set_error(const char *fmt, ...);
spmv_status hip_fail(hipError_t e, const char *what);

#define SMAT_HIP(expr)                                                   \
    do {                                                                 \
        hipError_t _e = (expr);                                          \
        if (_e != hipSuccess) return ::smat::hip_fail(_e, #expr);        \
    } while (0)

#define SMAT_LAUNCHED(what)                                              \
    do {                                                                 \
        hipError_t _e = hipGetLastError();                               \
        if (_e != hipSuccess) return ::smat::hip_fail(_e, what);         \
    } while (0)

// ----------------------------------------------------------------- K0 / K1
// Validation flags.
enum : uint32_t {
    kBadRowPtr0 = 1u, kBadRowPtrEnd = 2u, kBadRowPtrOrder = 4u,
    kBadColRange = 8u, kBadColOrder = 16u,
};

struct RowStats {       // device-side reduction target for the row pass
    unsigned long long sum_rd, sum_rd2;
    int max_rd, min_rd;
};

struct EntryStats {     // device-side reduction targets of the entry passes
    unsigned long long blocks4;  // block pass
    int bandwidth;               // column validation
    int pad;
};

struct DiagStats {
    unsigned long long ndiags, ntrue;
};

spmv_status launch_validate_rows(int64_t m, int64_t nnz, const int32_t *rp, uint32_t *flags,
                                 hipStream_t s);
spmv_status launch_validate_entries(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                                    const int32_t *col, uint32_t *flags, int *bandwidth,
                                    hipStream_t s);
spmv_status launch_row_stats(int64_t m, const int32_t *rp, RowStats *out, hipStream_t s);
spmv_status launch_row_hist(int64_t m, const int32_t *rp, int max_rd, unsigned int *hist,
                            hipStream_t s);
spmv_status launch_powerlaw_fit(const unsigned int *hist, int max_rd, int64_t m, double *sums,
                                hipStream_t s);
spmv_status launch_entry_stats(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                               const int32_t *col, EntryStats *out, unsigned int *diag_hist,
                               bool blocks, hipStream_t s, const uint32_t *gate = nullptr,
                               const RowStats *gate_rs = nullptr);
spmv_status launch_diag_stats(int64_t m, int64_t n, const unsigned int *diag_hist, DiagStats *out,
                              hipStream_t s);
spmv_status launch_diag_compact(int64_t m, int64_t n, unsigned int *diag_hist, int32_t *offsets,
                                unsigned int *block_scratch, hipStream_t s);

// ----------------------------------------------------------------- K2 / K5
spmv_status launch_csr_to_coo(int64_t m, int64_t nnz, const int32_t *rp, int32_t *row_idx,
                              hipStream_t s);
spmv_status launch_csr_to_ell(int64_t m, int64_t m_pad, int K, const int32_t *rp,
                              const int32_t *col, const void *val, int elt, int32_t *ecol,
                              void *eval, hipStream_t s);
spmv_status launch_csr_to_dia(int64_t m, int64_t n, int64_t m_pad, int64_t nnz, const int32_t *rp,
                              const int32_t *col, const void *val, int elt,
                              const unsigned int *slot_map, void *data, uint32_t *present,
                              hipStream_t s);
spmv_status launch_coo_to_csr(int64_t m, int64_t nnz, const int32_t *row_idx, int32_t *rp,
                              hipStream_t s);
spmv_status launch_ell_to_csr(int64_t m, int64_t m_pad, int K, const int32_t *ecol,
                              const void *eval, int elt, int32_t *rp, int32_t *col, void *val,
                              int32_t *counts, unsigned int *scratch, hipStream_t s);
spmv_status launch_dia_to_csr(int64_t m, int64_t n, int64_t m_pad, int D, const int32_t *offs,
                              const void *data, const uint32_t *present, int elt, int32_t *rp,
                              int32_t *col, void *val, int32_t *counts, unsigned int *scratch,
                              hipStream_t s);
// 4x4 block CSR (block row R = rows 4R..4R+3): block counts per block row
// and their exclusive scan (brp, ceil(m/4)+1 entries; scratch as below),
// then block columns, zero-filled-beforehand values (16 per block,
// row-major) and 16 presence bits per block; the inverse for round trips.
spmv_status launch_bcsr_count(int64_t m, const int32_t *rp, const int32_t *col, int32_t *counts,
                              int32_t *brp, unsigned int *scratch, hipStream_t s);
spmv_status launch_csr_to_bcsr(int64_t m, const int32_t *rp, const int32_t *col, const void *val,
                               int elt, const int32_t *brp, int32_t *bcol, void *bval,
                               uint16_t *pres, hipStream_t s);
spmv_status launch_bcsr_to_csr(int64_t m, const int32_t *brp, const int32_t *bcol,
                               const void *bval, const uint16_t *pres, int elt, int32_t *rp,
                               int32_t *col, void *val, int32_t *counts, unsigned int *scratch,
                               hipStream_t s);
// BCSR SpMV: `lanes` lanes per block row (power of two <= 64).
spmv_status run_bcsr(int elt, bool nt, int64_t m, int64_t n, const int32_t *brp,
                     const int32_t *bcol, const void *bval, const void *x, void *y, int lanes,
                     int block, hipStream_t s);
// scratch: at least ceil(m / 4096) unsigned ints
spmv_status launch_exclusive_scan_rows(int64_t m, const int32_t *counts, int32_t *rp,
                                       unsigned int *scratch, hipStream_t s);

// Row binning for CSR_ADAPTIVE: bin_of(len) in [0, kAdaptiveBins).
struct BinSpec {
    int upper[kAdaptiveBins];   // inclusive upper row length per bin
};
spmv_status launch_bin_rows(int64_t m, const int32_t *rp, const BinSpec &spec,
                            unsigned int *block_counts, int32_t *rows_out,
                            unsigned int *bin_offsets_dev, hipStream_t s);

// ----------------------------------------------------------------- SpMV
struct DiaWindow { int d0, d1; };   // diagonals [d0, d1] share one LDS window

spmv_status run_csr_scalar(int elt, int64_t m, const int32_t *rp, const int32_t *col,
                           const void *val, const void *x, void *y, int block, hipStream_t s);
// `nt`: stream the matrix arrays with non-temporal loads.
spmv_status run_csr_vector(int elt, bool nt, int lanes, int64_t nrows, const int32_t *rp,
                           const int32_t *col, const void *val, const void *x, void *y, int block,
                           hipStream_t s);
// One launch over all length bins.  Launch position q (q = 0..7) serves bin
// 7 - q; first[q] is its first workgroup, first[8] the grid size.  Bin b holds
// rows[row_begin[b] .. row_begin[b+1]); bin 7 gives a 256-thread workgroup to
// each row, bins 6..0 give 64..1 lanes (256 / L rows per workgroup).
struct AdaptiveLaunch {
    unsigned first[9];
    unsigned row_begin[9];
    int lane_shift;   // column panels: lane width of bin b is 2^max(0, b - shift)
};
// rest: the launch geometry leaves out the longest bin (another kernel
// takes those rows); launched under its own kernel name.
// pk: rp / col / val are the copy in binned order (launch_pack_binned),
// indexed by binned position, instead of the plan's CSR indexed by row.
spmv_status run_csr_adaptive(int elt, bool nt, bool rest, const AdaptiveLaunch &a,
                             const int32_t *rows, const int32_t *rp, const int32_t *col,
                             const void *val, const void *x, void *y, hipStream_t s,
                             bool pk = false);
// Copy of the entries of the rows at binned positions [0, hi) in that order:
// launch_binned_scan fills brp (hi + 1 ints: each position's first entry,
// then the total; len hi ints and scan hi / 4096 + 2 unsigned of scratch),
// launch_pack_binned the entries bcol / bval (brp[hi] of them).
spmv_status launch_binned_scan(int64_t hi, const int32_t *rows, const int32_t *rp, int32_t *len,
                               unsigned *scan, int32_t *brp, hipStream_t s);
spmv_status launch_pack_binned(int64_t hi, const int32_t *rows, const int32_t *rp,
                               const int32_t *col, const void *val, int elt, const int32_t *brp,
                               int32_t *bcol, void *bval, hipStream_t s);
// Column panels; prow is P x (m+1) position-indexed segment starts.  With
// `partial` (P x m values) all panels run in one launch, one per XCD, and a
// second kernel adds the partials of binned positions [red_lo, red_hi);
// without it, one launch per panel.  `part`: the geometry leaves some bins
// to other kernels (launched under the *_rest kernel names).
spmv_status run_csr_panels(int elt, bool nt, const AdaptiveLaunch &a, const int32_t *rows, int P,
                           int64_t m, const int32_t *prow, const int32_t *pcol, const void *pval,
                           const void *x, void *y, void *partial, int64_t red_lo,
                           int64_t red_hi, bool part, hipStream_t s);
// float64 long rows (the binned order's longest bin) with x streamed through
// LDS; tpr (32 or 64) lanes per row.  prepare() raises the kernels' dynamic
// LDS limit (call before the first launch, outside graph capture).
spmv_status long_rows_lds_prepare();
spmv_status run_long_rows_lds(int tpr, int64_t nrows, const int32_t *rows, const int32_t *rp,
                              const int32_t *col, const double *val, const double *x, int64_t n,
                              double *y, hipStream_t s);
// Long rows by tiles: x panels of long_tile_width(elt) values, workgroup
// (row block, panel).  seg: (P + 1) * n7 segment starts in CSR positions,
// filled by launch_long_tile_seg from the rows (ascending columns); blocks:
// nblocks triples (first row, end row, log2 lanes per row) over the rows'
// order.  The entries are packed by launch_long_tile_pack in (row block,
// panel, row) order: pk[k], k = P r0 + p (r1 - r0) + (r - r0) for the block
// [r0, r1) holding r, is row r's first entry in panel p and pk[k + 1] its
// end (P n7 + 1 ints); off (16-bit column - p W) and val hold the packed
// entries, kb two ints per row (k at p = 0, r1 - r0).  part: P * n7 float64
// partials.  y receives the rows rows[0 .. n7).
int64_t long_tile_width(int elt);
// Raises the tile kernels' dynamic LDS limit (before the first launch,
// outside graph capture).
spmv_status long_tiles_prepare();
spmv_status launch_long_tile_seg(int64_t n7, int64_t P, int64_t W, const int32_t *rows,
                                 const int32_t *rp, const int32_t *col, int32_t *seg,
                                 hipStream_t s);
spmv_status launch_long_tile_pack(int64_t n7, int64_t P, int64_t W, const int32_t *rows,
                                  const int32_t *rp, const int32_t *col, const void *val, int elt,
                                  const int32_t *seg, const int32_t *kb, const int32_t *pk,
                                  uint16_t *off, void *pval, hipStream_t s);
// reduce false: the tiles' partials only, added later by
// run_csr_adaptive_tiles.
spmv_status run_long_tiles(int elt, int64_t n7, int64_t P, int64_t nblocks,
                           const int32_t *blocks, const int32_t *pk, const int32_t *rows,
                           const uint16_t *off, const void *val, const void *x, int64_t n,
                           double *part, void *y, hipStream_t s, bool reduce = true);
// After run_long_tiles(..., reduce = false): the binned launch `a` of the
// short rows (entries from the binned-order copy) and the sums of the n7
// long rows' P panel partials `part` into y[lrows[r]], in one launch.
spmv_status run_csr_adaptive_tiles(int elt, bool nt, const AdaptiveLaunch &a, const int32_t *rows,
                                   const int32_t *rp, const int32_t *col, const void *val,
                                   const void *x, void *y, int64_t n7, int64_t P,
                                   const int32_t *lrows, const double *part, hipStream_t s);
// Build column panels of width w from a CSR matrix whose rows are visited in
// the binned order `rows`.  cnt: P*(m+1) ints; prow: P*(m+1)+1 ints; inv: m
// ints; scan: P*(m+1)/4096+1 unsigned.
spmv_status launch_csr_to_panels(int64_t m, int64_t nnz, const int32_t *rp, const int32_t *col,
                                 const void *val, int elt, const int32_t *rows, int P, int64_t w,
                                 int32_t *inv, int32_t *cnt, int32_t *prow, unsigned *scan,
                                 int32_t *pcol, void *pval, hipStream_t s);
// Inverse: rebuild CSR (row_ptr m+1, col, val) from the panels.
spmv_status launch_panels_to_csr(int64_t m, const int32_t *rows, int P, const int32_t *prow,
                                 const int32_t *pcol, const void *pval, int elt, int32_t *rp,
                                 int32_t *col, void *val, int32_t *counts, unsigned *scan,
                                 hipStream_t s);
// split rows: segments (row, begin, end) reduce into partials, then fix-up
spmv_status run_csr_split(int elt, int64_t nseg, const int64_t *segs, double *partials,
                          int64_t nrows, const int64_t *row_seg_begin, const int32_t *rows,
                          const int32_t *col, const void *val, const void *x, void *y,
                          hipStream_t s);
spmv_status run_ell(int elt, bool nt, int64_t m, int64_t m_pad, int K, const int32_t *ecol,
                    const void *eval, const void *x, void *y, int block, int unroll, bool wide,
                    hipStream_t s);
spmv_status run_dia(int elt, bool nt, bool lds, int64_t m, int64_t n, int64_t m_pad, int D,
                    const int32_t *offs_dev, int nwin, const DiaWindow *win_dev, int max_span,
                    const void *data, const void *x, void *y, int block, int rows_per_thread,
                    bool wide, hipStream_t s);
spmv_status run_coo(int elt, bool nt, int64_t m, int64_t nnz, const int32_t *row_idx,
                    const int32_t *col, const void *val, const void *x, void *y, int chunk,
                    double *head, double *tail, uint32_t *flags, hipStream_t s);
spmv_status run_fill_zero(int elt, int64_t m, void *y, hipStream_t s);

// ----------------------------------------------------------------- MLP
spmv_status run_mlp_infer(const float *params, int n_out, const float *mean, const float *stdv,
                          const float *raw, int64_t rows, float *scores, hipStream_t s);

// ----------------------------------------------------------------- features
// Feature extraction (validation included) with every device buffer taken
// from `region` (`bytes` bytes of device memory the caller owns) and the
// results read back through pageable host memory: no allocation.
// features_region_bytes(m, n) is what an m x n matrix needs; a smaller
// region gives SPMV_EUNSUPPORTED.  Synchronises `s`.
size_t features_region_bytes(int64_t m, int64_t n);
spmv_status features_in_region(const spmv_csr *A, spmv_features *out, hipStream_t s,
                               void *region, size_t bytes);

// ----------------------------------------------------------------- misc
spmv_status run_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
size_t stream_read_out_bytes();
spmv_status run_stream_read(const void *src, size_t bytes, void *out, hipStream_t s);
int64_t gather_probe_threads();
spmv_status run_gather_probe(const void *table, const int32_t *idx, const void *val,
                             int64_t count, int elt, void *out, hipStream_t s);

}  // namespace smat
