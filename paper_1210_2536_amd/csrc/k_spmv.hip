// SpMV kernels for gfx950: one implementation family per storage format
// (paper Section 2.1 and Table 4), all computing
//     y_i = sum over stored entries of row i of a_ij x_j.
//
// Numerics: float64 data multiplies and accumulates in float64 with fused
// multiply-add; float32 data is widened to float64 (the product of two
// float32 numbers is exact there), accumulated in float64 and rounded once.
// Every kernel bounds its sequential summation chain (at most a few thousand
// additions per partial sum; long rows are split across lanes and
// workgroups), which keeps the float64 result within 1e-12 (|A||x|)_i.
//
// Results are deterministic: no floating-point atomics anywhere; partial
// sums that cross workgroups are combined by a second kernel in a fixed
// order.
#include "spmv_device.hpp"

#include <climits>

namespace smat {
namespace {

inline unsigned grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- CSR scalar
// One thread per row: the plain CSR kernel (the "naive" CSR SpMV that the
// paper's Introduction contrasts against tuned kernels).
template <typename T>
__global__ __launch_bounds__(1024) void k_csr_scalar(int64_t m, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const T *__restrict__ val,
                                                     const T *__restrict__ x, T *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    y[i] = (T)csr_row_seq<T>(i, rp, col, val, x);
}

// ---------------------------------------------------------------- CSR vector
// L lanes per row (L = 1..64, a sub-wavefront group); lanes stride the row so
// each trip of the group loads L consecutive entries; xor-shuffle reduction.
template <typename T, int L, bool NT>
__global__ __launch_bounds__(1024) void k_csr_vector(int64_t nrows,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const T *__restrict__ val,
                                                     const T *__restrict__ x, T *__restrict__ y) {
    int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t row = gt / L;
    int lane = threadIdx.x & (L - 1);
    if (row >= nrows) return;  // whole lane groups leave together
    double acc = csr_row_lanes<T, L, NT>(row, lane, rp, col, val, x);
    if (lane == 0) y[row] = (T)acc;
}

// ---------------------------------------------------------------- CSR adaptive
// Rows binned by length, all bins in one launch.  Workgroups are handed out
// longest bin first: launch position q serves bin 7 - q, where bin 7 gives a
// whole 256-thread workgroup to each row and bins 6..0 give 64..1 lanes.
// PK: the row pointers, columns and values are the plan's copy in binned
// row order (k_pack_binned), indexed by binned position, so that the rows
// of a bin read their entries from one contiguous range.
constexpr int kRowBlock = 512;     // split-row segments

template <typename T, bool NT, bool PK>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_adaptive(AdaptiveLaunch a,
                                                              const int32_t *__restrict__ rows,
                                                              const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ col,
                                                              const T *__restrict__ val,
                                                              const T *__restrict__ x,
                                                              T *__restrict__ y) {
    __shared__ double part[kAdaptBlock / kWave];
    adaptive_block<T, NT, PK>(a, blockIdx.x, rows, rp, col, val, x, y, part);
}

// The same launch without the longest bin, whose rows another kernel takes
// (the launch geometry has it empty); its own name keeps the two launch
// forms apart in kernel traces.  Likewise the *_rest panel kernels below.
template <typename T, bool NT, bool PK>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_adaptive_rest(
    AdaptiveLaunch a, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ y) {
    __shared__ double part[kAdaptBlock / kWave];
    adaptive_block<T, NT, PK>(a, blockIdx.x, rows, rp, col, val, x, y, part);
}

// The entries of the rows at binned positions [0, hi) copied in that order:
// brp (hi + 1 entries, filled by an exclusive scan of the row lengths) gives
// position pos's range in bcol / bval.  One wave per position, lanes
// striding the row; values are copied as bits.
template <typename U>
__global__ __launch_bounds__(256) void k_pack_binned(int64_t hi, const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const U *__restrict__ val,
                                                     const int32_t *__restrict__ brp,
                                                     int32_t *__restrict__ bcol,
                                                     U *__restrict__ bval) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int lane = threadIdx.x & 63;
    for (int64_t pos = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64; pos < hi;
         pos += waves) {
        const int32_t row = rows[pos];
        const int64_t b = rp[row], e = rp[row + 1], d = (int64_t)brp[pos] - b;
        for (int64_t q = b + lane; q < e; q += 64) {
            bcol[q + d] = col[q];
            bval[q + d] = val[q];
        }
    }
}

__global__ __launch_bounds__(256) void k_binned_lengths(int64_t hi, const int32_t *__restrict__ rows,
                                                        const int32_t *__restrict__ rp,
                                                        int32_t *__restrict__ len) {
    const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos < hi) len[pos] = rp[rows[pos] + 1] - rp[rows[pos]];
}

// ---------------------------------------------------------------- CSR panels
// Cache blocking of x for matrices whose columns are spread over an x too
// large for L2: the columns are cut into P panels whose slice of x fits in
// L2; one launch per panel adds that panel's part of every row to y (ACC
// after the first panel), so the random column gathers hit L2 instead of
// the next level.  Rows keep the length-binned order and lane widths of the
// adaptive kernel, scaled down by the panel count (lane_shift); prow holds,
// per panel and per binned position, the start of that row's segment.
//
// Where a row's panel sum goes (OUT): 0 stores y[row], 1 adds it to y[row]
// (panels after the first, one launch per panel), 2 stores it at the row's
// binned position of the panel's partial vector (all panels in one launch:
// consecutive lanes write consecutive words; the reduction scatters to y).
constexpr int kOutStore = 0, kOutAdd = 1, kOutPosition = 2;

template <typename T, int OUT>
__device__ __forceinline__ void panel_out(int64_t r, const int32_t *__restrict__ rows, double s,
                                          T *__restrict__ y) {
    if constexpr (OUT == kOutPosition) {
        y[r] = (T)s;
    } else {
        const int64_t row = rows[r];
        y[row] = OUT == kOutAdd ? (T)((double)y[row] + s) : (T)s;
    }
}

template <typename T, int L, bool NT, int OUT>
__device__ __forceinline__ void panel_lanes(unsigned local, unsigned rbeg, unsigned rend,
                                            const int32_t *__restrict__ rows,
                                            const int32_t *__restrict__ prow,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val, const T *__restrict__ x,
                                            T *__restrict__ y) {
    int64_t r = (int64_t)rbeg + (int64_t)local * (kAdaptBlock / L) + threadIdx.x / L;
    int lane = threadIdx.x & (L - 1);
    if (r < rend) {
        double acc = lanes_sum<T, L, NT>(prow[r], prow[r + 1], lane, col, val, x);
        if (lane == 0) panel_out<T, OUT>(r, rows, acc, y);
    }
}

// Work of workgroup `bid` of one panel's binned launch geometry.
template <typename T, bool NT, int OUT>
__device__ __forceinline__ void panel_block(const AdaptiveLaunch &a, unsigned bid,
                                            const int32_t *__restrict__ rows,
                                            const int32_t *__restrict__ prow,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val, const T *__restrict__ x,
                                            T *__restrict__ y, double *part) {
    int q = 0;
    while (q < 7 && bid >= a.first[q + 1]) ++q;
    const int b = 7 - q;
    const unsigned local = bid - a.first[q];
    const unsigned rb = a.row_begin[b], re = a.row_begin[b + 1];
    if (b == 7) {
        const unsigned r = rb + local;
        double s = block_sum<T, kAdaptBlock, NT>(prow[r], prow[r + 1], col, val, x, part);
        if (threadIdx.x == 0) panel_out<T, OUT>(r, rows, s, y);
        return;
    }
    int lb = b - a.lane_shift;
    lb = lb < 0 ? 0 : lb;
    switch (lb) {
    case 6: panel_lanes<T, 64, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    case 5: panel_lanes<T, 32, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    case 4: panel_lanes<T, 16, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    case 3: panel_lanes<T, 8, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    case 2: panel_lanes<T, 4, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    case 1: panel_lanes<T, 2, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    default: panel_lanes<T, 1, NT, OUT>(local, rb, re, rows, prow, col, val, x, y); break;
    }
}

// One panel per launch (panels processed one after another by the whole GPU).
template <typename T, bool NT, bool ACC>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_panel(AdaptiveLaunch a,
                                                           const int32_t *__restrict__ rows,
                                                           const int32_t *__restrict__ prow,
                                                           const int32_t *__restrict__ col,
                                                           const T *__restrict__ val,
                                                           const T *__restrict__ x,
                                                           T *__restrict__ y) {
    __shared__ double part[kAdaptBlock / kWave];
    panel_block<T, NT, ACC ? kOutAdd : kOutStore>(a, blockIdx.x, rows, prow, col, val, x, y, part);
}

template <typename T, bool NT, bool ACC>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_panel_rest(
    AdaptiveLaunch a, const int32_t *__restrict__ rows, const int32_t *__restrict__ prow,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ y) {
    __shared__ double part[kAdaptBlock / kWave];
    panel_block<T, NT, ACC ? kOutAdd : kOutStore>(a, blockIdx.x, rows, prow, col, val, x, y, part);
}

// All P = 8 G panels in one launch.  Workgroups are dispatched to the eight
// XCDs in turn, so workgroup w runs on XCD w mod 8; it serves panel
// (w mod 8) + 8 g, where g = w / (8 nblk) is the group of 8 panels the launch
// is working through (groups follow each other in dispatch order).  Every
// XCD thus works on one panel at a time and its L2 holds just that slice of
// x -- the eight L2s cache disjoint slices instead of copies of the same one.
// Each panel writes its own partial vector; k_panel_reduce adds them in
// panel order.
template <typename T, bool NT>
__device__ __forceinline__ void panel_xcd_block(const AdaptiveLaunch &a, int64_t m,
                                                const int32_t *__restrict__ rows,
                                                const int32_t *__restrict__ prow,
                                                const int32_t *__restrict__ col,
                                                const T *__restrict__ val, const T *__restrict__ x,
                                                T *__restrict__ partial, double *part) {
    const unsigned nblk = a.first[8];
    const unsigned w = blockIdx.x;
    const int panel = (int)(w % 8u + 8u * (w / (8u * nblk)));
    const unsigned bid = (w / 8u) % nblk;
    panel_block<T, NT, kOutPosition>(a, bid, rows, prow + (int64_t)panel * (m + 1), col, val, x,
                                     partial + (int64_t)panel * m, part);
}

template <typename T, bool NT>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_panel_xcd(AdaptiveLaunch a, int64_t m,
                                                               const int32_t *__restrict__ rows,
                                                               const int32_t *__restrict__ prow,
                                                               const int32_t *__restrict__ col,
                                                               const T *__restrict__ val,
                                                               const T *__restrict__ x,
                                                               T *__restrict__ partial) {
    __shared__ double part[kAdaptBlock / kWave];
    panel_xcd_block<T, NT>(a, m, rows, prow, col, val, x, partial, part);
}

template <typename T, bool NT>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_panel_xcd_rest(
    AdaptiveLaunch a, int64_t m, const int32_t *__restrict__ rows, const int32_t *__restrict__ prow,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ partial) {
    __shared__ double part[kAdaptBlock / kWave];
    panel_xcd_block<T, NT>(a, m, rows, prow, col, val, x, partial, part);
}

// y[rows[i]] = sum over panels, in panel order, of the partials at binned
// position i (every row has exactly one position).
template <typename T>
__global__ void k_panel_reduce(int P, int64_t m, const int32_t *__restrict__ rows,
                               const T *__restrict__ partial, T *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += (double)partial[(int64_t)p * m + i];
    y[rows[i]] = (T)s;
}

// The same for binned positions [lo, hi) only (the other rows are written by
// other kernels: the longest bin, the shortest bins).
template <typename T>
__global__ void k_panel_reduce_rest(int P, int64_t m, const int32_t *__restrict__ rows,
                                    const T *__restrict__ partial, T *__restrict__ y,
                                    int64_t lo, int64_t hi) {
    int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= hi) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += (double)partial[(int64_t)p * m + i];
    y[rows[i]] = (T)s;
}

// Rows longer than one workgroup may sum alone: segments of a row reduce to
// partials (one workgroup each), then one thread per row adds them in order.
template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_csr_segment(const int64_t *__restrict__ segs,
                                                           const int32_t *__restrict__ col,
                                                           const T *__restrict__ val,
                                                           const T *__restrict__ x,
                                                           double *__restrict__ partials) {
    __shared__ double part[kRowBlock / kWave];
    int64_t b = segs[3 * blockIdx.x + 1], e = segs[3 * blockIdx.x + 2];
    double acc = 0.0;
#pragma unroll 4
    for (int64_t p = b + threadIdx.x; p < e; p += kRowBlock)
        acc = fma((double)val[p], (double)x[col[p]], acc);
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kRowBlock / kWave; ++w) s += part[w];
        partials[blockIdx.x] = s;
    }
}

template <typename T>
__global__ void k_csr_segment_fixup(int64_t nrows, const int64_t *__restrict__ row_seg_begin,
                                    const int32_t *__restrict__ rows,
                                    const double *__restrict__ partials, T *__restrict__ y) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int64_t q = row_seg_begin[r]; q < row_seg_begin[r + 1]; ++q) s += partials[q];
    y[rows[r]] = (T)s;
}

// ---------------------------------------------------------------- ELL
// Slot-major layout: thread i reads slot k of row i at k*m_pad + i, so a
// wavefront reads 64 consecutive values and 64 consecutive columns per slot.
// U slots are loaded before any is used, to keep more loads in flight.
// Wide form (V > 1): a lane takes V consecutive rows, so each slot's columns
// and values arrive in one load of V elements.
template <typename T, int U, bool NT, int V>
__global__ __launch_bounds__(1024) void k_ell(int64_t m, int64_t m_pad, int K,
                                              const int32_t *__restrict__ ecol,
                                              const T *__restrict__ eval, const T *__restrict__ x,
                                              T *__restrict__ y) {
    if constexpr (V == 1) {
        int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
        if (i >= m) return;
        y[i] = (T)ell_row<T, U, NT>(i, m_pad, K, ecol, eval, x);
    } else {
        int64_t i0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * V;
        if (i0 >= m) return;
        double acc[V];
        ell_rows_wide<T, U, V, NT>(i0, m, m_pad, K, ecol, eval, x, acc);
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (i0 + e < m) y[i0 + e] = (T)acc[e];
    }
}

// ---------------------------------------------------------------- DIA
// A workgroup owns R = blockDim * RPT consecutive rows.  Diagonals are grouped
// into windows whose offsets span at most `max_span`; for each window the
// slice x[r0 + lo, r0 + R + hi) is staged once in LDS and every diagonal of
// the window reads its shifted view from there, while the diagonal values
// stream from HBM with unit stride.  Summation runs over diagonals in
// ascending offset order, i.e. ascending column order as in CSR.
template <typename T, int RPT, bool NT, int V>
__global__ __launch_bounds__(256) void k_dia_lds(int64_t m, int64_t n, int64_t m_pad,
                                                 const int32_t *__restrict__ offs, int nwin,
                                                 const DiaWindow *__restrict__ win,
                                                 const T *__restrict__ data,
                                                 const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x * RPT * V;
    dia_tile_lds<T, RPT, NT, V>(r0, m, n, m_pad, offs, nwin, win, data, x, y, xs);
}

// DIA without LDS: x comes through L1/L2 (neighbouring diagonals hit the same
// cache lines).
template <typename T, int RPT, bool NT, int V>
__global__ __launch_bounds__(256) void k_dia_direct(int64_t m, int64_t n, int64_t m_pad, int D,
                                                    const int32_t *__restrict__ offs,
                                                    const T *__restrict__ data,
                                                    const T *__restrict__ x, T *__restrict__ y) {
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x * RPT * V;
    dia_tile_direct<T, RPT, NT, V>(r0, m, n, m_pad, D, offs, data, x, y);
}

// ---------------------------------------------------------------- long rows, x in LDS
// float64 rows of the longest bin (a workgroup each in the binned kernels)
// in groups of G = 1024 / TPR per workgroup.  x streams through LDS in
// column chunks of kLongChunk values with two buffers: the next chunk
// travels through registers (16-byte loads) while the current one is used,
// one barrier per chunk.  Lane t of a row takes the row's entries t, t + TPR,
// t + 2 TPR, ... in that order; since a row's columns ascend, the entries of
// one chunk come before those of the next, so a lane stops at its first
// entry past the chunk and resumes there.  Lane sums stay in registers
// across chunks and are added by xor shuffles at the end.  Rows of TPR lanes
// keep a float64 chain of length/TPR + log2 TPR.
constexpr int kLongChunk = 8192;                 // float64 x values per chunk
constexpr int kLongThreads = 1024;
constexpr size_t kLongLds = 2u * kLongChunk * sizeof(double);

template <int TPR>
__global__ __launch_bounds__(kLongThreads) void k_long_rows_lds(
    int64_t nrows, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ x, int64_t n, double *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int PIECES = kLongChunk / 2;      // 16-byte pieces per chunk
    constexpr int PER = PIECES / kLongThreads;  // pieces per thread
    constexpr int U = 4;                        // entries requested ahead
    constexpr int G = kLongThreads / TPR;
    static_assert(PIECES % kLongThreads == 0, "chunk must split evenly");
    const int t = threadIdx.x % TPR;
    const int64_t ri = (int64_t)blockIdx.x * G + threadIdx.x / TPR;
    const bool active = ri < nrows;
    const int32_t row = active ? rows[ri] : 0;
    int64_t p = active ? (int64_t)rp[row] + t : 0;
    const int64_t e = active ? (int64_t)rp[row + 1] : 0;
    double acc = 0.0;
    const int64_t nchunks = (n + kLongChunk - 1) / kLongChunk;
    d2 stage[PER];
    // the lane's next U entries (col INT_MAX past the row's end)
    int32_t cc[U];
    double vv[U];
    auto window = [&]() {
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = p + u * TPR < e ? col[p + u * TPR] : INT_MAX;
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = p + u * TPR < e ? val[p + u * TPR] : 0.0;
    };
    auto fetch = [&](int64_t c) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int64_t j0 = c * kLongChunk + 2 * ((int64_t)q * kLongThreads + threadIdx.x);
            if (j0 + 2 <= n) {
                __builtin_memcpy(&stage[q], x + j0, sizeof(d2));
            } else {
                stage[q][0] = j0 < n ? x[j0] : 0.0;
                stage[q][1] = 0.0;
            }
        }
    };
    fetch(0);
    window();
    for (int64_t c = 0; c < nchunks; ++c) {
        d2 *buf = reinterpret_cast<d2 *>(smem) + (c & 1) * PIECES;
#pragma unroll
        for (int q = 0; q < PER; ++q) buf[q * kLongThreads + threadIdx.x] = stage[q];
        __syncthreads();
        if (c + 1 < nchunks) fetch(c + 1);
        const double *xs = reinterpret_cast<const double *>(buf);
        const int64_t c0 = c * kLongChunk;
        const int64_t cend = c0 + kLongChunk < n ? c0 + kLongChunk : n;
        // columns ascend, so the window's entries inside the chunk are a
        // prefix of it; the window is refilled after each pass, the last
        // refill of a chunk being the first window of the next (its loads
        // are in flight across the barrier)
        for (;;) {
            int k = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (cc[u] < cend) {
                    acc = fma(vv[u], xs[cc[u] - c0], acc);
                    ++k;
                }
            }
            p += (int64_t)k * TPR;
            window();
            if (k < U) break;
        }
    }
#pragma unroll
    for (int off = TPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, TPR);
    if (t == 0 && active) y[row] = acc;
}

// ---------------------------------------------------------------- long rows, x panels per workgroup
// The long rows (longest first) are cut into row blocks of about equal entry
// counts and x into panels of kTileBytes.  Workgroup (b, p) copies x panel p
// into LDS once, then adds for every row of block b the row's entries whose
// columns fall in the panel, the segment [seg[p][r], seg[p + 1][r]) of row r:
// lane t of the row's TPR lanes takes the segment's entries t, t + TPR, ...
// in order, TPR being set per block so that short and long segments both
// keep the lanes busy.  The lane sums are added by xor shuffles into one
// float64 partial per (row, panel), and k_long_tiles_reduce (or, in binned
// CSR, the first workgroups of k_csr_adaptive_tiles) adds a row's partials
// in panel order and rounds once.  A row's float64 chain is at most
// (longest segment) / TPR + log2 TPR + panels long.
//
// The entries come packed in workgroup order (row block, panel, row; see
// k_long_tile_pack), so a workgroup streams one contiguous range, and their
// columns as 16-bit offsets into the panel (col - p W): a panel holds at
// most 20480 values, and the entry stream shrinks from 4 + sizeof(T) to
// 2 + sizeof(T) bytes per entry.
constexpr int kTileThreads = 1024;
constexpr int kTileBytes = 81920;   // x per workgroup: two workgroups fill a CU's LDS
constexpr int kTileUnroll = 4;      // entries per lane loaded ahead
static_assert(kTileBytes / 4 <= 65536, "panel offsets must fit 16 bits");

//
// Dispatch order: panels fastest (workgroup w serves panel w mod P of row
// block w / P).  The workgroups in flight then cover a few row blocks across
// all panels: each row's entries are read front to back by neighbouring
// workgroups and the GPU streams a small part of the matrix at a time
// (measured 6% faster on the largest Zipf matrices than row blocks
// fastest; padding P to a multiple of 8, so that panel p always runs on XCD
// p mod 8, was 1-2% slower again).
template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_long_tiles(
    int64_t n7, int64_t W, int64_t P, const int32_t *__restrict__ blocks,
    const int32_t *__restrict__ pk, const uint16_t *__restrict__ off,
    const T *__restrict__ val, const T *__restrict__ x, int64_t n, double *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int V = 16 / (int)sizeof(T);      // values per 16-byte piece
    typedef T vec __attribute__((ext_vector_type(V)));
    constexpr int PIECES = kTileBytes / 16;
    constexpr int PER = PIECES / kTileThreads;
    static_assert(PIECES % kTileThreads == 0, "panel must split evenly");
    const int64_t p = (int64_t)blockIdx.x % P, b = (int64_t)blockIdx.x / P;
    const int64_t c0 = p * W;
    vec *xv = reinterpret_cast<vec *>(smem);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = q * kTileThreads + threadIdx.x;
        const int64_t j0 = c0 + (int64_t)k * V;
        vec w;
        if (j0 + V <= n) {
            __builtin_memcpy(&w, x + j0, sizeof(w));
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) w[e] = j0 + e < n ? x[j0 + e] : T(0);
        }
        xv[k] = w;
    }
    __syncthreads();
    const T *xs = reinterpret_cast<const T *>(smem);
    const int64_t r0 = blocks[3 * b], r1 = blocks[3 * b + 1];
    const int lg = blocks[3 * b + 2];
    const int tpr = 1 << lg;
    const int t = threadIdx.x & (tpr - 1);
    const int grp = threadIdx.x >> lg;
    const int G = kTileThreads >> lg;
    // row r's packed range in panel p: [sb[r], se[r])
    const int32_t *sb = pk + (P * r0 + p * (r1 - r0) - r0), *se = sb + 1;
    double *pp = part + p * n7;
    // every lane of a wave runs the same iterations (the shuffles need them);
    // the next group's segment bounds are loaded before the current group's
    // entries, so blocks of many short segments do not wait on them
    int64_t r = r0 + grp;
    bool act = r < r1;
    int64_t qb = act ? (int64_t)sb[r] : 0, qe = act ? (int64_t)se[r] : 0;
    for (int64_t base = r0; base < r1; base += G) {
        const int64_t rn = base + G + grp;
        const bool actn = rn < r1;
        const int64_t nb = actn ? (int64_t)sb[rn] : 0, ne = actn ? (int64_t)se[rn] : 0;
        const int64_t e = qe;
        int64_t q = qb + t;
        double acc = 0.0;
        // kTileUnroll entries per lane and trip, all loads issued before any
        // is used; the remainder in one more trip whose loads past the
        // segment's end are skipped and whose products there are left out
        // (the same additions, in the same order, as one entry at a time)
        for (; q + (kTileUnroll - 1) * tpr < e; q += kTileUnroll * tpr) {
            uint32_t cc[kTileUnroll];
            T vv[kTileUnroll];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) cc[u] = off[q + u * tpr];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) vv[u] = val[q + u * tpr];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u)
                acc = fma((double)vv[u], (double)xs[cc[u]], acc);
        }
        if (q < e) {
            const int k = (int)((e - q + tpr - 1) / tpr);   // 1 .. kTileUnroll - 1
            uint32_t cc[kTileUnroll - 1];
            T vv[kTileUnroll - 1];
#pragma unroll
            for (int u = 0; u < kTileUnroll - 1; ++u) cc[u] = u < k ? off[q + u * tpr] : 0u;
#pragma unroll
            for (int u = 0; u < kTileUnroll - 1; ++u) vv[u] = u < k ? val[q + u * tpr] : T(0);
#pragma unroll
            for (int u = 0; u < kTileUnroll - 1; ++u) {
                const double v = fma((double)vv[u], (double)xs[cc[u]], acc);
                acc = u < k ? v : acc;
            }
        }
        for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (t == 0 && act) pp[r] = acc;
        r = rn;
        act = actn;
        qb = nb;
        qe = ne;
    }
}

// A long row's result: its panel partials added in a fixed order, rounded
// once.  A workgroup takes 32 rows; thread (g, i) adds the partials of panels
// g, g + 8, g + 16, ... of row i in that order (32 neighbouring rows per
// load, four of a thread's loads issued before their additions), and the
// eight group sums are added in group order.  Workgroup `bid` of such a
// reduction; every thread of the 256 calls it.
constexpr int kReduceRows = 32, kReduceGroups = 8;

template <typename T>
__device__ __forceinline__ void tiles_reduce_block(unsigned bid, int64_t n7, int64_t P,
                                                   const int32_t *__restrict__ rows,
                                                   const double *__restrict__ part,
                                                   T *__restrict__ y,
                                                   double (*gs)[kReduceRows]) {
    const int i = threadIdx.x % kReduceRows, g = threadIdx.x / kReduceRows;
    const int64_t r = (int64_t)bid * kReduceRows + i;
    double acc = 0.0;
    if (r < n7) {
        constexpr int G = kReduceGroups;
        int64_t p = g;
        for (; p + 3 * G < P; p += 4 * G) {
            const double v0 = part[p * n7 + r], v1 = part[(p + G) * n7 + r];
            const double v2 = part[(p + 2 * G) * n7 + r], v3 = part[(p + 3 * G) * n7 + r];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; p < P; p += G) acc += part[p * n7 + r];
    }
    gs[g][i] = acc;
    __syncthreads();
    if (g == 0 && r < n7) {
        double s = gs[0][i];
#pragma unroll
        for (int k = 1; k < kReduceGroups; ++k) s += gs[k][i];
        y[rows[r]] = (T)s;
    }
}

template <typename T>
__global__ __launch_bounds__(kReduceRows * kReduceGroups) void k_long_tiles_reduce(
    int64_t n7, int64_t P, const int32_t *__restrict__ rows, const double *__restrict__ part,
    T *__restrict__ y) {
    __shared__ double gs[kReduceGroups][kReduceRows];
    tiles_reduce_block<T>(blockIdx.x, n7, P, rows, part, y, gs);
}

// The short rows of a binned-CSR plan whose long rows are in tiles, launched
// after k_long_tiles: workgroups [0, rg) add the long rows' panel partials
// (as k_long_tiles_reduce), the others are the binned launch of the short
// rows; the two write disjoint rows of y.  One launch fewer per SpMV, and
// the partials' loads overlap the short rows' work.
static_assert(kReduceRows * kReduceGroups == kAdaptBlock, "one workgroup size for both parts");

template <typename T, bool NT, bool PK>
__global__ __launch_bounds__(kAdaptBlock) void k_csr_adaptive_tiles(
    AdaptiveLaunch a, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ y, unsigned rg, int64_t n7, int64_t P, const int32_t *__restrict__ lrows,
    const double *__restrict__ part) {
    __shared__ double sp[kAdaptBlock / kWave];
    __shared__ double gs[kReduceGroups][kReduceRows];
    if (blockIdx.x < rg) {
        tiles_reduce_block<T>(blockIdx.x, n7, P, lrows, part, y, gs);
        return;
    }
    adaptive_block<T, NT, PK>(a, blockIdx.x - rg, rows, rp, col, val, x, y, sp);
}

// Segment starts of the long rows in the x panels: seg[p * n7 + r] is the
// first entry of row rows[r] whose column is at least p * W (for p = P, the
// row's end), found by binary search over the row's ascending columns.
__global__ __launch_bounds__(256) void k_long_tile_seg(int64_t n7, int64_t P, int64_t W,
                                                       const int32_t *__restrict__ rows,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       int32_t *__restrict__ seg) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n7 * (P + 1)) return;
    const int64_t p = i / n7, r = i - p * n7;
    const int32_t row = rows[r];
    int64_t lo = rp[row], hi = rp[row + 1];
    const int64_t c = p * W;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    seg[i] = (int32_t)lo;
}

// Packing of the long rows' entries for the tiles: entry e of row rows[r],
// in panel p = col / W, goes to pk[kb[2r] + p kb[2r+1]] + (e - seg[p n7 +
// r]) with its column as col - p W (16 bits) and its value's bits.
// Workgroups take rows in turn, threads the row's entries.
template <typename U>
__global__ __launch_bounds__(256) void k_long_tile_pack(
    int64_t n7, int32_t W, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const U *__restrict__ val, const int32_t *__restrict__ seg,
    const int32_t *__restrict__ kb, const int32_t *__restrict__ pk, uint16_t *__restrict__ off,
    U *__restrict__ pval) {
    for (int64_t r = blockIdx.x; r < n7; r += gridDim.x) {
        const int32_t row = rows[r];
        const int64_t k0 = kb[2 * r], ks = kb[2 * r + 1];
        const int64_t e1 = rp[row + 1];
        for (int64_t e = rp[row] + threadIdx.x; e < e1; e += blockDim.x) {
            const int32_t c = col[e];
            const int64_t p = c / W;
            const int64_t dst = (int64_t)pk[k0 + p * ks] + (e - seg[p * n7 + r]);
            off[dst] = (uint16_t)(c - p * W);
            pval[dst] = val[e];
        }
    }
}

// ---------------------------------------------------------------- BCSR 4x4
// Two lane mappings, chosen by value type (both measured on gfx950):
//
// float32 (k_bcsr): a group of L lanes per block row; lane l takes blocks l,
// l+L, ... of its block row.  A block's 16 values (row-major) arrive in
// 16-byte loads, its 4 x values in one (element-aligned) load away from the
// last column block; each lane keeps one running sum per row (products of a
// block in column order), and the L lanes' sums are added by xor shuffles.
//
// float64 (k_bcsr_coop): a block's 128 bytes are read by 8 lanes together,
// 16 bytes (half a row) each, so consecutive lanes read consecutive 16-byte
// pieces and a wave's loads are fully coalesced.  A block row has L lanes
// (8 <= L <= 64): G = L / 8 groups, group g taking blocks g, g + G, ... of
// the row.  A lane reads the 2 x values under its piece in one load and
// keeps one running sum for its row; lanes of the same row (the pair inside
// a block, then the G groups) are added by xor shuffles in a fixed order.
//
// Zero-filled positions add exact zeros.
template <typename T, int L, bool NT>
__global__ __launch_bounds__(256) void k_bcsr(int64_t mb, int64_t m, int64_t n,
                                              const int32_t *__restrict__ brp,
                                              const int32_t *__restrict__ bcol,
                                              const T *__restrict__ bval,
                                              const T *__restrict__ x, T *__restrict__ y) {
    const int64_t R = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L;
    bcsr_row_lanes<T, L, NT>(R, threadIdx.x & (L - 1), mb, m, n, brp, bcol, bval, x, y);
}

template <int L, bool NT>
__global__ __launch_bounds__(256) void k_bcsr_coop(int64_t mb, int64_t m, int64_t n,
                                                   const int32_t *__restrict__ brp,
                                                   const int32_t *__restrict__ bcol,
                                                   const double *__restrict__ bval,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y) {
    const int64_t R = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L;
    bcsr_row_coop<L, NT>(R, threadIdx.x & (L - 1), mb, m, n, brp, bcol, bval, x, y);
}

// ---------------------------------------------------------------- COO
// Each wavefront owns a chunk of E*64 consecutive entries (rows ascending).
// Per trip the 64 lanes form their products and run a segmented inclusive
// scan keyed by row index (6 shuffle steps); the lane ending a row segment
// writes the row.  The running sum of a row that continues past a trip is
// carried to the next trip; a row cut by a chunk boundary leaves a partial
// (head: row began in an earlier chunk; tail: row continues in a later one)
// that k_coo_fixup adds up in chunk order.  Rows with no entries are
// written as 0 by the lane that sees the gap.
template <typename T>
__device__ __forceinline__ void coo_emit(int row, double v, int first_row, bool first_partial,
                                         int last_row, bool last_continues, int64_t w,
                                         double *head, double *tail, T *y) {
    if (row == first_row && first_partial)
        head[w] = v;
    else if (row == last_row && last_continues)
        tail[w] = v;
    else
        y[row] = (T)v;
}

template <typename T, bool NT>
__global__ __launch_bounds__(256) void k_coo(int64_t m, int64_t nnz, int E,
                                             const int32_t *__restrict__ ri,
                                             const int32_t *__restrict__ col,
                                             const T *__restrict__ val, const T *__restrict__ x,
                                             T *__restrict__ y, double *__restrict__ head,
                                             double *__restrict__ tail,
                                             uint32_t *__restrict__ flags) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t chunk = (int64_t)E * kWave;
    const int64_t c0 = w * chunk;
    if (c0 >= nnz) return;  // whole wavefront
    const int64_t c1 = c0 + chunk < nnz ? c0 + chunk : nnz;
    const int first_row = ri[c0];
    const int last_row = ri[c1 - 1];
    const int prev_row = c0 > 0 ? ri[c0 - 1] : -1;
    const int next_row = c1 < nnz ? ri[c1] : INT_MAX;
    const bool first_partial = prev_row == first_row;
    const bool last_continues = next_row == last_row;
    // empty rows between the previous chunk's last row and this chunk's first
    for (int64_t r = (int64_t)prev_row + 1 + lane; r < first_row; r += kWave) y[r] = T(0);
    // empty rows after the matrix's last stored entry
    if (c1 == nnz)
        for (int64_t r = (int64_t)last_row + 1 + lane; r < m; r += kWave) y[r] = T(0);

    int carry_row = -1;
    double carry = 0.0;
    int before = first_row;  // row of the entry preceding lane 0 of this trip
    for (int64_t it = c0; it < c1; it += kWave) {
        const int64_t p = it + lane;
        const bool valid = p < c1;
        const int r = valid ? ld<NT>(ri + p) : INT_MAX;
        double v = valid ? fma((double)ld<NT>(val + p), (double)x[ld<NT>(col + p)], 0.0) : 0.0;
        // rows skipped between consecutive entries have no entries: zero them
        int rb = __shfl_up(r, 1, kWave);
        if (lane == 0) rb = before;
        if (valid && r > rb + 1)
            for (int rr = rb + 1; rr < r; ++rr) y[rr] = T(0);
        const int r_lane0 = __shfl(r, 0, kWave);
        if (carry_row >= 0) {
            if (carry_row == r_lane0) {
                if (lane == 0) v = carry + v;
            } else if (lane == 0) {
                coo_emit<T>(carry_row, carry, first_row, first_partial, last_row,
                            last_continues, w, head, tail, y);
            }
        }
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            double vu = __shfl_up(v, off, kWave);
            int ru = __shfl_up(r, off, kWave);
            if (lane >= off && ru == r) v += vu;
        }
        const int rn = __shfl_down(r, 1, kWave);
        if (valid && lane != kWave - 1 && rn != r)
            coo_emit<T>(r, v, first_row, first_partial, last_row, last_continues, w, head, tail,
                        y);
        const int r_last = __shfl(r, kWave - 1, kWave);
        const double v_last = __shfl(v, kWave - 1, kWave);
        if (r_last != INT_MAX) {
            carry_row = r_last;
            carry = v_last;
            before = r_last;
        } else {
            carry_row = -1;
        }
    }
    if (carry_row >= 0 && lane == 0)
        coo_emit<T>(carry_row, carry, first_row, first_partial, last_row, last_continues, w, head,
                    tail, y);
    if (lane == 0)
        flags[w] = (first_partial ? 1u : 0u) | (last_continues ? 2u : 0u) |
                   (first_row == last_row ? 4u : 0u);
}

// The chunk in which a row that crosses chunk boundaries starts ("owner")
// adds its tail partial and the head partials of the following chunks, in
// chunk order, and writes the row.
template <typename T>
__global__ void k_coo_fixup(int64_t nchunks, int64_t chunk, int64_t nnz,
                            const int32_t *__restrict__ ri, const double *__restrict__ head,
                            const double *__restrict__ tail, const uint32_t *__restrict__ flags,
                            T *__restrict__ y) {
    int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (w >= nchunks) return;
    uint32_t f = flags[w];
    if (!(f & 2u)) return;                  // last row ends inside this chunk
    if ((f & 1u) && (f & 4u)) return;       // a middle piece of an earlier row
    int64_t c1 = (w + 1) * chunk < nnz ? (w + 1) * chunk : nnz;
    int row = ri[c1 - 1];
    double s = tail[w];
    for (int64_t w2 = w + 1; w2 < nchunks; ++w2) {
        s += head[w2];
        uint32_t f2 = flags[w2];
        if (!((f2 & 2u) && (f2 & 4u))) break;
    }
    y[row] = (T)s;
}

template <typename T>
__global__ void k_fill_zero(int64_t m, T *y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) y[i] = T(0);
}

// ---------------------------------------------------------------- dispatch

template <typename T, bool NT>
spmv_status csr_vector_dispatch(int lanes, int64_t nrows, const int32_t *rp, const int32_t *col,
                                const T *val, const T *x, T *y, int block, hipStream_t s) {
    if (nrows == 0) return SPMV_OK;
    if (block <= 0) block = 256;
    block = block < lanes ? lanes : block;
    unsigned g = grid_for(nrows * lanes, block);
    switch (lanes) {
    case 1: k_csr_vector<T, 1, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 2: k_csr_vector<T, 2, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 4: k_csr_vector<T, 4, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 8: k_csr_vector<T, 8, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 16: k_csr_vector<T, 16, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 32: k_csr_vector<T, 32, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    case 64: k_csr_vector<T, 64, NT><<<g, block, 0, s>>>(nrows, rp, col, val, x, y); break;
    default:
        set_error("csr_vector: lanes must be a power of two in [1, 64], got %d", lanes);
        return SPMV_EINVAL;
    }
    SMAT_LAUNCHED("csr_vector");
    return SPMV_OK;
}

// Rows per lane of the wide forms: 16 bytes of values per load.
template <typename T> constexpr int kWideRows = 16 / (int)sizeof(T);

template <typename T, bool NT, int V>
void ell_launch(unsigned g, int block, int unroll, int64_t m, int64_t m_pad, int K,
                const int32_t *ecol, const T *eval, const T *x, T *y, hipStream_t s) {
    switch (unroll) {
    case 1: k_ell<T, 1, NT, V><<<g, block, 0, s>>>(m, m_pad, K, ecol, eval, x, y); break;
    case 2: k_ell<T, 2, NT, V><<<g, block, 0, s>>>(m, m_pad, K, ecol, eval, x, y); break;
    default: k_ell<T, 4, NT, V><<<g, block, 0, s>>>(m, m_pad, K, ecol, eval, x, y); break;
    }
}

template <typename T, bool NT>
spmv_status ell_dispatch(int64_t m, int64_t m_pad, int K, const int32_t *ecol, const T *eval,
                         const T *x, T *y, int block, int unroll, bool wide, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    if (block <= 0) block = 256;
    constexpr int W = kWideRows<T>;
    if (wide)
        ell_launch<T, NT, W>(grid_for((m + W - 1) / W, block), block, unroll, m, m_pad, K, ecol,
                             eval, x, y, s);
    else
        ell_launch<T, NT, 1>(grid_for(m, block), block, unroll, m, m_pad, K, ecol, eval, x, y, s);
    SMAT_LAUNCHED("ell");
    return SPMV_OK;
}

template <typename T, bool NT, int V>
void dia_launch(bool lds, unsigned g, int block, int rpt, size_t sh, int64_t m, int64_t n,
                int64_t m_pad, int D, const int32_t *offs, int nwin, const DiaWindow *win,
                const T *data, const T *x, T *y, hipStream_t s) {
    if (lds) {
        switch (rpt) {
        case 1: k_dia_lds<T, 1, NT, V><<<g, block, sh, s>>>(m, n, m_pad, offs, nwin, win, data, x, y); break;
        case 2: k_dia_lds<T, 2, NT, V><<<g, block, sh, s>>>(m, n, m_pad, offs, nwin, win, data, x, y); break;
        case 4: k_dia_lds<T, 4, NT, V><<<g, block, sh, s>>>(m, n, m_pad, offs, nwin, win, data, x, y); break;
        default: k_dia_lds<T, 8, NT, V><<<g, block, sh, s>>>(m, n, m_pad, offs, nwin, win, data, x, y); break;
        }
    } else {
        switch (rpt) {
        case 1: k_dia_direct<T, 1, NT, V><<<g, block, 0, s>>>(m, n, m_pad, D, offs, data, x, y); break;
        case 2: k_dia_direct<T, 2, NT, V><<<g, block, 0, s>>>(m, n, m_pad, D, offs, data, x, y); break;
        case 4: k_dia_direct<T, 4, NT, V><<<g, block, 0, s>>>(m, n, m_pad, D, offs, data, x, y); break;
        default: k_dia_direct<T, 8, NT, V><<<g, block, 0, s>>>(m, n, m_pad, D, offs, data, x, y); break;
        }
    }
}

template <typename T, bool NT>
spmv_status dia_dispatch(bool lds, int64_t m, int64_t n, int64_t m_pad, int D,
                         const int32_t *offs, int nwin, const DiaWindow *win, int max_span,
                         const T *data, const T *x, T *y, int block, int rpt, bool wide,
                         hipStream_t s) {
    if (m == 0) return SPMV_OK;
    if (block <= 0 || block > 256) block = 256;
    if (rpt != 1 && rpt != 2 && rpt != 4 && rpt != 8) rpt = 4;
    constexpr int W = kWideRows<T>;
    const int V = wide ? W : 1;
    int64_t tile = (int64_t)block * rpt * V;
    unsigned g = grid_for(m, (int)tile);
    size_t sh = lds ? (size_t)(tile + max_span) * sizeof(T) : 0;
    if (wide)
        dia_launch<T, NT, W>(lds, g, block, rpt, sh, m, n, m_pad, D, offs, nwin, win, data, x, y, s);
    else
        dia_launch<T, NT, 1>(lds, g, block, rpt, sh, m, n, m_pad, D, offs, nwin, win, data, x, y, s);
    SMAT_LAUNCHED(lds ? "dia_lds" : "dia_direct");
    return SPMV_OK;
}

template <typename T, bool NT>
spmv_status coo_dispatch(int64_t m, int64_t nnz, const int32_t *ri, const int32_t *col,
                         const T *val, const T *x, T *y, int chunk, double *head, double *tail,
                         uint32_t *flags, hipStream_t s) {
    int64_t per = (int64_t)chunk * kWave;
    int64_t nchunks = (nnz + per - 1) / per;
    unsigned g = grid_for(nchunks * kWave, 256);
    k_coo<T, NT><<<g, 256, 0, s>>>(m, nnz, chunk, ri, col, val, x, y, head, tail, flags);
    SMAT_LAUNCHED("coo");
    k_coo_fixup<T><<<grid_for(nchunks, 256), 256, 0, s>>>(nchunks, per, nnz, ri, head, tail,
                                                          flags, y);
    SMAT_LAUNCHED("coo_fixup");
    return SPMV_OK;
}

template <typename T, bool NT, bool PK>
void adaptive_launch(bool rest, unsigned nblk, const AdaptiveLaunch &a, const int32_t *rows,
                     const int32_t *rp, const int32_t *col, const T *val, const T *x, T *y,
                     hipStream_t s) {
    if (rest)
        k_csr_adaptive_rest<T, NT, PK><<<nblk, kAdaptBlock, 0, s>>>(a, rows, rp, col, val, x, y);
    else
        k_csr_adaptive<T, NT, PK><<<nblk, kAdaptBlock, 0, s>>>(a, rows, rp, col, val, x, y);
}

template <typename T>
spmv_status adaptive_dispatch(bool nt, bool rest, bool pk, const AdaptiveLaunch &a,
                              const int32_t *rows, const int32_t *rp, const int32_t *col,
                              const T *val, const T *x, T *y, hipStream_t s) {
    const unsigned nblk = a.first[8];
    if (nblk == 0) return SPMV_OK;
    if (nt && pk)
        adaptive_launch<T, true, true>(rest, nblk, a, rows, rp, col, val, x, y, s);
    else if (nt)
        adaptive_launch<T, true, false>(rest, nblk, a, rows, rp, col, val, x, y, s);
    else if (pk)
        adaptive_launch<T, false, true>(rest, nblk, a, rows, rp, col, val, x, y, s);
    else
        adaptive_launch<T, false, false>(rest, nblk, a, rows, rp, col, val, x, y, s);
    SMAT_LAUNCHED("csr_adaptive");
    return SPMV_OK;
}

template <typename T, bool NT>
spmv_status panel_dispatch(const AdaptiveLaunch &a, const int32_t *rows, int P, int64_t m,
                           const int32_t *prow, const int32_t *pcol, const T *pval, const T *x,
                           T *y, T *partial, int64_t red_lo, int64_t red_hi, bool rest,
                           hipStream_t s) {
    const unsigned nblk = a.first[8];
    if (nblk == 0 && red_hi <= red_lo) return SPMV_OK;
    if (partial) {
        if (nblk) {
            if (rest)
                k_csr_panel_xcd_rest<T, NT><<<nblk * (unsigned)P, kAdaptBlock, 0, s>>>(
                    a, m, rows, prow, pcol, pval, x, partial);
            else
                k_csr_panel_xcd<T, NT><<<nblk * (unsigned)P, kAdaptBlock, 0, s>>>(
                    a, m, rows, prow, pcol, pval, x, partial);
            SMAT_LAUNCHED("csr_panel_xcd");
        }
        if (rest) {
            if (red_hi > red_lo)
                k_panel_reduce_rest<T><<<grid_for(red_hi - red_lo, 256), 256, 0, s>>>(
                    P, m, rows, partial, y, red_lo, red_hi);
        } else {
            k_panel_reduce<T><<<grid_for(m, 256), 256, 0, s>>>(P, m, rows, partial, y);
        }
        SMAT_LAUNCHED("panel_reduce");
        return SPMV_OK;
    }
    if (nblk == 0) return SPMV_OK;
    for (int p = 0; p < P; ++p) {
        const int32_t *pr = prow + (int64_t)p * (m + 1);
        if (rest) {
            if (p == 0)
                k_csr_panel_rest<T, NT, false><<<nblk, kAdaptBlock, 0, s>>>(a, rows, pr, pcol,
                                                                             pval, x, y);
            else
                k_csr_panel_rest<T, NT, true><<<nblk, kAdaptBlock, 0, s>>>(a, rows, pr, pcol, pval,
                                                                            x, y);
        } else if (p == 0) {
            k_csr_panel<T, NT, false><<<nblk, kAdaptBlock, 0, s>>>(a, rows, pr, pcol, pval, x, y);
        } else {
            k_csr_panel<T, NT, true><<<nblk, kAdaptBlock, 0, s>>>(a, rows, pr, pcol, pval, x, y);
        }
        SMAT_LAUNCHED("csr_panel");
    }
    return SPMV_OK;
}

template <typename T, bool NT>
spmv_status bcsr_dispatch(int64_t m, int64_t n, const int32_t *brp, const int32_t *bcol,
                          const T *bval, const T *x, T *y, int lanes, int block, hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb == 0) return SPMV_OK;
    if (block <= 0 || block > 256) block = 256;
    if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)) || lanes > block) {
        set_error("bcsr: lanes must be a power of two in [1, min(64, block)], got %d", lanes);
        return SPMV_EINVAL;
    }
    if constexpr (sizeof(T) == 8) {
        if (lanes < 8) lanes = 8;  // a float64 block takes 8 lanes
        if (lanes > block) {
            set_error("bcsr: block of %d threads cannot hold %d lanes per block row", block,
                      lanes);
            return SPMV_EINVAL;
        }
        const unsigned g = grid_for(mb, block / lanes);
#define L_CASE(L)                                                                          \
    case L: k_bcsr_coop<L, NT><<<g, block, 0, s>>>(mb, m, n, brp, bcol, bval, x, y); break;
        switch (lanes) { L_CASE(8) L_CASE(16) L_CASE(32) L_CASE(64) }
#undef L_CASE
    } else {
        const unsigned g = grid_for(mb, block / lanes);
#define L_CASE(L)                                                                            \
    case L: k_bcsr<T, L, NT><<<g, block, 0, s>>>(mb, m, n, brp, bcol, bval, x, y); break;
        switch (lanes) {
            L_CASE(1) L_CASE(2) L_CASE(4) L_CASE(8) L_CASE(16) L_CASE(32) L_CASE(64)
        }
#undef L_CASE
    }
    SMAT_LAUNCHED("bcsr");
    return SPMV_OK;
}

}  // namespace

spmv_status run_bcsr(int elt, bool nt, int64_t m, int64_t n, const int32_t *brp,
                     const int32_t *bcol, const void *bval, const void *x, void *y, int lanes,
                     int block, hipStream_t s) {
#define CALL(T, NT)                                                                         \
    bcsr_dispatch<T, NT>(m, n, brp, bcol, (const T *)bval, (const T *)x, (T *)y, lanes, block, s)
    return elt == 8 ? (nt ? CALL(double, true) : CALL(double, false))
                    : (nt ? CALL(float, true) : CALL(float, false));
#undef CALL
}

spmv_status run_csr_panels(int elt, bool nt, const AdaptiveLaunch &a, const int32_t *rows, int P,
                           int64_t m, const int32_t *prow, const int32_t *pcol, const void *pval,
                           const void *x, void *y, void *partial, int64_t red_lo,
                           int64_t red_hi, bool part, hipStream_t s) {
    if (elt == 8)
        return nt ? panel_dispatch<double, true>(a, rows, P, m, prow, pcol, (const double *)pval,
                                                 (const double *)x, (double *)y,
                                                 (double *)partial, red_lo, red_hi, part, s)
                  : panel_dispatch<double, false>(a, rows, P, m, prow, pcol, (const double *)pval,
                                                  (const double *)x, (double *)y,
                                                  (double *)partial, red_lo, red_hi, part, s);
    return nt ? panel_dispatch<float, true>(a, rows, P, m, prow, pcol, (const float *)pval,
                                            (const float *)x, (float *)y, (float *)partial,
                                            red_lo, red_hi, part, s)
              : panel_dispatch<float, false>(a, rows, P, m, prow, pcol, (const float *)pval,
                                             (const float *)x, (float *)y, (float *)partial,
                                             red_lo, red_hi, part, s);
}

// Typed entry points: elt selects float (4) or double (8), nt the streaming
// cache policy.
#define SMAT_TYPED(elt, nt, CALL)                                                      \
    ((elt) == 8 ? ((nt) ? CALL(double, true) : CALL(double, false))                    \
                : ((nt) ? CALL(float, true) : CALL(float, false)))

spmv_status run_csr_scalar(int elt, int64_t m, const int32_t *rp, const int32_t *col,
                           const void *val, const void *x, void *y, int block, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    if (block <= 0) block = 256;
    unsigned g = grid_for(m, block);
    if (elt == 8)
        k_csr_scalar<double><<<g, block, 0, s>>>(m, rp, col, (const double *)val,
                                                 (const double *)x, (double *)y);
    else
        k_csr_scalar<float><<<g, block, 0, s>>>(m, rp, col, (const float *)val,
                                                (const float *)x, (float *)y);
    SMAT_LAUNCHED("csr_scalar");
    return SPMV_OK;
}

spmv_status run_csr_vector(int elt, bool nt, int lanes, int64_t nrows, const int32_t *rp,
                           const int32_t *col, const void *val, const void *x, void *y, int block,
                           hipStream_t s) {
#define CALL(T, NT)                                                                          \
    csr_vector_dispatch<T, NT>(lanes, nrows, rp, col, (const T *)val, (const T *)x, (T *)y, \
                               block, s)
    return SMAT_TYPED(elt, nt, CALL);
#undef CALL
}

spmv_status run_csr_adaptive(int elt, bool nt, bool rest, const AdaptiveLaunch &a,
                             const int32_t *rows, const int32_t *rp, const int32_t *col,
                             const void *val, const void *x, void *y, hipStream_t s, bool pk) {
    if (elt == 8)
        return adaptive_dispatch<double>(nt, rest, pk, a, rows, rp, col, (const double *)val,
                                         (const double *)x, (double *)y, s);
    return adaptive_dispatch<float>(nt, rest, pk, a, rows, rp, col, (const float *)val,
                                    (const float *)x, (float *)y, s);
}

spmv_status launch_binned_scan(int64_t hi, const int32_t *rows, const int32_t *rp, int32_t *len,
                               unsigned *scan, int32_t *brp, hipStream_t s) {
    if (hi <= 0) {
        SMAT_HIP(hipMemsetAsync(brp, 0, sizeof(int32_t), s));
        return SPMV_OK;
    }
    k_binned_lengths<<<(unsigned)((hi + 255) / 256), 256, 0, s>>>(hi, rows, rp, len);
    SMAT_LAUNCHED("binned_lengths");
    return launch_exclusive_scan_rows(hi, len, brp, scan, s);
}

spmv_status launch_pack_binned(int64_t hi, const int32_t *rows, const int32_t *rp,
                               const int32_t *col, const void *val, int elt, const int32_t *brp,
                               int32_t *bcol, void *bval, hipStream_t s) {
    if (hi <= 0) return SPMV_OK;
    const unsigned grid = (unsigned)std::min<int64_t>((hi + 3) / 4, 65536);
    if (elt == 8)
        k_pack_binned<uint64_t><<<grid, 256, 0, s>>>(hi, rows, rp, col, (const uint64_t *)val, brp,
                                                     bcol, (uint64_t *)bval);
    else
        k_pack_binned<uint32_t><<<grid, 256, 0, s>>>(hi, rows, rp, col, (const uint32_t *)val, brp,
                                                     bcol, (uint32_t *)bval);
    SMAT_LAUNCHED("pack_binned");
    return SPMV_OK;
}

spmv_status long_rows_lds_prepare() {
    // the kernels use more than the default 64 KB of dynamic LDS
    SMAT_HIP(hipFuncSetAttribute((const void *)k_long_rows_lds<32>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLongLds));
    SMAT_HIP(hipFuncSetAttribute((const void *)k_long_rows_lds<64>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLongLds));
    return SPMV_OK;
}

spmv_status run_long_rows_lds(int tpr, int64_t nrows, const int32_t *rows, const int32_t *rp,
                              const int32_t *col, const double *val, const double *x, int64_t n,
                              double *y, hipStream_t s) {
    if (nrows == 0) return SPMV_OK;
    if (tpr != 32 && tpr != 64) {
        set_error("long rows: %d lanes per row (32 or 64)", tpr);
        return SPMV_EINVAL;
    }
    const int64_t G = kLongThreads / tpr;
    const unsigned g = (unsigned)((nrows + G - 1) / G);
    if (tpr == 32)
        k_long_rows_lds<32><<<g, kLongThreads, kLongLds, s>>>(nrows, rows, rp, col, val, x, n, y);
    else
        k_long_rows_lds<64><<<g, kLongThreads, kLongLds, s>>>(nrows, rows, rp, col, val, x, n, y);
    SMAT_LAUNCHED("long_rows_lds");
    return SPMV_OK;
}

int64_t long_tile_width(int elt) { return kTileBytes / elt; }

spmv_status long_tiles_prepare() {
    // the tile kernels use more than the default 64 KB of dynamic LDS
    SMAT_HIP(hipFuncSetAttribute((const void *)k_long_tiles<double>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kTileBytes));
    SMAT_HIP(hipFuncSetAttribute((const void *)k_long_tiles<float>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kTileBytes));
    return SPMV_OK;
}

spmv_status launch_long_tile_seg(int64_t n7, int64_t P, int64_t W, const int32_t *rows,
                                 const int32_t *rp, const int32_t *col, int32_t *seg,
                                 hipStream_t s) {
    const int64_t count = n7 * (P + 1);
    if (count == 0) return SPMV_OK;
    k_long_tile_seg<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(n7, P, W, rows, rp, col, seg);
    SMAT_LAUNCHED("long_tile_seg");
    return SPMV_OK;
}

spmv_status launch_long_tile_pack(int64_t n7, int64_t P, int64_t W, const int32_t *rows,
                                  const int32_t *rp, const int32_t *col, const void *val, int elt,
                                  const int32_t *seg, const int32_t *kb, const int32_t *pk,
                                  uint16_t *off, void *pval, hipStream_t s) {
    if (n7 == 0) return SPMV_OK;
    if (W < 1 || W > 65536 || P < 1 || (elt != 4 && elt != 8)) {
        set_error("long-row tiles: panel width %lld beyond 16-bit offsets", (long long)W);
        return SPMV_EINVAL;
    }
    const unsigned grid = (unsigned)std::min<int64_t>(n7, 4096);
    if (elt == 8)
        k_long_tile_pack<uint64_t><<<grid, 256, 0, s>>>(n7, (int32_t)W, rows, rp, col,
                                                        (const uint64_t *)val, seg, kb, pk, off,
                                                        (uint64_t *)pval);
    else
        k_long_tile_pack<uint32_t><<<grid, 256, 0, s>>>(n7, (int32_t)W, rows, rp, col,
                                                        (const uint32_t *)val, seg, kb, pk, off,
                                                        (uint32_t *)pval);
    SMAT_LAUNCHED("long_tile_pack");
    return SPMV_OK;
}

spmv_status run_long_tiles(int elt, int64_t n7, int64_t P, int64_t nblocks,
                           const int32_t *blocks, const int32_t *pk, const int32_t *rows,
                           const uint16_t *off, const void *val, const void *x, int64_t n,
                           double *part, void *y, hipStream_t s, bool reduce) {
    if (n7 == 0) return SPMV_OK;
    if (P < 1 || P > 65535 || nblocks < 1 || nblocks > INT_MAX || (elt != 4 && elt != 8)) {
        set_error("long-row tiles: %lld panels, %lld row blocks", (long long)P,
                  (long long)nblocks);
        return SPMV_EINVAL;
    }
    const int64_t W = kTileBytes / elt;
    if (P * nblocks > INT_MAX) {
        set_error("long-row tiles: %lld workgroups", (long long)(P * nblocks));
        return SPMV_EINVAL;
    }
    const unsigned grid = (unsigned)(P * nblocks);
    const unsigned rg = (unsigned)((n7 + kReduceRows - 1) / kReduceRows);
    if (elt == 8)
        k_long_tiles<double><<<grid, kTileThreads, kTileBytes, s>>>(
            n7, W, P, blocks, pk, off, (const double *)val, (const double *)x, n, part);
    else
        k_long_tiles<float><<<grid, kTileThreads, kTileBytes, s>>>(
            n7, W, P, blocks, pk, off, (const float *)val, (const float *)x, n, part);
    SMAT_LAUNCHED("long_tiles");
    if (!reduce) return SPMV_OK;
    if (elt == 8)
        k_long_tiles_reduce<double><<<rg, kReduceRows * kReduceGroups, 0, s>>>(n7, P, rows, part,
                                                                              (double *)y);
    else
        k_long_tiles_reduce<float><<<rg, kReduceRows * kReduceGroups, 0, s>>>(n7, P, rows, part,
                                                                             (float *)y);
    SMAT_LAUNCHED("long_tiles_reduce");
    return SPMV_OK;
}

template <typename T>
spmv_status adaptive_tiles_dispatch(bool nt, const AdaptiveLaunch &a, const int32_t *rows,
                                    const int32_t *rp, const int32_t *col, const T *val,
                                    const T *x, T *y, int64_t n7, int64_t P,
                                    const int32_t *lrows, const double *part, hipStream_t s) {
    const unsigned rg = (unsigned)((n7 + kReduceRows - 1) / kReduceRows);
    const unsigned grid = rg + a.first[8];
    if (grid == 0) return SPMV_OK;
    if (nt)
        k_csr_adaptive_tiles<T, true, true><<<grid, kAdaptBlock, 0, s>>>(a, rows, rp, col, val, x,
                                                                         y, rg, n7, P, lrows, part);
    else
        k_csr_adaptive_tiles<T, false, true><<<grid, kAdaptBlock, 0, s>>>(
            a, rows, rp, col, val, x, y, rg, n7, P, lrows, part);
    SMAT_LAUNCHED("csr_adaptive_tiles");
    return SPMV_OK;
}

spmv_status run_csr_adaptive_tiles(int elt, bool nt, const AdaptiveLaunch &a, const int32_t *rows,
                                   const int32_t *rp, const int32_t *col, const void *val,
                                   const void *x, void *y, int64_t n7, int64_t P,
                                   const int32_t *lrows, const double *part, hipStream_t s) {
    if (elt == 8)
        return adaptive_tiles_dispatch<double>(nt, a, rows, rp, col, (const double *)val,
                                               (const double *)x, (double *)y, n7, P, lrows, part,
                                               s);
    return adaptive_tiles_dispatch<float>(nt, a, rows, rp, col, (const float *)val,
                                          (const float *)x, (float *)y, n7, P, lrows, part, s);
}

spmv_status run_csr_split(int elt, int64_t nseg, const int64_t *segs, double *partials,
                          int64_t nrows, const int64_t *row_seg_begin, const int32_t *rows,
                          const int32_t *col, const void *val, const void *x, void *y,
                          hipStream_t s) {
    if (nrows == 0) return SPMV_OK;
    if (elt == 8) {
        k_csr_segment<double><<<(unsigned)nseg, kRowBlock, 0, s>>>(
            segs, col, (const double *)val, (const double *)x, partials);
        SMAT_LAUNCHED("csr_segment");
        k_csr_segment_fixup<double><<<grid_for(nrows, 64), 64, 0, s>>>(
            nrows, row_seg_begin, rows, partials, (double *)y);
    } else {
        k_csr_segment<float><<<(unsigned)nseg, kRowBlock, 0, s>>>(
            segs, col, (const float *)val, (const float *)x, partials);
        SMAT_LAUNCHED("csr_segment");
        k_csr_segment_fixup<float><<<grid_for(nrows, 64), 64, 0, s>>>(
            nrows, row_seg_begin, rows, partials, (float *)y);
    }
    SMAT_LAUNCHED("csr_segment_fixup");
    return SPMV_OK;
}

spmv_status run_ell(int elt, bool nt, int64_t m, int64_t m_pad, int K, const int32_t *ecol,
                    const void *eval, const void *x, void *y, int block, int unroll, bool wide,
                    hipStream_t s) {
#define CALL(T, NT)                                                                             \
    ell_dispatch<T, NT>(m, m_pad, K, ecol, (const T *)eval, (const T *)x, (T *)y, block, unroll, \
                        wide, s)
    return SMAT_TYPED(elt, nt, CALL);
#undef CALL
}

spmv_status run_dia(int elt, bool nt, bool lds, int64_t m, int64_t n, int64_t m_pad, int D,
                    const int32_t *offs_dev, int nwin, const DiaWindow *win_dev, int max_span,
                    const void *data, const void *x, void *y, int block, int rows_per_thread,
                    bool wide, hipStream_t s) {
    if (D == 0) return run_fill_zero(elt, m, y, s);
#define CALL(T, NT)                                                                      \
    dia_dispatch<T, NT>(lds, m, n, m_pad, D, offs_dev, nwin, win_dev, max_span,          \
                        (const T *)data, (const T *)x, (T *)y, block, rows_per_thread, wide, s)
    return SMAT_TYPED(elt, nt, CALL);
#undef CALL
}

spmv_status run_coo(int elt, bool nt, int64_t m, int64_t nnz, const int32_t *row_idx,
                    const int32_t *col, const void *val, const void *x, void *y, int chunk,
                    double *head, double *tail, uint32_t *flags, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    if (nnz == 0) return run_fill_zero(elt, m, y, s);
#define CALL(T, NT)                                                                         \
    coo_dispatch<T, NT>(m, nnz, row_idx, col, (const T *)val, (const T *)x, (T *)y, chunk, \
                        head, tail, flags, s)
    return SMAT_TYPED(elt, nt, CALL);
#undef CALL
}

spmv_status run_fill_zero(int elt, int64_t m, void *y, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    if (elt == 8)
        k_fill_zero<double><<<grid_for(m, 256), 256, 0, s>>>(m, (double *)y);
    else
        k_fill_zero<float><<<grid_for(m, 256), 256, 0, s>>>(m, (float *)y);
    SMAT_LAUNCHED("fill_zero");
    return SPMV_OK;
}

}  // namespace smat
