// K0 CSR validation and K1 feature extraction (paper Section 3: CSR input;
// Section 4, Table 3: the feature parameters; Section 6: staged extraction).
//
// Entry-parallel passes give every thread a short contiguous run of
// nonzeros; the thread finds the row of its first entry by binary search on
// row_ptr and then walks forward, so work is balanced over nnz whatever the
// row-length distribution (the same nnz-balanced split the paper uses for its
// threads, Section 6).
#include "internal.hpp"

#include <climits>

namespace smat {
namespace {

constexpr int kEntryRun = 8;      // nonzeros per thread in entry passes
constexpr int kBlock = 256;
constexpr int kHash = 1024;       // LDS hash slots for the diagonal census
constexpr int kRowHistLds = 1024; // row-length bins kept in LDS

__device__ __forceinline__ int64_t row_of_entry(const int32_t *__restrict__ rp, int64_t m,
                                                int64_t p) {
    // largest i in [0, m) with rp[i] <= p; with a valid row_ptr this is the
    // row that holds entry p (empty rows have rp[i] == rp[i+1] and lose).
    int64_t lo = 0, hi = m - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void k_validate_rows(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                uint32_t *flags) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > m) return;
    uint32_t bad = 0;
    int32_t v = rp[i];
    if (i == 0 && v != 0) bad |= kBadRowPtr0;
    if (i == m && (int64_t)v != nnz) bad |= kBadRowPtrEnd;
    if (i < m && rp[i + 1] < v) bad |= kBadRowPtrOrder;
    if (v < 0 || (int64_t)v > nnz) bad |= kBadRowPtrOrder;
    if (bad) atomicOr(flags, bad);
}

// Column checks, and the bandwidth max |j - i| on the way (meaningful once
// the checks pass).  It runs beside the row_ptr check, so it must stay in
// bounds whatever row_ptr holds: rows are only looked up in rp[0..m] (m >= 1
// whenever nnz > 0) and columns only read below nnz; a row_ptr that ends a
// row past the last one is flagged as out of order.
__global__ void k_validate_entries(int64_t m, int64_t n, int64_t nnz,
                                   const int32_t *__restrict__ rp,
                                   const int32_t *__restrict__ col, uint32_t *flags,
                                   int *bandwidth) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t p0 = t * kEntryRun;
    uint32_t bad = 0;
    int bw = 0;
    if (p0 < nnz) {
        int64_t p1 = p0 + kEntryRun < nnz ? p0 + kEntryRun : nnz;
        int64_t row = row_of_entry(rp, m, p0);
        int64_t rend = rp[row + 1];
        for (int64_t p = p0; p < p1; ++p) {
            while (p >= rend && row + 1 < m) rend = rp[++row + 1];
            if (p >= rend) {   // entries beyond rp[m]: a broken row_ptr
                bad |= kBadRowPtrOrder;
                break;
            }
            int32_t c = col[p];
            if (c < 0 || (int64_t)c >= n) bad |= kBadColRange;
            if (p + 1 < rend && p + 1 < nnz && col[p + 1] <= c) bad |= kBadColOrder;
            int64_t d = (int64_t)c - row;
            int ad = (int)(d < 0 ? -d : d);
            bw = ad > bw ? ad : bw;
        }
    }
    if (bad) atomicOr(flags, bad);
    // every lane of the wave is here: reduce across it, one atomic per wave
    for (int off = kWave / 2; off > 0; off >>= 1) {
        int o = __shfl_xor(bw, off, kWave);
        bw = o > bw ? o : bw;
    }
    if (threadIdx.x % kWave == 0 && bw > 0) atomicMax(bandwidth, bw);
}

template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T *lds, T identity) {
    // wave reduction by xor shuffles, then across the waves of the block
    for (int off = kWave / 2; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, kWave));
    int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    int nw = blockDim.x / kWave;
    if (w == 0) {
        v = lane < nw ? lds[lane] : identity;
        for (int off = kWave / 2; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, kWave));
    }
    __syncthreads();
    return v;  // valid in thread 0
}

struct OpAdd { template <typename T> __device__ T operator()(T a, T b) const { return a + b; } };
struct OpMax { template <typename T> __device__ T operator()(T a, T b) const { return a > b ? a : b; } };
struct OpMin { template <typename T> __device__ T operator()(T a, T b) const { return a < b ? a : b; } };

__global__ void k_row_stats(int64_t m, const int32_t *__restrict__ rp, RowStats *out) {
    __shared__ unsigned long long lds_u[kBlock / kWave];
    __shared__ int lds_i[kBlock / kWave];
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0, mn = INT_MAX;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long k = (unsigned long long)(rp[i + 1] - rp[i]);
        s1 += k;
        s2 += k * k;
        mx = (int)k > mx ? (int)k : mx;
        mn = (int)k < mn ? (int)k : mn;
    }
    s1 = block_reduce(s1, OpAdd(), lds_u, 0ull);
    s2 = block_reduce(s2, OpAdd(), lds_u, 0ull);
    mx = block_reduce(mx, OpMax(), lds_i, 0);
    mn = block_reduce(mn, OpMin(), lds_i, INT_MAX);
    if (threadIdx.x == 0) {
        atomicAdd(&out->sum_rd, s1);
        atomicAdd(&out->sum_rd2, s2);
        atomicMax(&out->max_rd, mx);
        atomicMin(&out->min_rd, mn);
    }
}

__global__ void k_row_hist(int64_t m, const int32_t *__restrict__ rp, int max_rd,
                           unsigned int *hist) {
    __shared__ unsigned int h[kRowHistLds];
    int nl = max_rd + 1 < kRowHistLds ? max_rd + 1 : kRowHistLds;
    for (int b = threadIdx.x; b < nl; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int k = rp[i + 1] - rp[i];
        if (k < kRowHistLds)
            atomicAdd(&h[k], 1u);
        else
            atomicAdd(&hist[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nl; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Least-squares fit of ln(count_k / m) on ln k over k >= 1 with count_k > 0
// (Section 4, parameter R).  One workgroup, fixed summation order, centred
// second pass.  sums = {count, mean_x, mean_y, sxy, sxx}.
__global__ void k_powerlaw_fit(const unsigned int *__restrict__ hist, int max_rd, int64_t m,
                               double *sums) {
    __shared__ double lds[1024 / kWave];
    double c = 0, sx = 0, sy = 0;
    double dm = (double)m;
    for (int k = 1 + threadIdx.x; k <= max_rd; k += blockDim.x) {
        unsigned int h = hist[k];
        if (h) {
            c += 1.0;
            sx += log((double)k);
            sy += log((double)h / dm);
        }
    }
    c = block_reduce(c, OpAdd(), lds, 0.0);
    sx = block_reduce(sx, OpAdd(), lds, 0.0);
    sy = block_reduce(sy, OpAdd(), lds, 0.0);
    __shared__ double mean[3];
    if (threadIdx.x == 0) {
        mean[0] = c;
        mean[1] = c > 0 ? sx / c : 0.0;
        mean[2] = c > 0 ? sy / c : 0.0;
    }
    __syncthreads();
    double xb = mean[1], yb = mean[2];
    double sxy = 0, sxx = 0;
    for (int k = 1 + threadIdx.x; k <= max_rd; k += blockDim.x) {
        unsigned int h = hist[k];
        if (h) {
            double dx = log((double)k) - xb;
            double dy = log((double)h / dm) - yb;
            sxy += dx * dy;
            sxx += dx * dx;
        }
    }
    sxy = block_reduce(sxy, OpAdd(), lds, 0.0);
    sxx = block_reduce(sxx, OpAdd(), lds, 0.0);
    if (threadIdx.x == 0) {
        sums[0] = mean[0];
        sums[1] = xb;
        sums[2] = yb;
        sums[3] = sxy;
        sums[4] = sxx;
    }
}

// Does row r (sorted columns [rp[r], rp[r+1])) hold a column in [lo, lo+3]?
__device__ __forceinline__ bool row_has_block(const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ col, int64_t r,
                                              int32_t lo) {
    int64_t a = rp[r], b = rp[r + 1];
    while (a < b) {  // first entry >= lo
        int64_t mid = (a + b) >> 1;
        if (col[mid] < lo)
            a = mid + 1;
        else
            b = mid;
    }
    return a < rp[r + 1] && col[a] <= lo + 3;
}

// BLOCKS: count the nonempty aligned 4x4 blocks (a few binary searches per
// block start); with a histogram, take the diagonal census.  Either or both.
//
// A census launched together with the CSR checks (gate, gate_rs non-NULL)
// runs only when both checks passed (gate[0] | gate[1] == 0) and the
// zero-fill bound still allows DIA (max_RD M <= 20 NNZ); the checks and the
// row pass precede it on the stream.  Every thread reads the same words, so
// a workgroup leaves as a whole.
template <bool BLOCKS>
__global__ void k_entry_stats(int64_t m, int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                              const int32_t *__restrict__ col, EntryStats *out,
                              unsigned int *diag_hist, const uint32_t *gate,
                              const RowStats *gate_rs) {
    if (gate && (gate[0] | gate[1])) return;
    if (gate_rs && (int64_t)gate_rs->max_rd * m > 20 * nnz) return;
    __shared__ int hkey[kHash];
    __shared__ unsigned int hcnt[kHash];
    __shared__ unsigned long long lds_u[kBlock / kWave];
    const bool census = diag_hist != nullptr;
    if (census) {
        for (int b = threadIdx.x; b < kHash; b += blockDim.x) {
            hkey[b] = INT_MIN;
            hcnt[b] = 0;
        }
        __syncthreads();
    }
    unsigned long long nb = 0;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t p0 = t * kEntryRun;
    if (p0 < nnz) {
        int64_t p1 = p0 + kEntryRun < nnz ? p0 + kEntryRun : nnz;
        int64_t row = row_of_entry(rp, m, p0);
        int64_t rbeg = rp[row], rend = rp[row + 1];
        for (int64_t p = p0; p < p1; ++p) {
            while (p >= rend) {
                ++row;
                rbeg = rend;
                rend = rp[row + 1];
            }
            int32_t c = col[p];
            int64_t d = (int64_t)c - row;
            if (BLOCKS) {  // first entry of its aligned 4x4 block, in row-major order?
                int32_t lo = c & ~3;
                bool fresh = !(p > rbeg && (col[p - 1] & ~3) == lo);
                for (int64_t r2 = row & ~(int64_t)3; fresh && r2 < row; ++r2)
                    if (row_has_block(rp, col, r2, lo)) fresh = false;
                nb += fresh;
            }
            if (census) {
                int key = (int)d;
                unsigned int hsh = ((unsigned int)key * 2654435761u) >> 22;  // 10 bits
                bool done = false;
                for (int probe = 0; probe < 8 && !done; ++probe) {
                    int slot = (hsh + probe) & (kHash - 1);
                    int prev = atomicCAS(&hkey[slot], INT_MIN, key);
                    if (prev == INT_MIN || prev == key) {
                        atomicAdd(&hcnt[slot], 1u);
                        done = true;
                    }
                }
                if (!done) atomicAdd(&diag_hist[d + m - 1], 1u);
            }
        }
    }
    if (BLOCKS) {
        nb = block_reduce(nb, OpAdd(), lds_u, 0ull);
        if (threadIdx.x == 0) atomicAdd(&out->blocks4, nb);
    }
    if (census) {
        __syncthreads();
        for (int b = threadIdx.x; b < kHash; b += blockDim.x)
            if (hcnt[b]) atomicAdd(&diag_hist[(int64_t)hkey[b] + m - 1], hcnt[b]);
    }
}

// Occupied diagonals and "true" diagonals (5 count > 3 length).
__global__ void k_diag_stats(int64_t m, int64_t n, const unsigned int *__restrict__ hist,
                             DiagStats *out) {
    __shared__ unsigned long long lds[kBlock / kWave];
    unsigned long long nd = 0, nt = 0;
    int64_t nb = m + n - 1;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        unsigned int c = hist[b];
        if (c) {
            int64_t d = b - (m - 1);
            int64_t len = (m < n - d ? m : n - d) - (d < 0 ? -d : 0);
            nd += 1;
            nt += 5ull * c > 3ull * (unsigned long long)len;
        }
    }
    nd = block_reduce(nd, OpAdd(), lds, 0ull);
    nt = block_reduce(nt, OpAdd(), lds, 0ull);
    if (threadIdx.x == 0) {
        atomicAdd(&out->ndiags, nd);
        atomicAdd(&out->ntrue, nt);
    }
}

constexpr int kCompactPer = 16;   // bins per thread in the compaction

__global__ void k_diag_count_blocks(int64_t nbins, const unsigned int *__restrict__ hist,
                                    unsigned int *block_counts) {
    __shared__ unsigned int lds[kBlock / kWave];
    int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kCompactPer;
    unsigned int c = 0;
    for (int q = 0; q < kCompactPer; ++q)
        if (base + q < nbins && hist[base + q]) ++c;
    c = block_reduce(c, OpAdd(), lds, 0u);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = c;
}

// Exclusive scan of `count` values in place by one workgroup of 1024 threads.
__global__ void k_scan_single(unsigned int *v, int64_t count) {
    __shared__ unsigned int part[1024];
    __shared__ unsigned int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < count; base += 1024) {
        int64_t i = base + threadIdx.x;
        unsigned int x = i < count ? v[i] : 0;
        part[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            unsigned int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        unsigned int incl = part[threadIdx.x];
        if (i < count) v[i] = carry + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += incl;
        __syncthreads();
    }
}

// Write ascending offsets and turn each occupied histogram bin into its slot.
__global__ void k_diag_write(int64_t m, int64_t nbins, unsigned int *hist,
                             const unsigned int *__restrict__ block_base, int32_t *offsets) {
    __shared__ unsigned int part[kBlock];
    int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kCompactPer;
    unsigned int c = 0;
    for (int q = 0; q < kCompactPer; ++q)
        if (base + q < nbins && hist[base + q]) ++c;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        unsigned int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned int slot = block_base[blockIdx.x] + part[threadIdx.x] - c;
    for (int q = 0; q < kCompactPer; ++q) {
        int64_t b = base + q;
        if (b < nbins && hist[b]) {
            offsets[slot] = (int32_t)(b - (m - 1));
            hist[b] = slot;
            ++slot;
        }
    }
}

inline unsigned int grid_for(int64_t work, int block, int64_t cap = 1 << 20) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned int)g;
}

}  // namespace

spmv_status launch_validate_rows(int64_t m, int64_t nnz, const int32_t *rp, uint32_t *flags,
                                 hipStream_t s) {
    k_validate_rows<<<grid_for(m + 1, kBlock, INT_MAX), kBlock, 0, s>>>(m, nnz, rp, flags);
    SMAT_LAUNCHED("validate_rows");
    return SPMV_OK;
}

spmv_status launch_validate_entries(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                                    const int32_t *col, uint32_t *flags, int *bandwidth,
                                    hipStream_t s) {
    if (nnz == 0) return SPMV_OK;
    int64_t threads = (nnz + kEntryRun - 1) / kEntryRun;
    k_validate_entries<<<grid_for(threads, kBlock, INT_MAX), kBlock, 0, s>>>(m, n, nnz, rp, col,
                                                                            flags, bandwidth);
    SMAT_LAUNCHED("validate_entries");
    return SPMV_OK;
}

spmv_status launch_row_stats(int64_t m, const int32_t *rp, RowStats *out, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    k_row_stats<<<grid_for(m, kBlock, 4096), kBlock, 0, s>>>(m, rp, out);
    SMAT_LAUNCHED("row_stats");
    return SPMV_OK;
}

spmv_status launch_row_hist(int64_t m, const int32_t *rp, int max_rd, unsigned int *hist,
                            hipStream_t s) {
    if (m == 0) return SPMV_OK;
    k_row_hist<<<grid_for(m, kBlock, 2048), kBlock, 0, s>>>(m, rp, max_rd, hist);
    SMAT_LAUNCHED("row_hist");
    return SPMV_OK;
}

spmv_status launch_powerlaw_fit(const unsigned int *hist, int max_rd, int64_t m, double *sums,
                                hipStream_t s) {
    k_powerlaw_fit<<<1, 1024, 0, s>>>(hist, max_rd, m, sums);
    SMAT_LAUNCHED("powerlaw_fit");
    return SPMV_OK;
}

spmv_status launch_entry_stats(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                               const int32_t *col, EntryStats *out, unsigned int *diag_hist,
                               bool blocks, hipStream_t s, const uint32_t *gate,
                               const RowStats *gate_rs) {
    if (nnz == 0) return SPMV_OK;
    int64_t threads = (nnz + kEntryRun - 1) / kEntryRun;
    const unsigned g = grid_for(threads, kBlock, INT_MAX);
    if (blocks)
        k_entry_stats<true><<<g, kBlock, 0, s>>>(m, n, nnz, rp, col, out, diag_hist, gate,
                                                 gate_rs);
    else
        k_entry_stats<false><<<g, kBlock, 0, s>>>(m, n, nnz, rp, col, out, diag_hist, gate,
                                                  gate_rs);
    SMAT_LAUNCHED("entry_stats");
    return SPMV_OK;
}

spmv_status launch_diag_stats(int64_t m, int64_t n, const unsigned int *diag_hist, DiagStats *out,
                              hipStream_t s) {
    k_diag_stats<<<grid_for(m + n - 1, kBlock, 4096), kBlock, 0, s>>>(m, n, diag_hist, out);
    SMAT_LAUNCHED("diag_stats");
    return SPMV_OK;
}

spmv_status launch_diag_compact(int64_t m, int64_t n, unsigned int *diag_hist, int32_t *offsets,
                                unsigned int *block_scratch, hipStream_t s) {
    int64_t nbins = m + n - 1;
    int64_t per_block = (int64_t)kBlock * kCompactPer;
    int64_t nblk = (nbins + per_block - 1) / per_block;
    k_diag_count_blocks<<<(unsigned)nblk, kBlock, 0, s>>>(nbins, diag_hist, block_scratch);
    SMAT_LAUNCHED("diag_count_blocks");
    k_scan_single<<<1, 1024, 0, s>>>(block_scratch, nblk);
    SMAT_LAUNCHED("scan_single");
    k_diag_write<<<(unsigned)nblk, kBlock, 0, s>>>(m, nbins, diag_hist, block_scratch, offsets);
    SMAT_LAUNCHED("diag_write");
    return SPMV_OK;
}

// Shared with the conversion file: exclusive scan of per-row counts into a
// row_ptr of m+1 entries.
namespace {
__global__ void k_block_sums(int64_t m, const int32_t *__restrict__ counts, unsigned int *bsum) {
    __shared__ unsigned int lds[kBlock / kWave];
    int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kCompactPer;
    unsigned int c = 0;
    for (int q = 0; q < kCompactPer; ++q)
        if (base + q < m) c += (unsigned int)counts[base + q];
    c = block_reduce(c, OpAdd(), lds, 0u);
    if (threadIdx.x == 0) bsum[blockIdx.x] = c;
}

__global__ void k_scan_write(int64_t m, const int32_t *__restrict__ counts,
                             const unsigned int *__restrict__ bbase, int32_t *rp) {
    __shared__ unsigned int part[kBlock];
    int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kCompactPer;
    unsigned int c = 0;
    for (int q = 0; q < kCompactPer; ++q)
        if (base + q < m) c += (unsigned int)counts[base + q];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        unsigned int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned int run = bbase[blockIdx.x] + part[threadIdx.x] - c;
    for (int q = 0; q < kCompactPer; ++q) {
        int64_t i = base + q;
        if (i < m) {
            rp[i] = (int32_t)run;
            run += (unsigned int)counts[i];
        }
        if (i == m - 1) rp[m] = (int32_t)run;
    }
}
}  // namespace

spmv_status launch_exclusive_scan_rows(int64_t m, const int32_t *counts, int32_t *rp,
                                       unsigned int *scratch, hipStream_t s) {
    if (m == 0) {
        SMAT_HIP(hipMemsetAsync(rp, 0, sizeof(int32_t), s));
        return SPMV_OK;
    }
    int64_t per_block = (int64_t)kBlock * kCompactPer;
    int64_t nblk = (m + per_block - 1) / per_block;
    k_block_sums<<<(unsigned)nblk, kBlock, 0, s>>>(m, counts, scratch);
    SMAT_LAUNCHED("block_sums");
    k_scan_single<<<1, 1024, 0, s>>>(scratch, nblk);
    SMAT_LAUNCHED("scan_single");
    k_scan_write<<<(unsigned)nblk, kBlock, 0, s>>>(m, counts, scratch, rp);
    SMAT_LAUNCHED("scan_write");
    return SPMV_OK;
}

}  // namespace smat
