// K2 format conversions (paper Section 2.1: the four basic formats; Table 4
// and Section 4: ELL and DIA pay for zero fill) and K5 row binning for the
// length-adaptive CSR kernel.
//
// Layouts (Figure 1 did not survive; standard definitions):
//   COO  row index per stored entry, CSR order; columns and values are the
//        CSR arrays themselves.
//   ELL  K = max_RD slots per row, slot k of row i at k*m_pad + i (slot-major,
//        coalesced across rows); empty slots hold col -1 and value +0.0.
//   DIA  occupied diagonals d = j - i ascending; entry (i, i+off) at
//        slot*m_pad + i; absent slots hold +0.0; a presence bitmap (bit s of
//        uint32 word s >> 5) keeps explicit zeros distinguishable.
// Values are copied as raw bit patterns (uint32 / uint64), never through
// floating-point registers, so conversions are bit exact.
#include "internal.hpp"

namespace smat {
namespace {

constexpr int kBlock = 256;
constexpr int kEntryRun = 8;

__device__ __forceinline__ int64_t row_of_entry(const int32_t *__restrict__ rp, int64_t m,
                                                int64_t p) {
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

inline unsigned grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

__global__ void k_csr_to_coo(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                             int32_t *__restrict__ row_idx) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t p0 = t * kEntryRun;
    if (p0 >= nnz) return;
    int64_t p1 = p0 + kEntryRun < nnz ? p0 + kEntryRun : nnz;
    int64_t row = row_of_entry(rp, m, p0);
    int64_t rend = rp[row + 1];
    for (int64_t p = p0; p < p1; ++p) {
        while (p >= rend) rend = rp[++row + 1];
        row_idx[p] = (int32_t)row;
    }
}

template <typename U>
__global__ void k_csr_to_ell(int64_t m, int64_t m_pad, int K, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ col, const U *__restrict__ val,
                             int32_t *__restrict__ ecol, U *__restrict__ eval) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m_pad) return;
    int64_t b = 0, len = 0;
    if (i < m) {
        b = rp[i];
        len = rp[i + 1] - b;
    }
    for (int k = 0; k < K; ++k) {
        int64_t s = (int64_t)k * m_pad + i;
        if (k < len) {
            ecol[s] = col[b + k];
            eval[s] = val[b + k];
        } else {
            ecol[s] = -1;
            eval[s] = 0;
        }
    }
}

template <typename U>
__global__ void k_csr_to_dia(int64_t m, int64_t m_pad, int64_t nnz, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ col, const U *__restrict__ val,
                             const unsigned int *__restrict__ slot_map, U *__restrict__ data,
                             uint32_t *present) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t p0 = t * kEntryRun;
    if (p0 >= nnz) return;
    int64_t p1 = p0 + kEntryRun < nnz ? p0 + kEntryRun : nnz;
    int64_t row = row_of_entry(rp, m, p0);
    int64_t rend = rp[row + 1];
    for (int64_t p = p0; p < p1; ++p) {
        while (p >= rend) rend = rp[++row + 1];
        int64_t d = (int64_t)col[p] - row;
        int64_t slot = slot_map[d + m - 1];
        int64_t s = slot * m_pad + row;
        data[s] = val[p];
        atomicOr(&present[s >> 5], 1u << (s & 31));
    }
}

__global__ void k_coo_to_csr(int64_t m, int64_t nnz, const int32_t *__restrict__ row_idx,
                             int32_t *__restrict__ rp) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > m) return;
    int64_t a = 0, b = nnz;  // first entry with row_idx >= i
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (row_idx[mid] < i)
            a = mid + 1;
        else
            b = mid;
    }
    rp[i] = (int32_t)a;
}

__global__ void k_ell_count(int64_t m, int64_t m_pad, int K, const int32_t *__restrict__ ecol,
                            int32_t *__restrict__ counts) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int c = 0;
    for (int k = 0; k < K; ++k) c += ecol[(int64_t)k * m_pad + i] >= 0;
    counts[i] = c;
}

template <typename U>
__global__ void k_ell_gather(int64_t m, int64_t m_pad, int K, const int32_t *__restrict__ ecol,
                             const U *__restrict__ eval, const int32_t *__restrict__ rp,
                             int32_t *__restrict__ col, U *__restrict__ val) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t o = rp[i];
    for (int k = 0; k < K; ++k) {
        int64_t s = (int64_t)k * m_pad + i;
        int32_t c = ecol[s];
        if (c >= 0) {
            col[o] = c;
            val[o] = eval[s];
            ++o;
        }
    }
}

__device__ __forceinline__ bool bit_at(const uint32_t *__restrict__ w, int64_t s) {
    return (w[s >> 5] >> (s & 31)) & 1u;
}

__global__ void k_dia_count(int64_t m, int64_t m_pad, int D, const uint32_t *__restrict__ present,
                            int32_t *__restrict__ counts) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int c = 0;
    for (int d = 0; d < D; ++d) c += bit_at(present, (int64_t)d * m_pad + i);
    counts[i] = c;
}

template <typename U>
__global__ void k_dia_gather(int64_t m, int64_t m_pad, int D, const int32_t *__restrict__ offs,
                             const U *__restrict__ data, const uint32_t *__restrict__ present,
                             const int32_t *__restrict__ rp, int32_t *__restrict__ col,
                             U *__restrict__ val) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t o = rp[i];
    for (int d = 0; d < D; ++d) {
        int64_t s = (int64_t)d * m_pad + i;
        if (bit_at(present, s)) {
            col[o] = (int32_t)(i + offs[d]);
            val[o] = data[s];
            ++o;
        }
    }
}

// ---- column panels (cache blocking of x)
// first index in [b, e) whose column is >= v (columns sorted within a row)
__device__ __forceinline__ int32_t col_lower_bound(const int32_t *__restrict__ col, int32_t b,
                                                   int32_t e, int64_t v) {
    while (b < e) {
        int32_t mid = b + ((e - b) >> 1);
        if ((int64_t)col[mid] < v)
            b = mid + 1;
        else
            e = mid;
    }
    return b;
}

__global__ void k_inverse_perm(int64_t m, const int32_t *__restrict__ rows,
                               int32_t *__restrict__ inv) {
    int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos < m) inv[rows[pos]] = (int32_t)pos;
}

// cnt[p*(m+1) + pos] = entries of row rows[pos] in panel p; position m is a
// zero pad so one exclusive scan over the whole array yields every panel's
// segment starts and, at position m, the panel's end.
__global__ void k_panel_count(int64_t m, const int32_t *__restrict__ rp,
                              const int32_t *__restrict__ col, const int32_t *__restrict__ rows,
                              int P, int64_t w, int32_t *__restrict__ cnt) {
    int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos > m) return;
    if (pos == m) {
        for (int p = 0; p < P; ++p) cnt[(int64_t)p * (m + 1) + m] = 0;
        return;
    }
    int64_t row = rows[pos];
    int32_t b = rp[row], e = rp[row + 1];
    int32_t prev = b;
    for (int p = 0; p < P; ++p) {
        int32_t next = p == P - 1 ? e : col_lower_bound(col, prev, e, (int64_t)(p + 1) * w);
        cnt[(int64_t)p * (m + 1) + pos] = next - prev;
        prev = next;
    }
}

template <typename U>
__global__ void k_panel_scatter(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ col, const U *__restrict__ val,
                                const int32_t *__restrict__ inv, int64_t w,
                                const int32_t *__restrict__ prow, int32_t *__restrict__ pcol,
                                U *__restrict__ pval) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t p0 = t * kEntryRun;
    if (p0 >= nnz) return;
    int64_t p1 = p0 + kEntryRun < nnz ? p0 + kEntryRun : nnz;
    int64_t row = row_of_entry(rp, m, p0);
    int64_t rend = rp[row + 1];
    for (int64_t p = p0; p < p1; ++p) {
        while (p >= rend) rend = rp[++row + 1];
        int32_t c = col[p];
        int64_t panel = c / w;
        int32_t seg = col_lower_bound(col, rp[row], (int32_t)rend, panel * w);
        int64_t dst = prow[panel * (m + 1) + inv[row]] + (p - seg);
        pcol[dst] = c;
        pval[dst] = val[p];
    }
}

__global__ void k_panel_rowcount(int64_t m, const int32_t *__restrict__ rows, int P,
                                 const int32_t *__restrict__ prow, int32_t *__restrict__ counts) {
    int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos >= m) return;
    int32_t tot = 0;
    for (int p = 0; p < P; ++p) {
        const int32_t *pr = prow + (int64_t)p * (m + 1);
        tot += pr[pos + 1] - pr[pos];
    }
    counts[rows[pos]] = tot;
}

template <typename U>
__global__ void k_panel_gather(int64_t m, const int32_t *__restrict__ rows, int P,
                               const int32_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                               const U *__restrict__ pval, const int32_t *__restrict__ rp,
                               int32_t *__restrict__ col, U *__restrict__ val) {
    int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos >= m) return;
    int64_t o = rp[rows[pos]];
    for (int p = 0; p < P; ++p) {
        const int32_t *pr = prow + (int64_t)p * (m + 1);
        for (int32_t j = pr[pos]; j < pr[pos + 1]; ++j) {
            col[o] = pcol[j];
            val[o] = pval[j];
            ++o;
        }
    }
}

// ---- row binning: bin b holds rows with upper[b-1] < len <= upper[b]
__device__ __forceinline__ int bin_of(int len, const BinSpec &spec) {
    int b = 0;
    while (b < kAdaptiveBins - 1 && len > spec.upper[b]) ++b;
    return b;
}

__global__ void k_bin_count(int64_t m, const int32_t *__restrict__ rp, BinSpec spec,
                            unsigned int *__restrict__ block_counts) {
    __shared__ unsigned int cnt[kAdaptiveBins];
    if (threadIdx.x < kAdaptiveBins) cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) atomicAdd(&cnt[bin_of(rp[i + 1] - rp[i], spec)], 1u);
    __syncthreads();
    // bin-major layout so each bin's blocks are contiguous for the scan
    if (threadIdx.x < kAdaptiveBins)
        block_counts[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan over the bin-major block counts, one workgroup; also the
// per-bin start offsets (bin_offsets[b], b <= kAdaptiveBins).
__global__ void k_bin_scan(unsigned int *v, int64_t nblk, unsigned int *bin_offsets) {
    __shared__ unsigned int part[1024];
    __shared__ unsigned int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    int64_t count = nblk * kAdaptiveBins;
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
        if (i < count) {
            v[i] = carry + incl - x;
            if (i % nblk == 0) bin_offsets[i / nblk] = carry + incl - x;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) bin_offsets[kAdaptiveBins] = carry;
}

// Stable scatter: rows keep ascending order inside each bin.
__global__ void k_bin_scatter(int64_t m, const int32_t *__restrict__ rp, BinSpec spec,
                              const unsigned int *__restrict__ block_base,
                              int32_t *__restrict__ rows_out) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ unsigned int wave_cnt[kWaves][kAdaptiveBins];
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int b = i < m ? bin_of(rp[i + 1] - rp[i], spec) : -1;
    unsigned long long below = lane ? (~0ull >> (kWave - lane)) : 0ull;
    unsigned int rank = 0;
    for (int q = 0; q < kAdaptiveBins; ++q) {
        unsigned long long mask = __ballot(b == q);
        if (b == q) rank = __popcll(mask & below);
        if (lane == 0) wave_cnt[w][q] = __popcll(mask);
    }
    __syncthreads();
    if (b >= 0) {
        unsigned int pos = block_base[(int64_t)b * gridDim.x + blockIdx.x] + rank;
        for (int w2 = 0; w2 < w; ++w2) pos += wave_cnt[w2][b];
        rows_out[pos] = (int32_t)i;
    }
}

// ---------------------------------------------------------------- BCSR 4x4
// One thread per block row R (rows 4R..4R+3): the distinct column blocks
// col >> 2 of those rows, ascending, by a 4-way merge of the sorted rows.
__device__ __forceinline__ void bcsr_rows(int64_t R, int64_t m, const int32_t *__restrict__ rp,
                                          int32_t (&p)[4], int32_t (&e)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int64_t r = 4 * R + k;
        p[k] = r < m ? rp[r] : 0;
        e[k] = r < m ? rp[r + 1] : 0;
    }
}

__device__ __forceinline__ int32_t bcsr_next_block(const int32_t (&p)[4], const int32_t (&e)[4],
                                                   const int32_t *__restrict__ col) {
    int32_t c = INT32_MAX;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (p[k] < e[k]) c = min(c, col[p[k]] >> 2);
    return c;
}

__global__ void k_bcsr_count(int64_t mb, int64_t m, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ col, int32_t *__restrict__ counts) {
    int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= mb) return;
    int32_t p[4], e[4];
    bcsr_rows(R, m, rp, p, e);
    int32_t cnt = 0;
    for (int32_t c = bcsr_next_block(p, e, col); c != INT32_MAX; c = bcsr_next_block(p, e, col)) {
        ++cnt;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            while (p[k] < e[k] && (col[p[k]] >> 2) == c) ++p[k];
    }
    counts[R] = cnt;
}

// Values are moved as bit patterns (U = uint32 / uint64); bval must be
// zero-filled beforehand.  pres holds 16 presence bits per block.
template <typename U>
__global__ void k_bcsr_fill(int64_t mb, int64_t m, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ col, const U *__restrict__ val,
                            const int32_t *__restrict__ brp, int32_t *__restrict__ bcol,
                            U *__restrict__ bval, uint16_t *__restrict__ pres) {
    int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= mb) return;
    int32_t p[4], e[4];
    bcsr_rows(R, m, rp, p, e);
    int64_t kb = brp[R];
    for (int32_t c = bcsr_next_block(p, e, col); c != INT32_MAX;
         c = bcsr_next_block(p, e, col), ++kb) {
        bcol[kb] = c;
        unsigned bits = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            while (p[k] < e[k] && (col[p[k]] >> 2) == c) {
                const int cc = col[p[k]] & 3;
                bval[kb * 16 + k * 4 + cc] = val[p[k]];
                bits |= 1u << (k * 4 + cc);
                ++p[k];
            }
        pres[kb] = (uint16_t)bits;
    }
}

// Inverse: per row, the count of stored entries, then the entries in block
// order (ascending columns).
__global__ void k_bcsr_rowcount(int64_t mb, int64_t m, const int32_t *__restrict__ brp,
                                const uint16_t *__restrict__ pres, int32_t *__restrict__ counts) {
    int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= mb) return;
    int32_t c[4] = {0, 0, 0, 0};
    for (int64_t kb = brp[R]; kb < brp[R + 1]; ++kb) {
        const unsigned bits = pres[kb];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] += __popc((bits >> (4 * k)) & 15u);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (4 * R + k < m) counts[4 * R + k] = c[k];
}

template <typename U>
__global__ void k_bcsr_gather(int64_t mb, int64_t m, const int32_t *__restrict__ brp,
                              const int32_t *__restrict__ bcol, const U *__restrict__ bval,
                              const uint16_t *__restrict__ pres, const int32_t *__restrict__ rp,
                              int32_t *__restrict__ col, U *__restrict__ val) {
    int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= mb) return;
    for (int k = 0; k < 4; ++k) {
        const int64_t r = 4 * R + k;
        if (r >= m) break;
        int64_t q = rp[r];
        for (int64_t kb = brp[R]; kb < brp[R + 1]; ++kb) {
            const unsigned bits = pres[kb];
            for (int cc = 0; cc < 4; ++cc)
                if ((bits >> (4 * k + cc)) & 1u) {
                    col[q] = bcol[kb] * 4 + cc;
                    val[q] = bval[kb * 16 + k * 4 + cc];
                    ++q;
                }
        }
    }
}

}  // namespace


spmv_status launch_csr_to_coo(int64_t m, int64_t nnz, const int32_t *rp, int32_t *row_idx,
                              hipStream_t s) {
    if (nnz == 0) return SPMV_OK;
    k_csr_to_coo<<<grid_for((nnz + kEntryRun - 1) / kEntryRun, kBlock), kBlock, 0, s>>>(
        m, nnz, rp, row_idx);
    SMAT_LAUNCHED("csr_to_coo");
    return SPMV_OK;
}

spmv_status launch_csr_to_ell(int64_t m, int64_t m_pad, int K, const int32_t *rp,
                              const int32_t *col, const void *val, int elt, int32_t *ecol,
                              void *eval, hipStream_t s) {
    if (K == 0 || m_pad == 0) return SPMV_OK;
    if (elt == 8)
        k_csr_to_ell<uint64_t><<<grid_for(m_pad, kBlock), kBlock, 0, s>>>(
            m, m_pad, K, rp, col, (const uint64_t *)val, ecol, (uint64_t *)eval);
    else
        k_csr_to_ell<uint32_t><<<grid_for(m_pad, kBlock), kBlock, 0, s>>>(
            m, m_pad, K, rp, col, (const uint32_t *)val, ecol, (uint32_t *)eval);
    SMAT_LAUNCHED("csr_to_ell");
    return SPMV_OK;
}

spmv_status launch_csr_to_dia(int64_t m, int64_t n, int64_t m_pad, int64_t nnz, const int32_t *rp,
                              const int32_t *col, const void *val, int elt,
                              const unsigned int *slot_map, void *data, uint32_t *present,
                              hipStream_t s) {
    (void)n;
    if (nnz == 0) return SPMV_OK;
    unsigned g = grid_for((nnz + kEntryRun - 1) / kEntryRun, kBlock);
    if (elt == 8)
        k_csr_to_dia<uint64_t><<<g, kBlock, 0, s>>>(m, m_pad, nnz, rp, col,
                                                    (const uint64_t *)val, slot_map,
                                                    (uint64_t *)data, present);
    else
        k_csr_to_dia<uint32_t><<<g, kBlock, 0, s>>>(m, m_pad, nnz, rp, col,
                                                    (const uint32_t *)val, slot_map,
                                                    (uint32_t *)data, present);
    SMAT_LAUNCHED("csr_to_dia");
    return SPMV_OK;
}

spmv_status launch_coo_to_csr(int64_t m, int64_t nnz, const int32_t *row_idx, int32_t *rp,
                              hipStream_t s) {
    k_coo_to_csr<<<grid_for(m + 1, kBlock), kBlock, 0, s>>>(m, nnz, row_idx, rp);
    SMAT_LAUNCHED("coo_to_csr");
    return SPMV_OK;
}

spmv_status launch_ell_to_csr(int64_t m, int64_t m_pad, int K, const int32_t *ecol,
                              const void *eval, int elt, int32_t *rp, int32_t *col, void *val,
                              int32_t *counts, unsigned int *scratch, hipStream_t s) {
    if (m > 0) {
        k_ell_count<<<grid_for(m, kBlock), kBlock, 0, s>>>(m, m_pad, K, ecol, counts);
        SMAT_LAUNCHED("ell_count");
    }
    spmv_status st = launch_exclusive_scan_rows(m, counts, rp, scratch, s);
    if (st != SPMV_OK) return st;
    if (m == 0) return SPMV_OK;
    if (elt == 8)
        k_ell_gather<uint64_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, m_pad, K, ecol, (const uint64_t *)eval, rp, col, (uint64_t *)val);
    else
        k_ell_gather<uint32_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, m_pad, K, ecol, (const uint32_t *)eval, rp, col, (uint32_t *)val);
    SMAT_LAUNCHED("ell_gather");
    return SPMV_OK;
}

spmv_status launch_dia_to_csr(int64_t m, int64_t n, int64_t m_pad, int D, const int32_t *offs,
                              const void *data, const uint32_t *present, int elt, int32_t *rp,
                              int32_t *col, void *val, int32_t *counts, unsigned int *scratch,
                              hipStream_t s) {
    (void)n;
    if (m > 0) {
        k_dia_count<<<grid_for(m, kBlock), kBlock, 0, s>>>(m, m_pad, D, present, counts);
        SMAT_LAUNCHED("dia_count");
    }
    spmv_status st = launch_exclusive_scan_rows(m, counts, rp, scratch, s);
    if (st != SPMV_OK) return st;
    if (m == 0) return SPMV_OK;
    if (elt == 8)
        k_dia_gather<uint64_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, m_pad, D, offs, (const uint64_t *)data, present, rp, col, (uint64_t *)val);
    else
        k_dia_gather<uint32_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, m_pad, D, offs, (const uint32_t *)data, present, rp, col, (uint32_t *)val);
    SMAT_LAUNCHED("dia_gather");
    return SPMV_OK;
}

spmv_status launch_csr_to_panels(int64_t m, int64_t nnz, const int32_t *rp, const int32_t *col,
                                 const void *val, int elt, const int32_t *rows, int P, int64_t w,
                                 int32_t *inv, int32_t *cnt, int32_t *prow, unsigned *scan,
                                 int32_t *pcol, void *pval, hipStream_t s) {
    if (m == 0) return SPMV_OK;
    k_inverse_perm<<<grid_for(m, kBlock), kBlock, 0, s>>>(m, rows, inv);
    SMAT_LAUNCHED("inverse_perm");
    k_panel_count<<<grid_for(m + 1, kBlock), kBlock, 0, s>>>(m, rp, col, rows, P, w, cnt);
    SMAT_LAUNCHED("panel_count");
    spmv_status st = launch_exclusive_scan_rows((int64_t)P * (m + 1), cnt, prow, scan, s);
    if (st != SPMV_OK) return st;
    if (nnz == 0) return SPMV_OK;
    unsigned g = grid_for((nnz + kEntryRun - 1) / kEntryRun, kBlock);
    if (elt == 8)
        k_panel_scatter<uint64_t><<<g, kBlock, 0, s>>>(m, nnz, rp, col, (const uint64_t *)val, inv,
                                                       w, prow, pcol, (uint64_t *)pval);
    else
        k_panel_scatter<uint32_t><<<g, kBlock, 0, s>>>(m, nnz, rp, col, (const uint32_t *)val, inv,
                                                       w, prow, pcol, (uint32_t *)pval);
    SMAT_LAUNCHED("panel_scatter");
    return SPMV_OK;
}

spmv_status launch_panels_to_csr(int64_t m, const int32_t *rows, int P, const int32_t *prow,
                                 const int32_t *pcol, const void *pval, int elt, int32_t *rp,
                                 int32_t *col, void *val, int32_t *counts, unsigned *scan,
                                 hipStream_t s) {
    if (m > 0) {
        k_panel_rowcount<<<grid_for(m, kBlock), kBlock, 0, s>>>(m, rows, P, prow, counts);
        SMAT_LAUNCHED("panel_rowcount");
    }
    spmv_status st = launch_exclusive_scan_rows(m, counts, rp, scan, s);
    if (st != SPMV_OK || m == 0) return st;
    if (elt == 8)
        k_panel_gather<uint64_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, rows, P, prow, pcol, (const uint64_t *)pval, rp, col, (uint64_t *)val);
    else
        k_panel_gather<uint32_t><<<grid_for(m, kBlock), kBlock, 0, s>>>(
            m, rows, P, prow, pcol, (const uint32_t *)pval, rp, col, (uint32_t *)val);
    SMAT_LAUNCHED("panel_gather");
    return SPMV_OK;
}

spmv_status launch_bin_rows(int64_t m, const int32_t *rp, const BinSpec &spec,
                            unsigned int *block_counts, int32_t *rows_out,
                            unsigned int *bin_offsets_dev, hipStream_t s) {
    if (m == 0) {
        SMAT_HIP(hipMemsetAsync(bin_offsets_dev, 0, sizeof(unsigned) * (kAdaptiveBins + 1), s));
        return SPMV_OK;
    }
    unsigned nblk = grid_for(m, kBlock);
    k_bin_count<<<nblk, kBlock, 0, s>>>(m, rp, spec, block_counts);
    SMAT_LAUNCHED("bin_count");
    k_bin_scan<<<1, 1024, 0, s>>>(block_counts, nblk, bin_offsets_dev);
    SMAT_LAUNCHED("bin_scan");
    k_bin_scatter<<<nblk, kBlock, 0, s>>>(m, rp, spec, block_counts, rows_out);
    SMAT_LAUNCHED("bin_scatter");
    return SPMV_OK;
}

spmv_status launch_bcsr_count(int64_t m, const int32_t *rp, const int32_t *col, int32_t *counts,
                              int32_t *brp, unsigned int *scratch, hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb > 0) {
        k_bcsr_count<<<grid_for(mb, kBlock), kBlock, 0, s>>>(mb, m, rp, col, counts);
        SMAT_LAUNCHED("bcsr_count");
    }
    return launch_exclusive_scan_rows(mb, counts, brp, scratch, s);
}

spmv_status launch_csr_to_bcsr(int64_t m, const int32_t *rp, const int32_t *col, const void *val,
                               int elt, const int32_t *brp, int32_t *bcol, void *bval,
                               uint16_t *pres, hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb == 0) return SPMV_OK;
    if (elt == 8)
        k_bcsr_fill<uint64_t><<<grid_for(mb, kBlock), kBlock, 0, s>>>(
            mb, m, rp, col, (const uint64_t *)val, brp, bcol, (uint64_t *)bval, pres);
    else
        k_bcsr_fill<uint32_t><<<grid_for(mb, kBlock), kBlock, 0, s>>>(
            mb, m, rp, col, (const uint32_t *)val, brp, bcol, (uint32_t *)bval, pres);
    SMAT_LAUNCHED("bcsr_fill");
    return SPMV_OK;
}

spmv_status launch_bcsr_to_csr(int64_t m, const int32_t *brp, const int32_t *bcol,
                               const void *bval, const uint16_t *pres, int elt, int32_t *rp,
                               int32_t *col, void *val, int32_t *counts, unsigned int *scratch,
                               hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb > 0) {
        k_bcsr_rowcount<<<grid_for(mb, kBlock), kBlock, 0, s>>>(mb, m, brp, pres, counts);
        SMAT_LAUNCHED("bcsr_rowcount");
    }
    spmv_status st = launch_exclusive_scan_rows(m, counts, rp, scratch, s);
    if (st != SPMV_OK || mb == 0) return st;
    if (elt == 8)
        k_bcsr_gather<uint64_t><<<grid_for(mb, kBlock), kBlock, 0, s>>>(
            mb, m, brp, bcol, (const uint64_t *)bval, pres, rp, col, (uint64_t *)val);
    else
        k_bcsr_gather<uint32_t><<<grid_for(mb, kBlock), kBlock, 0, s>>>(
            mb, m, brp, bcol, (const uint32_t *)bval, pres, rp, col, (uint32_t *)val);
    SMAT_LAUNCHED("bcsr_gather");
    return SPMV_OK;
}

}  // namespace smat
