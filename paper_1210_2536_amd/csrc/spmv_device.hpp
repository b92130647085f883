// Per-row / per-tile SpMV device functions shared by the stand-alone kernels
// and the persistent multilevel kernel, so both compute every output with the
// same operations in the same order (bitwise-identical results).
//
// NT selects the cache policy of the matrix streams (values, column indices,
// diagonals): non-temporal loads keep them from displacing the reused x
// vector in L2, which helps banded matrices and can hurt gathers from
// large, randomly indexed x.  It is a tuning parameter (spmv_params
// stream_nt); the arithmetic is identical either way.
#pragma once

#include "internal.hpp"

namespace smat {

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Plain CSR row: one thread, storage order.
template <typename T>
__device__ __forceinline__ double csr_row_seq(int64_t i, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ col,
                                              const T *__restrict__ val,
                                              const T *__restrict__ x) {
    double acc = 0.0;
    int32_t b = rp[i], e = rp[i + 1];
    for (int32_t p = b; p < e; ++p) acc = fma((double)val[p], (double)x[col[p]], acc);
    return acc;
}

// CSR row by a group of L lanes (lane = 0..L-1); lanes stride the row and
// reduce by xor shuffles.  Every lane of the group returns the row sum.
template <typename T, int L, bool NT>
__device__ __forceinline__ double lanes_sum(int32_t b, int32_t e, int lane,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val,
                                            const T *__restrict__ x) {
    double acc = 0.0;
#pragma unroll 4
    for (int32_t p = b + lane; p < e; p += L)
        acc = fma((double)ld<NT>(val + p), (double)x[ld<NT>(col + p)], acc);
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
    return acc;
}

template <typename T, int L, bool NT>
__device__ __forceinline__ double csr_row_lanes(int64_t row, int lane,
                                                const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ col,
                                                const T *__restrict__ val,
                                                const T *__restrict__ x) {
    return lanes_sum<T, L, NT>(rp[row], rp[row + 1], lane, col, val, x);
}

// Entries [b, e) summed by a whole workgroup of B threads (B a multiple of
// 64); thread 0 returns the sum.  `part` is LDS scratch of B / 64 doubles.
template <typename T, int B, bool NT>
__device__ __forceinline__ double block_sum(int32_t b, int32_t e, const int32_t *__restrict__ col,
                                            const T *__restrict__ val, const T *__restrict__ x,
                                            double *part) {
    double acc = 0.0;
#pragma unroll 4
    for (int32_t p = b + threadIdx.x; p < e; p += B)
        acc = fma((double)ld<NT>(val + p), (double)x[ld<NT>(col + p)], acc);
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < B / kWave; ++w) s += part[w];
    __syncthreads();
    return s;
}

template <typename T, int B, bool NT>
__device__ __forceinline__ double csr_row_block(int64_t row, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ col,
                                                const T *__restrict__ val,
                                                const T *__restrict__ x, double *part) {
    return block_sum<T, B, NT>(rp[row], rp[row + 1], col, val, x, part);
}

// Length-binned CSR (one launch serves every bin, longest first).  Workgroup
// `bid` of the launch geometry `a` finds its bin b (7: a whole workgroup per
// row; 6..0: 64..1 lanes per row) and its rows in the binned order `rows`.
constexpr int kAdaptBlock = 256;

template <typename T, int L, bool NT, bool PK = false>
__device__ __forceinline__ void adaptive_lanes(unsigned local, unsigned rbeg, unsigned rend,
                                               const int32_t *__restrict__ rows,
                                               const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ col,
                                               const T *__restrict__ val, const T *__restrict__ x,
                                               T *__restrict__ y) {
    int64_t r = (int64_t)rbeg + (int64_t)local * (kAdaptBlock / L) + threadIdx.x / L;
    int lane = threadIdx.x & (L - 1);
    if (r < rend) {
        int64_t row = rows[r];
        double acc = csr_row_lanes<T, L, NT>(PK ? r : row, lane, rp, col, val, x);
        if (lane == 0) y[row] = (T)acc;
    }
}

// Every thread of the (kAdaptBlock-thread) workgroup must call it; `part` is
// LDS scratch of kAdaptBlock / 64 doubles.
template <typename T, bool NT, bool PK = false>
__device__ __forceinline__ void adaptive_block(const AdaptiveLaunch &a, unsigned bid,
                                               const int32_t *__restrict__ rows,
                                               const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ col,
                                               const T *__restrict__ val, const T *__restrict__ x,
                                               T *__restrict__ y, double *part) {
    int q = 0;
    while (q < 7 && bid >= a.first[q + 1]) ++q;
    const int b = 7 - q;
    const unsigned local = bid - a.first[q];
    const unsigned rb = a.row_begin[b], re = a.row_begin[b + 1];
    switch (b) {
    case 7: {
        int64_t row = rows[rb + local];
        double s = csr_row_block<T, kAdaptBlock, NT>(PK ? (int64_t)(rb + local) : row, rp, col,
                                                     val, x, part);
        if (threadIdx.x == 0) y[row] = (T)s;
        break;
    }
    case 6: adaptive_lanes<T, 64, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    case 5: adaptive_lanes<T, 32, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    case 4: adaptive_lanes<T, 16, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    case 3: adaptive_lanes<T, 8, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    case 2: adaptive_lanes<T, 4, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    case 1: adaptive_lanes<T, 2, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    default: adaptive_lanes<T, 1, NT, PK>(local, rb, re, rows, rp, col, val, x, y); break;
    }
}

// ELL row: slots in order, U slots loaded ahead of use.
template <typename T, int U, bool NT>
__device__ __forceinline__ double ell_row(int64_t i, int64_t m_pad, int K,
                                          const int32_t *__restrict__ ecol,
                                          const T *__restrict__ eval, const T *__restrict__ x) {
    double acc = 0.0;
    int k = 0;
    for (; k + U <= K; k += U) {
        int32_t c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t s = (int64_t)(k + u) * m_pad + i;
            c[u] = ld<NT>(ecol + s);
            v[u] = ld<NT>(eval + s);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) acc = fma((double)v[u], (double)x[c[u]], acc);
    }
    for (; k < K; ++k) {
        int64_t s = (int64_t)k * m_pad + i;
        int32_t c = ld<NT>(ecol + s);
        if (c >= 0) acc = fma((double)ld<NT>(eval + s), (double)x[c], acc);
    }
    return acc;
}

// V consecutive elements of a matrix stream as one load (V * sizeof(T) bytes;
// the address is a multiple of that size).
template <typename T, int V, bool NT>
__device__ __forceinline__ void ld_rows(const T *p, T (&v)[V]) {
    if constexpr (V == 1) {
        v[0] = ld<NT>(p);
    } else {
        typedef T vec __attribute__((ext_vector_type(V)));
        vec w = ld<NT>(reinterpret_cast<const vec *>(p));
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = w[e];
    }
}

// ELL rows i0 .. i0+V-1 of one lane (i0 a multiple of V, i0 < m): the slot
// columns and values of the V rows come in one load each.  Each row's sum
// runs over its slots in order, exactly as ell_row.
template <typename T, int U, int V, bool NT>
__device__ __forceinline__ void ell_rows_wide(int64_t i0, int64_t m, int64_t m_pad, int K,
                                              const int32_t *__restrict__ ecol,
                                              const T *__restrict__ eval,
                                              const T *__restrict__ x, double (&acc)[V]) {
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] = 0.0;
    int k = 0;
    for (; k + U <= K; k += U) {
        int32_t c[U][V];
        T v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t s = (int64_t)(k + u) * m_pad + i0;
            ld_rows<int32_t, V, NT>(ecol + s, c[u]);
            ld_rows<T, V, NT>(eval + s, v[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (i0 + e < m && c[u][e] >= 0)
                    acc[e] = fma((double)v[u][e], (double)x[c[u][e]], acc[e]);
    }
    for (; k < K; ++k) {
        int64_t s = (int64_t)k * m_pad + i0;
        int32_t c[V];
        T v[V];
        ld_rows<int32_t, V, NT>(ecol + s, c);
        ld_rows<T, V, NT>(eval + s, v);
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (i0 + e < m && c[e] >= 0) acc[e] = fma((double)v[e], (double)x[c[e]], acc[e]);
    }
}

// DIA tile with x windows staged in LDS; every thread of the workgroup must
// call it (it synchronises).  The tile holds R = blockDim * RPT * V rows; a
// lane takes V consecutive rows per step (one V-wide load of each diagonal),
// steps q = 0..RPT-1 being blockDim * V rows apart.  Each row sums its
// diagonals in ascending offset order whatever RPT and V.
template <typename T, int RPT, bool NT, int V = 1>
__device__ __forceinline__ void dia_tile_lds(int64_t r0, int64_t m, int64_t n, int64_t m_pad,
                                             const int32_t *__restrict__ offs, int nwin,
                                             const DiaWindow *__restrict__ win,
                                             const T *__restrict__ data,
                                             const T *__restrict__ x, T *__restrict__ y, T *xs) {
    const int R = blockDim.x * RPT * V;
    double acc[RPT][V];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[q][e] = 0.0;
    for (int w = 0; w < nwin; ++w) {
        const int d0 = win[w].d0, d1 = win[w].d1;
        const int lo = offs[d0], hi = offs[d1];
        const int len = R + (hi - lo);
        __syncthreads();  // previous window fully consumed
        for (int t = threadIdx.x; t < len; t += blockDim.x) {
            int64_t j = r0 + lo + t;
            xs[t] = (j >= 0 && j < n) ? x[j] : T(0);
        }
        __syncthreads();
        for (int d = d0; d <= d1; ++d) {
            const int sh = offs[d] - lo;
            const T *dd = data + (int64_t)d * m_pad + r0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int il = (threadIdx.x + q * blockDim.x) * V;
                if (r0 + il < m) {
                    T v[V];
                    ld_rows<T, V, NT>(dd + il, v);
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        acc[q][e] = fma((double)v[e], (double)xs[il + e + sh], acc[q][e]);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i0 = r0 + (int64_t)(threadIdx.x + q * blockDim.x) * V;
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (i0 + e < m) y[i0 + e] = (T)acc[q][e];
    }
}

// DIA tile reading x through the caches (same row layout as dia_tile_lds).
template <typename T, int RPT, bool NT, int V = 1>
__device__ __forceinline__ void dia_tile_direct(int64_t r0, int64_t m, int64_t n, int64_t m_pad,
                                                int D, const int32_t *__restrict__ offs,
                                                const T *__restrict__ data,
                                                const T *__restrict__ x, T *__restrict__ y) {
    double acc[RPT][V];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[q][e] = 0.0;
    for (int d = 0; d < D; ++d) {
        const int64_t off = offs[d];
        const T *dd = data + (int64_t)d * m_pad;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t i0 = r0 + (int64_t)(threadIdx.x + q * blockDim.x) * V;
            if (i0 < m) {
                T v[V];
                ld_rows<T, V, NT>(dd + i0, v);
                const int64_t j0 = i0 + off;
                if (V > 1 && j0 >= 0 && j0 + V <= n) {
                    // x[j0 .. j0+V) in one load; j0 is only element-aligned
                    typedef T vec __attribute__((ext_vector_type(V)));
                    vec xv;
                    __builtin_memcpy(&xv, x + j0, sizeof(vec));
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        acc[q][e] = fma((double)v[e], (double)xv[e], acc[q][e]);
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const int64_t j = j0 + e;
                        if (j >= 0 && j < n)
                            acc[q][e] = fma((double)v[e], (double)x[j], acc[q][e]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i0 = r0 + (int64_t)(threadIdx.x + q * blockDim.x) * V;
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (i0 + e < m) y[i0 + e] = (T)acc[q][e];
    }
}

// ---------------------------------------------------------------- BCSR 4x4
// Block row R (rows 4R .. 4R+3) by L lanes; every lane of the wave must
// call (the lane sums are added by shuffles), R >= mb contributing nothing.
//
// bcsr_row_lanes (float32 form): lane l takes blocks l, l + L, ... of its
// block row; a block's 16 values (row-major) arrive in 16-byte loads, its 4
// x values in one (element-aligned) load away from the last column block;
// one running sum per row, the L lanes' sums added by xor shuffles.
template <typename T, int L, bool NT>
__device__ __forceinline__ void bcsr_row_lanes(int64_t R, int lane, int64_t mb, int64_t m,
                                               int64_t n, const int32_t *__restrict__ brp,
                                               const int32_t *__restrict__ bcol,
                                               const T *__restrict__ bval,
                                               const T *__restrict__ x, T *__restrict__ y) {
    constexpr int V = 16 / (int)sizeof(T);   // values per 16-byte load
    typedef T vec __attribute__((ext_vector_type(V)));
    typedef T vec4 __attribute__((ext_vector_type(4)));
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (R < mb) {
        const int32_t kb = brp[R], ke = brp[R + 1];
        for (int32_t k = kb + lane; k < ke; k += L) {
            T v[16];
            const vec *src = reinterpret_cast<const vec *>(bval + (int64_t)k * 16);
#pragma unroll
            for (int q = 0; q < 16 / V; ++q) {
                vec w = ld<NT>(src + q);
#pragma unroll
                for (int e = 0; e < V; ++e) v[q * V + e] = w[e];
            }
            const int64_t c0 = (int64_t)ld<NT>(bcol + k) * 4;
            T xv[4];
            if (c0 + 4 <= n) {
                vec4 t;
                __builtin_memcpy(&t, x + c0, sizeof(t));
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) xv[cc] = t[cc];
            } else {
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) xv[cc] = c0 + cc < n ? x[c0 + cc] : T(0);
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int cc = 0; cc < 4; ++cc)
                    acc[rr] = fma((double)v[rr * 4 + cc], (double)xv[cc], acc[rr]);
        }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) acc[rr] += __shfl_xor(acc[rr], off, L);
    if (R < mb && lane == 0) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
            if (4 * R + rr < m) y[4 * R + rr] = (T)acc[rr];
    }
}

// bcsr_row_coop (float64 form, 8 <= L <= 64): a block's 128 bytes are read
// by 8 lanes together, 16 bytes (half a row) each, so a wave's loads are
// contiguous; G = L / 8 groups, group g taking blocks g, g + G, ...; a lane
// reads the 2 x values under its piece in one load and keeps one running
// sum for its row; the lanes of a row (the pair inside a block, then the G
// groups) are added by xor shuffles in a fixed order.
template <int L, bool NT>
__device__ __forceinline__ void bcsr_row_coop(int64_t R, int lane, int64_t mb, int64_t m,
                                              int64_t n, const int32_t *__restrict__ brp,
                                              const int32_t *__restrict__ bcol,
                                              const double *__restrict__ bval,
                                              const double *__restrict__ x,
                                              double *__restrict__ y) {
    constexpr int S = 8;                    // lanes per block, 2 values each
    constexpr int G = L / S;                // blocks of a row in flight
    static_assert(L >= S && L <= 64 && (L & (L - 1)) == 0, "lanes per block row");
    typedef double vec2 __attribute__((ext_vector_type(2)));
    const int g = lane / S, j = lane % S;
    const int row = j / 2;                  // block row of this lane's piece
    const int cc0 = 2 * (j % 2);            // first column of the piece
    double acc = 0.0;
    if (R < mb) {
        const int32_t kb = brp[R], ke = brp[R + 1];
        for (int32_t k = kb + g; k < ke; k += G) {
            const vec2 w = ld<NT>(reinterpret_cast<const vec2 *>(bval + (int64_t)k * 16) + j);
            const int64_t c0 = (int64_t)ld<NT>(bcol + k) * 4 + cc0;
            double x0, x1;
            if (c0 + 2 <= n) {
                vec2 t;
                __builtin_memcpy(&t, x + c0, sizeof(t));
                x0 = t[0];
                x1 = t[1];
            } else {
                x0 = c0 < n ? x[c0] : 0.0;
                x1 = c0 + 1 < n ? x[c0 + 1] : 0.0;
            }
            acc = fma(w[0], x0, acc);
            acc = fma(w[1], x1, acc);
        }
    }
    acc += __shfl_xor(acc, 1, L);   // the two halves of a block row
#pragma unroll
    for (int off = S; off < L; off <<= 1) acc += __shfl_xor(acc, off, L);
    if (R < mb && g == 0 && cc0 == 0 && 4 * R + row < m) y[4 * R + row] = acc;
}

}  // namespace smat
