// K11 multilevel batch: y_l = A_l x_l for every level of an AMG-style
// hierarchy (the paper's motivation, Section 1: AMG spends most of its time
// in SpMV over a series of diverse level matrices), or for any set of
// independent SpMVs of one value type (up to kMaxLevels plans).  Small
// matrices are far too small to fill the GPU on their own, so
//   mode 0: one persistent launch; workgroup w takes the (level, tile) work
//           items w, w + grid, w + 2 grid, ... of the list that runs through
//           the levels in order (largest first), so consecutive workgroups
//           share a level's tiles and no counter or atomic is involved;
//   mode 1: the per-level launches captured once into a HIP graph and
//           replayed.
// K12 stream copy (achievable HBM bandwidth probe) lives here as well.
#include "plan.hpp"
#include "spmv_device.hpp"

#include <algorithm>
#include <memory>

namespace smat {
namespace {

constexpr int kMaxLevels = 4096;      // persistent mode
constexpr int kMaxGraphPlans = 4096;  // graph mode
constexpr int kPBlock = 256;   // persistent workgroup size
constexpr int kPDiaRpt = 4;    // rows per thread of a DIA tile

enum LevelKind {
    LK_SCALAR = 0, LK_VECTOR = 1, LK_ADAPTIVE = 2, LK_ELL = 3, LK_DIA = 4, LK_DIA_DIRECT = 5,
    LK_BCSR = 6
};

// One level: its kernel kind, the tile shape of its plan (wide: a lane owns
// 16 bytes of consecutive rows in DIA / ELL) and its arrays.
struct LevelDesc {
    int kind, lanes, K, D, nwin, nt, wide;
    int64_t m, n, m_pad, tile_rows, tile_begin, mb;
    const int32_t *rp, *col, *ecol, *offs, *rows, *brp, *bcol;
    const void *val, *eval, *data, *bval;
    const DiaWindow *win;
    AdaptiveLaunch alaunch;
};

template <typename T, int L, bool NT>
__device__ __forceinline__ void vector_tile(const LevelDesc &d, int64_t tile, const T *x, T *y) {
    int64_t row = tile * (kPBlock / L) + threadIdx.x / L;
    int lane = threadIdx.x & (L - 1);
    if (row < d.m) {
        double acc = csr_row_lanes<T, L, NT>(row, lane, d.rp, d.col, (const T *)d.val, x);
        if (lane == 0) y[row] = (T)acc;
    }
}

// Level-kind sets the persistent kernel is compiled for (bit k: LevelKind
// k).  A launch takes the smallest set that holds the kinds of its levels:
// a kernel carrying only CSR code needs far fewer registers than one that
// also carries the wide DIA tiles, so more of its waves fit a CU.
constexpr unsigned kKindsRow = (1u << LK_SCALAR) | (1u << LK_VECTOR);
constexpr unsigned kKindsCsr = kKindsRow | (1u << LK_ADAPTIVE);
constexpr unsigned kKindsEll = 1u << LK_ELL;
constexpr unsigned kKindsDia = (1u << LK_DIA) | (1u << LK_DIA_DIRECT);
constexpr unsigned kKindsBcsr = 1u << LK_BCSR;
constexpr unsigned kKindsAll = kKindsCsr | kKindsEll | kKindsDia | kKindsBcsr;

// A tile of a BCSR level: kPBlock / L block rows, L lanes each.
template <typename T, int L, bool NT>
__device__ __forceinline__ void bcsr_tile(const LevelDesc &d, int64_t tile, const T *x, T *y) {
    const int64_t R = tile * (kPBlock / L) + threadIdx.x / L;
    if constexpr (sizeof(T) == 8) {
        if constexpr (L >= 8)
            bcsr_row_coop<L, NT>(R, threadIdx.x & (L - 1), d.mb, d.m, d.n, d.brp, d.bcol,
                                 (const double *)d.bval, x, y);
    } else {
        bcsr_row_lanes<T, L, NT>(R, threadIdx.x & (L - 1), d.mb, d.m, d.n, d.brp, d.bcol,
                                 (const T *)d.bval, x, y);
    }
}

// One (level, tile) work item; the same device functions as the stand-alone
// kernels, so each row is computed exactly as by the level's own run.  Only
// the kinds in KINDS are compiled in (the launch guarantees the levels'
// kinds are among them).
template <typename T, bool NT, unsigned KINDS>
__device__ __forceinline__ void batch_item(const LevelDesc &d, int64_t tile, const T *x, T *y,
                                           T *xs, double *part) {
    constexpr int W = 16 / (int)sizeof(T);
    switch (d.kind) {
    case LK_SCALAR: {
        if constexpr (!(KINDS & (1u << LK_SCALAR))) break;
        int64_t i = tile * kPBlock + threadIdx.x;
        if (i < d.m) y[i] = (T)csr_row_seq<T>(i, d.rp, d.col, (const T *)d.val, x);
        break;
    }
    case LK_VECTOR:
        if constexpr (!(KINDS & (1u << LK_VECTOR))) break;
        switch (d.lanes) {
        case 1: vector_tile<T, 1, NT>(d, tile, x, y); break;
        case 2: vector_tile<T, 2, NT>(d, tile, x, y); break;
        case 4: vector_tile<T, 4, NT>(d, tile, x, y); break;
        case 8: vector_tile<T, 8, NT>(d, tile, x, y); break;
        case 16: vector_tile<T, 16, NT>(d, tile, x, y); break;
        case 32: vector_tile<T, 32, NT>(d, tile, x, y); break;
        default: vector_tile<T, 64, NT>(d, tile, x, y); break;
        }
        break;
    case LK_ADAPTIVE:
        if constexpr (!(KINDS & (1u << LK_ADAPTIVE))) break;
        adaptive_block<T, NT, true>(d.alaunch, (unsigned)tile, d.rows, d.rp, d.col,
                                    (const T *)d.val, x, y, part);
        break;
    case LK_ELL:
        if constexpr (!(KINDS & (1u << LK_ELL))) break;
        if (d.wide) {
            int64_t i0 = (tile * kPBlock + threadIdx.x) * W;
            if (i0 < d.m) {
                double acc[W];
                ell_rows_wide<T, 4, W, NT>(i0, d.m, d.m_pad, d.K, d.ecol, (const T *)d.eval, x,
                                           acc);
#pragma unroll
                for (int e = 0; e < W; ++e)
                    if (i0 + e < d.m) y[i0 + e] = (T)acc[e];
            }
        } else {
            int64_t i = tile * kPBlock + threadIdx.x;
            if (i < d.m) y[i] = (T)ell_row<T, 4, NT>(i, d.m_pad, d.K, d.ecol, (const T *)d.eval, x);
        }
        break;
    case LK_DIA:
        if constexpr (!(KINDS & (1u << LK_DIA))) break;
        if (d.wide)
            dia_tile_lds<T, kPDiaRpt, NT, W>(tile * d.tile_rows, d.m, d.n, d.m_pad, d.offs,
                                             d.nwin, d.win, (const T *)d.data, x, y, xs);
        else
            dia_tile_lds<T, kPDiaRpt, NT>(tile * d.tile_rows, d.m, d.n, d.m_pad, d.offs, d.nwin,
                                          d.win, (const T *)d.data, x, y, xs);
        break;
    case LK_BCSR:
        if constexpr (!(KINDS & (1u << LK_BCSR))) break;
        switch (d.lanes) {
        case 1: bcsr_tile<T, 1, NT>(d, tile, x, y); break;
        case 2: bcsr_tile<T, 2, NT>(d, tile, x, y); break;
        case 4: bcsr_tile<T, 4, NT>(d, tile, x, y); break;
        case 8: bcsr_tile<T, 8, NT>(d, tile, x, y); break;
        case 16: bcsr_tile<T, 16, NT>(d, tile, x, y); break;
        case 32: bcsr_tile<T, 32, NT>(d, tile, x, y); break;
        default: bcsr_tile<T, 64, NT>(d, tile, x, y); break;
        }
        break;
    default:
        if constexpr (!(KINDS & (1u << LK_DIA_DIRECT))) break;
        if (d.wide)
            dia_tile_direct<T, kPDiaRpt, NT, W>(tile * d.tile_rows, d.m, d.n, d.m_pad, d.D,
                                                d.offs, (const T *)d.data, x, y);
        else
            dia_tile_direct<T, kPDiaRpt, NT>(tile * d.tile_rows, d.m, d.n, d.m_pad, d.D, d.offs,
                                             (const T *)d.data, x, y);
        break;
    }
}

// Work items base .. total-1 (items below `base` belong to levels launched
// on their own before this kernel), strided over the grid; an item's level
// is found by binary search over the levels' first items.  xy: the levels'
// x pointers, then their y pointers.
template <typename T, unsigned KINDS>
__global__ __launch_bounds__(kPBlock) void k_batch_persistent(const LevelDesc *__restrict__ L,
                                                              int nlev, int64_t base,
                                                              int64_t total,
                                                              const void *const *__restrict__ xy) {
    extern __shared__ unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    __shared__ double part[kPBlock / kWave];
    for (int64_t t = base + blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = nlev - 1;   // the last level whose first item is <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const LevelDesc &d = L[lo];
        const int64_t tile = t - d.tile_begin;
        const T *x = (const T *)xy[lo];
        T *y = (T *)const_cast<void *>(xy[nlev + lo]);
        if (d.nt)
            batch_item<T, true, KINDS>(d, tile, x, y, xs, part);
        else
            batch_item<T, false, KINDS>(d, tile, x, y, xs, part);
        __syncthreads();  // LDS reuse by the next item
    }
}

// Grid-stride copy of 16-byte words, four independent words per thread and
// trip (all loads issued before the stores), streaming cache policy.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const v4u *__restrict__ src,
                                                     v4u *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        v4u a = __builtin_nontemporal_load(src + i);
        v4u b = __builtin_nontemporal_load(src + i + stride);
        v4u c = __builtin_nontemporal_load(src + i + 2 * stride);
        v4u d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Read-dominant bandwidth probe: a fixed grid streams the source with
// 16-byte non-temporal loads, eight in flight per thread, and each thread
// writes the word-wise sum of what it loaded (so no load can be dropped).
constexpr int kReadProbeBlocks = 256 * 8, kReadProbeThreads = 256;

__global__ __launch_bounds__(kReadProbeThreads) void k_stream_read(const v4u *__restrict__ src,
                                                                   int64_t n,
                                                                   v4u *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    v4u acc = {0u, 0u, 0u, 0u};
    for (; i + 7 * stride < n; i += 8 * stride) {
        v4u a = __builtin_nontemporal_load(src + i);
        v4u b = __builtin_nontemporal_load(src + i + stride);
        v4u c = __builtin_nontemporal_load(src + i + 2 * stride);
        v4u d = __builtin_nontemporal_load(src + i + 3 * stride);
        v4u e = __builtin_nontemporal_load(src + i + 4 * stride);
        v4u f = __builtin_nontemporal_load(src + i + 5 * stride);
        v4u g = __builtin_nontemporal_load(src + i + 6 * stride);
        v4u h = __builtin_nontemporal_load(src + i + 7 * stride);
        acc += a + b + c + d + e + f + g + h;
    }
    for (; i < n; i += stride) acc += __builtin_nontemporal_load(src + i);
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = acc;
}

// Random-gather probe: thread t adds val[i] * table[idx[i]] over i = t,
// t + G, t + 2 G, ... (G threads in the grid) in that order, four entries per
// trip -- the memory pattern of a CSR row loop (two coalesced streams and
// one gather per entry) without row pointers or y.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_probe(const T *__restrict__ table,
                                                      const int32_t *__restrict__ idx,
                                                      const T *__restrict__ val, int64_t count,
                                                      T *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double acc = 0.0;
#pragma unroll 4
    for (int64_t i = t; i < count; i += stride)
        acc = fma((double)val[i], (double)table[idx[i]], acc);
    out[t] = (T)acc;
}

}  // namespace

int64_t gather_probe_threads() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    return (int64_t)cus * 8 * 256;
}

spmv_status run_gather_probe(const void *table, const int32_t *idx, const void *val,
                             int64_t count, int elt, void *out, hipStream_t s) {
    const int64_t threads = gather_probe_threads();
    const unsigned g = (unsigned)(threads / 256);
    if (elt == 8)
        k_gather_probe<double><<<g, 256, 0, s>>>((const double *)table, idx, (const double *)val,
                                                 count, (double *)out);
    else
        k_gather_probe<float><<<g, 256, 0, s>>>((const float *)table, idx, (const float *)val,
                                                count, (float *)out);
    SMAT_LAUNCHED("gather_probe");
    return SPMV_OK;
}

size_t stream_read_out_bytes() { return (size_t)kReadProbeBlocks * kReadProbeThreads * 16; }

spmv_status run_stream_read(const void *src, size_t bytes, void *out, hipStream_t s) {
    k_stream_read<<<kReadProbeBlocks, kReadProbeThreads, 0, s>>>((const v4u *)src,
                                                                  (int64_t)(bytes / 16),
                                                                  (v4u *)out);
    SMAT_LAUNCHED("stream_read");
    return SPMV_OK;
}

spmv_status run_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return SPMV_OK;
    int dev = 0, cus = 256;
    SMAT_HIP(hipGetDevice(&dev));
    SMAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t g = std::min<int64_t>((n + 1023) / 1024, (int64_t)cus * 8);
    k_stream_copy<<<(unsigned)g, 256, 0, s>>>((const v4u *)src, (v4u *)dst, n);
    SMAT_LAUNCHED("stream_copy");
    return SPMV_OK;
}

}  // namespace smat

using namespace smat;

struct spmv_batch_s {
    int mode = 0;
    int nlev = 0;
    int elt = 8;
    std::vector<spmv_plan_t> plans;
    std::vector<int> persistent_levels;  // indices handled inside the persistent kernel
    std::vector<int64_t> tile_begin;     // first work item of each of them
    std::vector<int> kinds;              // and their LevelKind
    std::vector<int> extra_levels;       // launched separately
    int split = 0;  // leading persistent levels launched as their own kernels instead
    smat::Dev desc;
    smat::Dev xy;                        // x then y pointers of the persistent levels
    std::vector<const void *> xy_host;   // what xy holds
    int64_t total_tiles = 0;
    size_t lds_bytes = 0;
    int grid = 0;
    // graph mode
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
    std::vector<const void *> gx;
    std::vector<void *> gy;
    ~spmv_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

extern "C" spmv_status spmv_batch_create(const spmv_plan_t *plans, int32_t nplans, int32_t mode,
                                         spmv_batch_t *out) {
    const int most = mode == 1 ? kMaxGraphPlans : kMaxLevels;
    if (!out || !plans || (mode != 0 && mode != 1) || nplans <= 0 || nplans > most) {
        set_error("spmv_batch_create: mode 0 with 1..%d plans or mode 1 with 1..%d", kMaxLevels,
                  kMaxGraphPlans);
        return SPMV_EINVAL;
    }
    *out = nullptr;
    auto B = std::make_unique<spmv_batch_s>();
    B->mode = mode;
    B->nlev = nplans;
    B->elt = plans[0] ? plans[0]->elt : 8;
    for (int l = 0; l < nplans; ++l) {
        if (!plans[l]) {
            set_error("plan %d is NULL", l);
            return SPMV_EINVAL;
        }
        if (mode == 0 && plans[l]->elt != B->elt) {
            set_error("all plans of a persistent batch must share one dtype");
            return SPMV_EINVAL;
        }
        B->plans.push_back(plans[l]);
    }
    if (mode == 1) {
        SMAT_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        *out = B.release();
        return SPMV_OK;
    }
    std::vector<LevelDesc> descs;
    int64_t tiles = 0;
    for (int l = 0; l < nplans; ++l) {
        const spmv_plan_s &P = *plans[l];
        const Variant &V = *P.var;
        LevelDesc d{};
        d.m = P.m;
        d.n = P.n;
        d.m_pad = P.m_pad;
        d.rp = P.rp.as<int32_t>();
        d.col = P.col.as<int32_t>();
        d.val = P.val.p;
        d.nt = V.prm.stream_nt == 1;
        d.wide = V.prm.wide_loads == 1 ? 1 : 0;
        const int64_t wrows = d.wide ? 16 / P.elt : 1;
        int64_t ntiles = -1;  // work items of this level (default: rows / tile_rows)
        switch (V.kernel) {
        case SPMV_K_CSR_SCALAR: d.kind = LK_SCALAR; d.tile_rows = kPBlock; break;
        case SPMV_K_CSR_VECTOR:
            d.kind = LK_VECTOR;
            d.lanes = V.prm.vector_lanes;
            d.tile_rows = kPBlock / d.lanes;
            break;
        case SPMV_K_CSR_ADAPTIVE:
            // one work item per workgroup of the level's binned launch; rows
            // split into segments or long rows through LDS need their own
            // kernels
            d.kind = (V.nsplit_rows > 0 || V.long_tpr || !V.binned_rp.p) ? -1 : LK_ADAPTIVE;
            d.alaunch = V.alaunch;
            d.rows = V.bin_rows.as<int32_t>();
            // the rows' entries from the plan's copy in binned order
            d.rp = V.binned_rp.as<int32_t>();
            d.col = V.binned_col.as<int32_t>();
            d.val = V.binned_val.p;
            d.tile_rows = 1;
            ntiles = V.alaunch.first[8];
            break;
        case SPMV_K_ELL:
            d.kind = LK_ELL;
            d.tile_rows = kPBlock * wrows;
            d.K = V.K;
            d.ecol = V.ecol.as<int32_t>();
            d.eval = V.eval.p;
            break;
        case SPMV_K_DIA:
        case SPMV_K_DIA_DIRECT:
            d.kind = V.kernel == SPMV_K_DIA ? LK_DIA : LK_DIA_DIRECT;
            d.tile_rows = (int64_t)kPBlock * kPDiaRpt * wrows;
            d.D = V.D;
            d.nwin = V.nwin;
            d.offs = V.dia_off.as<int32_t>();
            d.win = V.dia_win.as<DiaWindow>();
            d.data = V.dia_data.p;
            if (d.kind == LK_DIA)
                B->lds_bytes = std::max(B->lds_bytes,
                                        (size_t)(d.tile_rows + V.max_span) * (size_t)P.elt);
            if (V.D == 0) d.kind = -1;
            break;
        case SPMV_K_BCSR:
            // the level's own lane count (float64: at least the 8 lanes of
            // one block), kPBlock / lanes block rows per work item
            d.kind = LK_BCSR;
            d.lanes = P.elt == 8 ? std::max(8, V.prm.bcsr_lanes) : V.prm.bcsr_lanes;
            d.mb = (P.m + 3) / 4;
            d.brp = V.brp.as<int32_t>();
            d.bcol = V.bcol.as<int32_t>();
            d.bval = V.bval.p;
            d.tile_rows = 4 * (kPBlock / d.lanes);
            break;
        default:
            d.kind = -1;
        }
        if (d.kind < 0 || P.m == 0) {
            B->extra_levels.push_back(l);
            continue;
        }
        d.tile_begin = tiles;
        B->tile_begin.push_back(tiles);
        tiles += ntiles >= 0 ? ntiles : (P.m + d.tile_rows - 1) / d.tile_rows;
        B->persistent_levels.push_back(l);
        B->kinds.push_back(d.kind);
        descs.push_back(d);
    }
    B->total_tiles = tiles;
    if (B->lds_bytes > 64 * 1024) {
        set_error("DIA window too wide for the persistent kernel's LDS");
        return SPMV_EUNSUPPORTED;
    }
    spmv_status st = B->desc.alloc(sizeof(LevelDesc) * std::max<size_t>(1, descs.size()));
    if (st != SPMV_OK) return st;
    st = B->xy.alloc(2 * sizeof(void *) * std::max<size_t>(1, descs.size()));
    if (st != SPMV_OK) return st;
    if (!descs.empty())
        SMAT_HIP(hipMemcpy(B->desc.p, descs.data(), sizeof(LevelDesc) * descs.size(),
                           hipMemcpyHostToDevice));
    int dev = 0, cus = 0;
    SMAT_HIP(hipGetDevice(&dev));
    SMAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    B->grid = (int)std::min<int64_t>(std::max<int64_t>(1, tiles), (int64_t)cus * 8);
    *out = B.release();
    return SPMV_OK;
}

extern "C" spmv_status spmv_batch_run(spmv_batch_t B, const void *const *xs, void *const *ys,
                                      void *stream) {
    if (!B || !xs || !ys) {
        set_error("spmv_batch_run: NULL argument");
        return SPMV_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (B->mode == 1) {
        bool same = B->exec && B->gx.size() == (size_t)B->nlev;
        for (int l = 0; same && l < B->nlev; ++l) same = B->gx[l] == xs[l] && B->gy[l] == ys[l];
        if (!same) {
            if (B->exec) (void)hipGraphExecDestroy(B->exec);
            if (B->graph) (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
            SMAT_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
            spmv_status st = SPMV_OK;
            for (int l = 0; l < B->nlev && st == SPMV_OK; ++l)
                st = spmv_run(B->plans[l], xs[l], ys[l], B->cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(B->cap, &g);
            if (st != SPMV_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            B->graph = g;
            SMAT_HIP(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
            B->gx.assign(xs, xs + B->nlev);
            B->gy.assign(ys, ys + B->nlev);
        }
        SMAT_HIP(hipGraphLaunch(B->exec, s));
        return SPMV_OK;
    }
    {
        // the persistent levels' vectors, uploaded when they change (the
        // upload waits for the copy, so that a later change cannot race it)
        const size_t np = B->persistent_levels.size();
        std::vector<const void *> v(2 * np);
        for (size_t k = 0; k < np; ++k) {
            v[k] = xs[B->persistent_levels[k]];
            v[np + k] = ys[B->persistent_levels[k]];
        }
        if (np && v != B->xy_host) {
            SMAT_HIP(hipMemcpyAsync(B->xy.p, v.data(), sizeof(void *) * v.size(),
                                    hipMemcpyHostToDevice, s));
            SMAT_HIP(hipStreamSynchronize(s));
            B->xy_host = v;
        }
    }
    for (int i = 0; i < B->split; ++i) {
        const int l = B->persistent_levels[i];
        spmv_status st = spmv_run(B->plans[l], xs[l], ys[l], s);
        if (st != SPMV_OK) return st;
    }
    const int64_t base = B->split < (int)B->tile_begin.size() ? B->tile_begin[B->split]
                                                              : B->total_tiles;
    if (B->total_tiles > base) {
        const int grid = (int)std::min<int64_t>(B->grid, B->total_tiles - base);
        unsigned kinds = 0;
        for (size_t i = (size_t)B->split; i < B->kinds.size(); ++i) kinds |= 1u << B->kinds[i];
        const LevelDesc *L = B->desc.as<LevelDesc>();
        const int nl = (int)B->persistent_levels.size();
        const int64_t tot = B->total_tiles;
#define SMAT_PERSISTENT(T, K)                                                                \
    k_batch_persistent<T, K><<<grid, kPBlock, B->lds_bytes, s>>>(L, nl, base, tot,         \
                                                                 B->xy.as<const void *>())
#define SMAT_PERSISTENT_SET(T)                                                               \
    do {                                                                                     \
        if ((kinds & ~kKindsRow) == 0)                                                       \
            SMAT_PERSISTENT(T, kKindsRow);                                                   \
        else if ((kinds & ~(kKindsRow | kKindsBcsr)) == 0)                                   \
            SMAT_PERSISTENT(T, (kKindsRow | kKindsBcsr));                                    \
        else if ((kinds & ~kKindsCsr) == 0)                                                  \
            SMAT_PERSISTENT(T, kKindsCsr);                                                   \
        else if ((kinds & ~kKindsEll) == 0)                                                  \
            SMAT_PERSISTENT(T, kKindsEll);                                                   \
        else if ((kinds & ~kKindsDia) == 0)                                                  \
            SMAT_PERSISTENT(T, kKindsDia);                                                   \
        else if ((kinds & ~(kKindsCsr | kKindsEll | kKindsBcsr)) == 0)                       \
            SMAT_PERSISTENT(T, (kKindsCsr | kKindsEll | kKindsBcsr));                        \
        else                                                                                 \
            SMAT_PERSISTENT(T, kKindsAll);                                                   \
    } while (0)
        if (B->elt == 8)
            SMAT_PERSISTENT_SET(double);
        else
            SMAT_PERSISTENT_SET(float);
#undef SMAT_PERSISTENT_SET
#undef SMAT_PERSISTENT
        SMAT_LAUNCHED("batch_persistent");
    }
    for (int l : B->extra_levels) {
        spmv_status st = spmv_run(B->plans[l], xs[l], ys[l], s);
        if (st != SPMV_OK) return st;
    }
    return SPMV_OK;
}

extern "C" spmv_status spmv_batch_tune(spmv_batch_t B, const void *const *xs, void *const *ys,
                                       int32_t reps, void *stream, int32_t *grid_out) {
    if (!B || !xs || !ys) {
        set_error("spmv_batch_tune: NULL argument");
        return SPMV_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (reps < 1) reps = 5;
    if (B->mode == 0 && B->total_tiles > 0) {
        int dev = 0, cus = 0;
        SMAT_HIP(hipGetDevice(&dev));
        SMAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        hipEvent_t a, b;
        SMAT_HIP(hipEventCreate(&a));
        SMAT_HIP(hipEventCreate(&b));
        int best_grid = B->grid, best_split = 0;
        float best = 1e30f;
        spmv_status st = SPMV_OK;
        const int npers = (int)B->persistent_levels.size();
        // leading levels large enough to fill the GPU alone may run faster as
        // their own (tuned) kernels; at least one level stays persistent
        for (int split = 0; split <= std::min(2, npers - 1) && st == SPMV_OK; ++split) {
            B->split = split;
            for (int mult : {1, 2, 4, 8, 16}) {
                B->grid = (int)std::min<int64_t>(std::max<int64_t>(1, B->total_tiles),
                                                 (int64_t)cus * mult);
                st = spmv_batch_run(B, xs, ys, stream);  // warm-up
                std::vector<float> t;
                for (int r = 0; r < reps && st == SPMV_OK; ++r) {
                    (void)hipEventRecord(a, s);
                    st = spmv_batch_run(B, xs, ys, stream);
                    (void)hipEventRecord(b, s);
                    (void)hipEventSynchronize(b);
                    float f = 0;
                    (void)hipEventElapsedTime(&f, a, b);
                    t.push_back(f);
                }
                if (st != SPMV_OK) break;
                std::sort(t.begin(), t.end());
                if (t[t.size() / 2] < best) {
                    best = t[t.size() / 2];
                    best_grid = B->grid;
                    best_split = split;
                }
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        B->grid = best_grid;
        B->split = best_split;
        if (st != SPMV_OK) return st;
    }
    if (grid_out) *grid_out = B->grid;
    return SPMV_OK;
}

extern "C" spmv_status spmv_batch_shape(spmv_batch_t B, int32_t *grid, int32_t *split) {
    if (!B) {
        set_error("spmv_batch_shape: NULL batch");
        return SPMV_EINVAL;
    }
    if (grid) *grid = B->mode == 0 ? B->grid : 0;
    if (split) *split = B->mode == 0 ? B->split : 0;
    return SPMV_OK;
}

extern "C" spmv_status spmv_batch_destroy(spmv_batch_t B) {
    delete B;
    return SPMV_OK;
}
