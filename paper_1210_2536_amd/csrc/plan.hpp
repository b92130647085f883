// Plan and variant state shared by the C-ABI translation units.
#pragma once

#include <memory>
#include <vector>

#include "internal.hpp"

namespace smat {

// The caller's allocator in effect on this thread (both callbacks NULL: the
// library's hipMalloc / hipFree).  Plan creation installs opts.allocator for
// its duration with AllocScope.
extern thread_local spmv_allocator g_alloc;

struct AllocScope {
    spmv_allocator saved;
    explicit AllocScope(const spmv_allocator &a) : saved(g_alloc) { g_alloc = a; }
    ~AllocScope() { g_alloc = saved; }
    AllocScope(const AllocScope &) = delete;
    AllocScope &operator=(const AllocScope &) = delete;
};

// Device allocation owned by a plan or a candidate; it remembers the
// allocator it came from and returns the memory there.
struct Dev {
    void *p = nullptr;
    size_t bytes = 0;
    spmv_allocator from{};
    bool borrowed = false;   // memory owned elsewhere (see borrow), never freed
    Dev() = default;
    Dev(const Dev &) = delete;
    Dev &operator=(const Dev &) = delete;
    ~Dev() { release(); }
    void release() {
        if (p && !borrowed) {
            if (from.free)
                from.free(p, bytes, from.ctx);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        from = spmv_allocator{};
        borrowed = false;
    }
    // Use `b` bytes at `q` (device memory someone else owns) as this buffer.
    void borrow(void *q, size_t b) {
        release();
        p = q;
        bytes = b;
        borrowed = true;
    }
    spmv_status alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        if (g_alloc.alloc) {
            p = g_alloc.alloc(b, g_alloc.ctx);
            if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) {
                if (p) g_alloc.free(p, b, g_alloc.ctx);
                p = nullptr;
                set_error("caller's allocator gave no 256-byte aligned block of %zu bytes", b);
                return SPMV_ENOMEM;
            }
            from = g_alloc;
            bytes = b;
            return SPMV_OK;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed: %s", b, hipGetErrorString(e));
            return SPMV_ENOMEM;
        }
        bytes = b;
        return SPMV_OK;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Kernel-specific state: the matrix in one format plus launch parameters.
struct Variant {
    int kernel = -1;
    spmv_params prm{};
    // COO
    Dev row_idx, coo_head, coo_tail, coo_flags;
    // ELL
    Dev ecol, eval;
    int K = 0;
    // DIA
    Dev dia_off, dia_data, dia_present, dia_win;
    int D = 0, nwin = 0, max_span = 0;
    // CSR adaptive; binned_*: the entries of the launch's rows in
    // binned order (the launch reads them, the plan's CSR serves the rest)
    Dev bin_rows, bin_scratch, split_segs, split_partials, split_begin, split_rows;
    Dev binned_rp, binned_col, binned_val;
    unsigned bin_off[kAdaptiveBins + 1] = {};
    int bin_lanes[kAdaptiveBins] = {};
    AdaptiveLaunch alaunch{};
    // CSR column panels
    Dev prow, pcol, pval, ppart;
    int P = 0;
    // short rows summed directly (length bins 0 .. short_bins - 1) and the
    // launch geometries of the two parts
    int short_bins = 0;
    AdaptiveLaunch apanel{}, ashort{};
    int64_t panel_w = 0;
    int64_t nsplit_rows = 0, nsplit_segs = 0;
    // float64 long rows through LDS: lanes per row (0: off), their count,
    // and the binned launch without them
    int long_tpr = 0;
    int64_t n_long = 0;
    AdaptiveLaunch arest{};
    Dev long_rows;   // the long rows, longest first
    // long rows by tiles (x panel per workgroup) instead of x chunks
    bool long_tiles = false;
    int64_t tile_P = 0, tile_nb = 0;
    Dev tile_seg, tile_blocks, tile_part, tile_off, tile_pk, tile_val;
    // BCSR 4x4
    Dev brp, bcol, bval, bpres;
    int64_t nblocks = 0;
    uint64_t bytes() const {
        return row_idx.bytes + coo_head.bytes + coo_tail.bytes + coo_flags.bytes + ecol.bytes +
               eval.bytes + dia_off.bytes + dia_data.bytes + dia_present.bytes + dia_win.bytes +
               bin_rows.bytes + bin_scratch.bytes + split_segs.bytes + split_partials.bytes +
               split_begin.bytes + split_rows.bytes + prow.bytes + pcol.bytes + pval.bytes +
               ppart.bytes + brp.bytes + bcol.bytes + bval.bytes + bpres.bytes + long_rows.bytes +
               tile_seg.bytes + tile_blocks.bytes + tile_part.bytes + tile_off.bytes +
               tile_pk.bytes + tile_val.bytes + binned_rp.bytes + binned_col.bytes +
               binned_val.bytes;
    }
};


}  // namespace smat

struct spmv_selector_s {
    smat::Dev params, mean, stdv;
    int n_out = 0;
    bool has_domain = false;
    float lo[12] = {}, hi[12] = {};   // training range of the raw inputs
    // stage rule: a decision tree over the inputs known after the census
    std::vector<int32_t> st_feat, st_left, st_right, st_kernel;
    std::vector<float> st_thr, st_conf;
};

struct spmv_plan_s {
    spmv_allocator alloc{};            // the caller's allocator of this plan
    int device = -1;                   // the device the plan was created on
    int64_t m = 0, n = 0, nnz = 0;
    int dtype = 0, elt = 4;
    int64_t m_pad = 0;
    smat::Dev rp, col, val;             // CSR copy (CSR kernels and COO)
    bool has_csr = false;
    std::unique_ptr<smat::Variant> var; // the chosen kernel's state
    spmv_plan_info info{};
    smat::Dev diag_map;                 // diagonal -> slot map (kept only while converting)
    std::vector<int32_t> dia_offsets;
    // segmented plans: one plan per row segment, in row order
    std::vector<spmv_plan_s *> seg;
    std::vector<int64_t> seg_row0;
    ~spmv_plan_s() {
        for (auto *c : seg) delete c;
    }
};

