// devmatrix.cpp -- a CSR row block on the device with its SpMV schedule.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>

#include "cgmi_host.h"

namespace cgmi {

namespace {

int lanes_for_length(int64_t len) {
    int L = 1;
    while (L < len && L < 64) L <<= 1;
    return L;
}

void free_blocks(DevMatrix &M) {
    for (DevMatrix &B : M.blocks) dm_free(B);
    M.blocks.clear();
    delete M.cb;
    M.cb = nullptr;
}

void free_sliced(DevMatrix &M) {
    (void)hipFree(M.d_sell_off);
    (void)hipFree(M.d_sell_ci);
    (void)hipFree(M.d_sell_val);
    (void)hipFree(M.d_sell_val32);
    (void)hipFree(M.d_sell_idx);
    (void)hipFree(M.d_sell_dict);
    (void)hipFree(M.d_sell_len);
    M.d_sell_len = nullptr;
    M.d_sell_off = M.d_sell_ci = nullptr;
    M.d_sell_val = nullptr;
    M.d_sell_val32 = nullptr;
    M.d_sell_idx = nullptr;
    M.d_sell_dict = nullptr;
    M.sell_slots = 0;
    (void)hipFree(M.d_st_off);
    (void)hipFree(M.d_st_offs);
    (void)hipFree(M.d_st_mask);
    (void)hipFree(M.d_st_val);
    M.d_st_off = M.d_st_offs = nullptr;
    M.d_st_mask = nullptr;
    M.d_st_val = nullptr;
    M.st_slots = 0;
    (void)hipFree(M.d_sell_lenx);
    (void)hipFree(M.d_sell_gap);
    M.d_sell_lenx = nullptr;
    M.d_sell_gap = nullptr;
    M.gap_state = 0;
    M.use_gap = false;
}

// Slot offsets of the sliced layout: slice t holds max(1, longest row) slots
// of 64 entries each.
void slice_offsets(const DevMatrix &M, int32_t nt, std::vector<int32_t> &off) {
    const int32_t m = M.m;
    off.assign((size_t)nt + 1, 0);
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        int32_t w = 0;
        for (int32_t i = t * kWaveSize; i < std::min(m, (t + 1) * kWaveSize); ++i)
            w = std::max(w, M.h_rp[i + 1] - M.h_rp[i]);
        off[t + 1] = std::max(w, 1) * kWaveSize;
    }
    for (int32_t t = 0; t < nt; ++t) off[t + 1] += off[t];
}

// Stencil-sliced copy (see kTileStencil): per 64-row slice the sorted union
// of the rows' column offsets, slot j of each row at offset j (value 0 where
// absent) and a byte of slot bits per row.  false (nothing uploaded) when a
// slice has more than kSliceMaxWidth distinct offsets; needs the host values.
int build_stencil(DevMatrix &M, bool *fits) {
    *fits = false;
    if (M.d_st_val) {
        *fits = true;
        return CG_OK;
    }
    const int32_t m = M.m, nt = (m + kWaveSize - 1) / kWaveSize;
    constexpr int W = kSliceMaxWidth;
    std::vector<int32_t> offs((size_t)nt * W, 0), width((size_t)nt, 1), off((size_t)nt + 1, 0);
    std::atomic<bool> ok{true};
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        if (!ok.load(std::memory_order_relaxed)) continue;
        int32_t u[W];
        int nu = 0;
        for (int32_t i = t * kWaveSize; i < std::min(m, (t + 1) * kWaveSize) && nu <= W; ++i)
            for (int32_t k = M.h_rp[i]; k < M.h_rp[i + 1]; ++k) {
                const int32_t o = M.h_ci[k] - (M.pad_col_base + i);
                int e = 0;
                while (e < nu && u[e] != o) ++e;
                if (e == nu) {
                    if (nu == W) {
                        nu = W + 1;
                        break;
                    }
                    u[nu++] = o;
                }
            }
        if (nu > W) {
            ok = false;
            continue;
        }
        std::sort(u, u + nu);
        for (int e = 0; e < nu; ++e) offs[(size_t)t * W + e] = u[e];
        width[(size_t)t] = std::max(nu, 1);
    }
    if (!ok.load()) return CG_OK;
    for (int32_t t = 0; t < nt; ++t) off[t + 1] = off[t] + width[(size_t)t] * kWaveSize;
    if ((int64_t)off[nt] >= INT32_MAX) return CG_OK;
    const size_t slots = (size_t)off[nt];
    const bool host_vals = !M.h_val.empty();
    std::vector<double> sval(host_vals ? slots : 0, 0.0);
    std::vector<uint8_t> mask((size_t)nt * kWaveSize, 0);
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        const int32_t *u = &offs[(size_t)t * W];
        const int w = width[(size_t)t];
        for (int32_t l = 0; l < kWaveSize; ++l) {
            const int32_t i = t * kWaveSize + l;
            if (i >= m) break;
            uint8_t bits = 0;
            int e = 0;
            for (int32_t k = M.h_rp[i]; k < M.h_rp[i + 1]; ++k) {
                const int32_t o = M.h_ci[k] - (M.pad_col_base + i);
                while (e < w && u[e] != o) ++e;   // offsets ascend with the columns
                bits |= (uint8_t)(1u << e);
                if (host_vals) sval[(size_t)off[t] + (size_t)e * kWaveSize + l] = M.h_val[k];
                ++e;
            }
            mask[(size_t)i] = bits;
        }
    }
    hipError_t e = dmalloc(&M.d_st_off, off.size());
    if (e == hipSuccess) e = dmalloc(&M.d_st_offs, offs.size());
    if (e == hipSuccess) e = dmalloc(&M.d_st_mask, mask.size());
    if (e == hipSuccess) e = dmalloc(&M.d_st_val, slots);
    if (e == hipSuccess) e = hipMemcpy(M.d_st_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(M.d_st_offs, offs.data(), sizeof(int32_t) * offs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.d_st_mask, mask.data(), mask.size(), hipMemcpyHostToDevice);
    // values from the host copy, or zero until the owner writes them on the device
    if (e == hipSuccess)
        e = host_vals ? hipMemcpy(M.d_st_val, sval.data(), sizeof(double) * slots, hipMemcpyHostToDevice)
                      : hipMemset(M.d_st_val, 0, sizeof(double) * slots);
    if (e != hipSuccess) {
        (void)hipFree(M.d_st_off);
        (void)hipFree(M.d_st_offs);
        (void)hipFree(M.d_st_mask);
        (void)hipFree(M.d_st_val);
        M.d_st_off = M.d_st_offs = nullptr;
        M.d_st_mask = nullptr;
        M.d_st_val = nullptr;
        return fail(CG_ENOMEM, "stencil layout upload failed: %s", hipGetErrorString(e));
    }
    M.st_slots = slots;
    *fits = true;
    return CG_OK;
}


// Dictionary of column offsets (column - global row) of each 64-row slice;
// false if some slice has more than kDictSize - 1 distinct offsets or a row
// longer than kSliceMaxWidth.  dict: kDictSize entries per slice (unused and
// entry kDictSize-1 are 0); idx: one word of 8 nibbles per lane and slice.
bool dict_slice(const DevMatrix &M, int32_t t, int32_t *d, uint32_t *idx_t);

bool build_dict(const DevMatrix &M, std::vector<int32_t> &dict, std::vector<uint32_t> &idx) {
    const int32_t m = M.m, nt = (m + kWaveSize - 1) / kWaveSize;
    dict.assign((size_t)nt * kDictSize, 0);
    idx.assign((size_t)nt * kWaveSize, 0);
    std::atomic<bool> ok{true};
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        if (!ok.load(std::memory_order_relaxed)) continue;
        if (!dict_slice(M, t, &dict[(size_t)t * kDictSize], &idx[(size_t)t * kWaveSize])) ok = false;
    }
    return ok.load();
}

// Dictionary and packed indices of slice t; false if it does not fit.
bool dict_slice(const DevMatrix &M, int32_t t, int32_t *d, uint32_t *idx_t) {
    const int32_t m = M.m;
    {
        int nd = 0;
        for (int32_t l = 0; l < kWaveSize; ++l) {
            const int32_t i = t * kWaveSize + l;
            const int32_t len = i < m ? M.h_rp[i + 1] - M.h_rp[i] : 0;
            if (len > kSliceMaxWidth) return false;
            uint32_t w = 0;
            for (int j = 0; j < kSliceMaxWidth; ++j) {
                uint32_t nib = kDictPad;
                if (j < len) {
                    const int32_t off = M.h_ci[M.h_rp[i] + j] - (M.pad_col_base + i);
                    int e = 0;
                    while (e < nd && d[e] != off) ++e;
                    if (e == nd) {
                        if (nd == kDictSize - 1) return false;
                        d[nd++] = off;
                    }
                    nib = (uint32_t)e;
                }
                w |= nib << (4 * j);
            }
            idx_t[l] = w;
        }
    }
    return true;
}

// Column blocks when most entries lie farther than a block width from the
// diagonal of a vector of at least two blocks (gathers would miss the L2).
// Lanes-per-row classes.  Sliced tiles for rows of at most 64 nonzeros when
// slicing pads by at most 25%; stream tiles when requested and every 64-row
// tile fits; otherwise vector bins: rows of similar length keep their natural
// order (one bin, no indirection), spread-out lengths are binned by the power
// of two covering the row length (row list per bin), rows longer than
// kHugeRow go to a workgroup-per-row list at the end.
// Adaptive stream tiles over rows [0, m) of a CSR (row pointers rp, m + 1):
// runs of at most 64 rows whose entries span at most kStreamNnz slots from
// the first entry rounded down to a multiple of 4, greedy in row order.
// tiles receives the first row of every tile and m at the end; false when a
// single row does not fit a tile.
bool stream_tiles(const int32_t *rp, int32_t m, std::vector<int32_t> &tiles) {
    tiles.clear();
    if (m <= 0) return false;
    auto span = [&](int32_t a, int32_t b) { return (rp[a] & 3) + (int64_t)rp[b] - rp[a]; };
    tiles.push_back(0);
    for (int32_t r0 = 0; r0 < m;) {
        int32_t r1 = r0 + 1;
        if (span(r0, r1) > kStreamNnz) {
            tiles.clear();
            return false;
        }
        while (r1 < m && r1 - r0 < kWaveSize && span(r0, r1 + 1) <= kStreamNnz) ++r1;
        tiles.push_back(r1);
        r0 = r1;
    }
    return true;
}

// Upload the tile list of adaptive stream tiles and make S their schedule.
int set_stream_tiles(DevMatrix &M, Schedule &S, const std::vector<int32_t> &tiles) {
    S = Schedule{};
    S.kind = kTileStream;
    S.identity = 1;
    S.nbins = 1;
    S.bins[0] = Bin{kWaveSize, 0, M.m, 0};
    S.ntiles = (int32_t)tiles.size() - 1;
    (void)hipFree(M.d_tile_row);
    M.d_tile_row = nullptr;
    hipError_t e = dmalloc(&M.d_tile_row, tiles.size());
    if (e == hipSuccess)
        e = hipMemcpy(M.d_tile_row, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(CG_ENOMEM, "tile rows upload failed: %s", hipGetErrorString(e));
    return CG_OK;
}

void build_schedule(const DevMatrix &M, int kind_opt, Schedule &S, std::vector<int32_t> &rows_out,
                    bool skip_empty = false, std::vector<int32_t> *tiles_out = nullptr) {
    S = Schedule{};
    const int32_t m = M.m;
    rows_out.clear();
    S.identity = 1;
    if (m == 0) return;
    if (kind_opt == 5) {
        // column blocks: the per-block schedules are built separately; the
        // parent keeps 64-row tiles for sizing the grid of its start/finish kernels
        S.kind = kTileColBlocked;
        S.ntiles = (m + kWaveSize - 1) / kWaveSize;
        return;
    }
    auto len = [&](int32_t i) -> int64_t { return M.h_rp[i + 1] - M.h_rp[i]; };
    int64_t maxlen = 0;
#pragma omp parallel for reduction(max : maxlen) schedule(static)
    for (int32_t i = 0; i < m; ++i) maxlen = std::max<int64_t>(maxlen, len(i));
    const double mean = (double)M.h_rp[m] / (double)m;
    if (kind_opt == 0 && !skip_empty) {
        // scattered columns over a vector of at least two blocks: column blocks
        int64_t far = 0;
        int32_t ncols = 0;
#pragma omp parallel for reduction(+ : far) reduction(max : ncols) schedule(static)
        for (int32_t i = 0; i < m; ++i)
            for (int32_t k = M.h_rp[i]; k < M.h_rp[i + 1]; ++k) {
                const int64_t d = (int64_t)M.h_ci[k] - (M.pad_col_base + i);
                far += (d > kColBlockCols || d < -kColBlockCols);
                ncols = std::max(ncols, M.h_ci[k] + 1);
            }
        if (ncols >= 2 * kColBlockCols && 2 * far > M.nnz) {
            S.kind = kTileColBlocked;
            S.ntiles = (m + kWaveSize - 1) / kWaveSize;
            return;
        }
    }
    if (kind_opt == 4 || kind_opt == 3 || kind_opt == 7 || (kind_opt == 0 && maxlen <= 64)) {
        const int32_t nt = (m + kWaveSize - 1) / kWaveSize;
        int64_t slots = 0;
        int maxw = 0;
#pragma omp parallel for reduction(+ : slots) reduction(max : maxw) schedule(static)
        for (int32_t t = 0; t < nt; ++t) {
            int64_t w = 0;
            for (int32_t i = t * kWaveSize; i < std::min(m, (t + 1) * kWaveSize); ++i) w = std::max(w, len(i));
            w = std::max<int64_t>(w, 1);
            slots += w * kWaveSize;
            maxw = std::max<int>(maxw, (int)w);
        }
        if (maxlen <= 64 && slots < INT32_MAX && (kind_opt >= 3 || slots <= M.nnz + M.nnz / 4)) {
            S.kind = (kind_opt == 4 || kind_opt == 0) && maxlen <= kSliceMaxWidth ? kTileSlicedDict
                                                                                : kTileSliced;
            S.nbins = 1;
            S.bins[0] = Bin{std::max(1, maxw), 0, m, 0};
            S.ntiles = nt;
            return;
        }
    }
    // stream tiles on request, and automatically for larger matrices of short
    // rows that the slices do not take (irregular lengths): measured on
    // random-column SPD matrices, stream tiles beat the vector bins by 9-24%
    // at n >= 300K with mean rows <= 64 and at n >= 200K with mean rows
    // <= 32, and lost 3-17% on smaller or longer-row matrices
    const bool auto_stream = kind_opt == 0 && !skip_empty &&
                             ((mean <= 64.0 && m >= 262144) || (mean <= 32.0 && m >= 131072));
    if ((kind_opt == 2 || auto_stream) && tiles_out && stream_tiles(M.h_rp.data(), m, *tiles_out)) {
        S.kind = kTileStream;   // the caller uploads the tiles (set_stream_tiles)
        return;
    }
    if (!skip_empty && maxlen <= 64 && (double)maxlen <= 2.0 * mean + 1.0) {
        const int L = lanes_for_length(maxlen);
        S.nbins = 1;
        S.bins[0] = Bin{L, 0, m, 0};
        S.ntiles = (m + rows_per_wave_tile(L) - 1) / rows_per_wave_tile(L);
        return;
    }
    static const int classes[7] = {1, 2, 4, 8, 16, 32, 64};
    std::vector<std::vector<int32_t>> lists(7);
    std::vector<int32_t> huge;
    for (int32_t i = 0; i < m; ++i) {
        const int64_t l = len(i);
        if (l == 0 && skip_empty) continue;
        if (l > kHugeRow) {
            huge.push_back(i);
            continue;
        }
        const int L = lanes_for_length(l);
        int c = 0;
        while (classes[c] != L) ++c;
        lists[c].push_back(i);
    }
    S.identity = 0;
    int nb = 0, tile = 0, pos = 0;
    for (int c = 0; c < 7; ++c) {
        if (lists[c].empty()) continue;
        const int cnt = (int)lists[c].size();
        S.bins[nb] = Bin{classes[c], pos, cnt, tile};
        tile += (cnt + rows_per_wave_tile(classes[c]) - 1) / rows_per_wave_tile(classes[c]);
        rows_out.insert(rows_out.end(), lists[c].begin(), lists[c].end());
        pos += cnt;
        ++nb;
    }
    S.nbins = nb;
    S.ntiles = tile;
    S.huge_first = pos;
    S.huge_count = (int32_t)huge.size();
    rows_out.insert(rows_out.end(), huge.begin(), huge.end());
}

// Slot-major copy in slices of 64 rows padded to the slice's longest row
// (at least one slot, so every load stays inside the allocation).  Padding
// slots gather the row's own entry of the vector and are never summed.
int build_sliced(DevMatrix &M, bool with_cols) {
    if (M.d_sell_off && (M.d_sell_ci || !with_cols)) return CG_OK;
    const int32_t m = M.m, nt = M.sched.ntiles;
    std::vector<int32_t> off;
    slice_offsets(M, nt, off);
    const size_t slots = (size_t)off[nt] ? (size_t)off[nt] : 1;
    const bool first = !M.d_sell_off;
    const bool host_vals = !M.h_val.empty();
    std::vector<int32_t> sci(with_cols ? slots : 0, 0);
    std::vector<double> sval(first && host_vals ? slots : 0, 0.0);
    // row lengths for the two-rows-per-lane tiles (rows up to 255 entries;
    // those tiles take slices of at most kSliceMaxWidth slots)
    std::vector<uint8_t> slen(with_cols ? (size_t)nt * kWaveSize : 0, 0);
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        const int32_t w = (off[t + 1] - off[t]) / kWaveSize;
        for (int32_t l = 0; l < kWaveSize; ++l) {
            const int32_t i = t * kWaveSize + l;
            const int32_t b = i < m ? M.h_rp[i] : 0;
            const int32_t len = i < m ? M.h_rp[i + 1] - M.h_rp[i] : 0;
            const int32_t pad_col = i < m ? M.pad_col_base + i : M.pad_col_base;
            if (with_cols) slen[(size_t)i] = (uint8_t)std::min(len, 255);
            for (int32_t j = 0; j < w; ++j) {
                const size_t k = (size_t)off[t] + (size_t)j * kWaveSize + l;
                if (with_cols) sci[k] = j < len ? M.h_ci[b + j] : pad_col;
                if (!sval.empty()) sval[k] = j < len ? M.h_val[b + j] : 0.0;
            }
        }
    }
    hipError_t e = hipSuccess;
    if (first) {
        e = dmalloc(&M.d_sell_off, off.size());
        if (e == hipSuccess) e = dmalloc(&M.d_sell_val, slots);
        if (e == hipSuccess)
            e = hipMemcpy(M.d_sell_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice);
        // values from the host copy, or zero until the owner writes them on the device
        if (e == hipSuccess)
            e = host_vals ? hipMemcpy(M.d_sell_val, sval.data(), sizeof(double) * slots, hipMemcpyHostToDevice)
                          : hipMemset(M.d_sell_val, 0, sizeof(double) * slots);
        M.sell_slots = slots;
    }
    if (e == hipSuccess && with_cols) {
        e = dmalloc(&M.d_sell_ci, slots);
        if (e == hipSuccess)
            e = hipMemcpy(M.d_sell_ci, sci.data(), sizeof(int32_t) * slots, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = dmalloc(&M.d_sell_len, slen.size());
        if (e == hipSuccess) e = hipMemcpy(M.d_sell_len, slen.data(), slen.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_sliced(M);
        return fail(CG_ENOMEM, "sliced layout upload failed: %s", hipGetErrorString(e));
    }
    return CG_OK;
}

// Gap-coded columns of the sliced layout (see sell_lenx / sell_gap): built
// when every code fits (rows of at most 15 entries, consecutive columns at
// most 2^16 apart, first columns within 2^19 of the row's own index); *fits
// says whether they apply.  An empty row, and a padding row of the last
// slice, starts at the block's last row, a column every lane may gather.
int build_gaps(DevMatrix &M, bool *fits) {
    *fits = false;
    if (M.gap_state < 0) return CG_OK;
    if (M.gap_state > 0) {
        *fits = true;
        return CG_OK;
    }
    const int32_t m = M.m, nt = M.sched.ntiles;
    // offset of row i's first column from its global index
    auto first_off = [&](int32_t i) -> int64_t {
        const int64_t own = (int64_t)M.pad_col_base + i;
        if (i < m && M.h_rp[i + 1] > M.h_rp[i]) return (int64_t)M.h_ci[M.h_rp[i]] - own;
        return (int64_t)M.pad_col_base + std::max(m - 1, 0) - own;
    };
    int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
    for (int32_t i = 0; i < m; ++i) {
        const int64_t o = first_off(i);
        bad |= M.h_rp[i + 1] - M.h_rp[i] > 15 || o < -(1 << 19) || o >= (1 << 19);
        for (int32_t k = M.h_rp[i] + 1; k < M.h_rp[i + 1]; ++k) {
            const int64_t d = (int64_t)M.h_ci[k] - (int64_t)M.h_ci[k - 1];
            bad |= d < 1 || d > 0x10000;
        }
    }
    if (bad) {
        M.gap_state = -1;
        return CG_OK;
    }
    std::vector<int32_t> off;
    slice_offsets(M, nt, off);
    const size_t slots = (size_t)off[nt] ? (size_t)off[nt] : 1;
    std::vector<uint16_t> code(slots, 0);
    std::vector<uint8_t> lenx((size_t)nt * kWaveSize, 0);
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < nt; ++t) {
        const int32_t w = (off[t + 1] - off[t]) / kWaveSize;
        for (int32_t l = 0; l < kWaveSize; ++l) {
            const int32_t i = t * kWaveSize + l;
            const int32_t b = i < m ? M.h_rp[i] : 0;
            const int32_t len = i < m ? M.h_rp[i + 1] - M.h_rp[i] : 0;
            const uint32_t o = (uint32_t)first_off(i) & 0xFFFFFu;   // 20-bit two's complement
            lenx[(size_t)i] = (uint8_t)(len | ((o >> 16) << 4));
            code[(size_t)off[t] + l] = (uint16_t)(o & 0xFFFFu);
            for (int32_t j = 1; j < std::min(w, len); ++j)
                code[(size_t)off[t] + (size_t)j * kWaveSize + l] = (uint16_t)(M.h_ci[b + j] - M.h_ci[b + j - 1] - 1);
        }
    }
    hipError_t e = dmalloc(&M.d_sell_lenx, lenx.size() ? lenx.size() : 1);
    if (e == hipSuccess) e = dmalloc(&M.d_sell_gap, code.size());
    if (e == hipSuccess && !lenx.empty())
        e = hipMemcpy(M.d_sell_lenx, lenx.data(), lenx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.d_sell_gap, code.data(), sizeof(uint16_t) * code.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(M.d_sell_lenx);
        (void)hipFree(M.d_sell_gap);
        M.d_sell_lenx = nullptr;
        M.d_sell_gap = nullptr;
        return fail(CG_ENOMEM, "gap-coded columns upload failed: %s", hipGetErrorString(e));
    }
    M.gap_state = 1;
    *fits = true;
    return CG_OK;
}

// Column blocks of block_cols columns: block b holds, for every row, the
// row's entries with columns in [b block_cols, (b+1) block_cols) (a
// contiguous sub-range, columns being sorted), uploaded as its own CSR with
// a vector-bin schedule over its non-empty rows.
int build_blocks(DevMatrix &M, int32_t block_cols, int cus, int grid_cap, bool need_f32) {
    if (M.cb && M.block_cols == block_cols) return CG_OK;
    free_blocks(M);
    M.block_cols = block_cols;
    const int32_t m = M.m;
    int32_t ncols = 0;
    for (int32_t c : M.h_ci) ncols = std::max(ncols, c + 1);
    const int32_t nb = std::max(1, (ncols + block_cols - 1) / block_cols);
    if (nb > kMaxColBlocks) return fail(CG_EINVAL, "%d column blocks exceed %d", nb, kMaxColBlocks);
    ColBlocks *cb = new (std::nothrow) ColBlocks();
    if (!cb) return fail(CG_ENOMEM, "out of host memory");
    M.cb = cb;
    cb->nb = nb;
    M.blocks.resize(nb);
    std::vector<int32_t> cur(M.h_rp.begin(), M.h_rp.end() - 1);   // per-row cursor
    std::vector<int32_t> rp, ci;
    std::vector<double> va;
    for (int32_t b = 0; b < nb; ++b) {
        const int64_t lim = (int64_t)(b + 1) * block_cols;
        try {
            rp.assign((size_t)m + 1, 0);
            ci.clear();
            va.clear();
            for (int32_t i = 0; i < m; ++i) {
                int32_t k = cur[i];
                while (k < M.h_rp[i + 1] && M.h_ci[k] < lim) {
                    ci.push_back(M.h_ci[k]);
                    va.push_back(M.h_val[k]);
                    ++k;
                }
                cur[i] = k;
                rp[i + 1] = (int32_t)ci.size();
            }
        } catch (...) {
            return fail(CG_ENOMEM, "out of host memory");
        }
        DevMatrix &B = M.blocks[b];
        int rc = dm_upload(B, m, rp.data(), ci.data(), va.data(), M.pad_col_base);
        if (rc) return rc;
        // Natural row order, L lanes per row with L the power of two covering
        // half the block's mean row length, so each pass reads the row
        // pointers and reads and writes q in whole lines; bins by row length
        // (the row list) scattered those accesses, about 2.5x the compulsory
        // L2 misses per pass at n = 2M.  A block with a row longer than
        // kHugeRow keeps the bins (such rows take a whole workgroup there).
        std::vector<int32_t> rows;
        int64_t bmax = 0;
        for (int32_t i = 0; i < m; ++i) bmax = std::max<int64_t>(bmax, rp[i + 1] - rp[i]);
        // Adaptive stream tiles when every row fits one: every lane keeps 8
        // gathers in flight and the entries move in 16-byte loads.
        std::vector<int32_t> tiles;
        if (stream_tiles(rp.data(), m, tiles)) {
            rc = set_stream_tiles(B, B.sched, tiles);
            if (rc) return rc;
        } else if (m > 0 && bmax <= kHugeRow) {
            const int L = lanes_for_length(((int64_t)rp[m] + 2ll * m - 1) / (2ll * m));
            Schedule &S = B.sched;
            S = Schedule{};
            S.identity = 1;
            S.nbins = 1;
            S.bins[0] = Bin{L, 0, m, 0};
            S.ntiles = (m + rows_per_wave_tile(L) - 1) / rows_per_wave_tile(L);
        } else {
            build_schedule(B, 1, B.sched, rows, true);
        }
        if (!rows.empty()) {
            const hipError_t e = hipMemcpy(B.d_rows, rows.data(), sizeof(int32_t) * rows.size(),
                                           hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(CG_EDEVICE, "row list upload failed: %s", hipGetErrorString(e));
        }
        if (need_f32) {
            rc = dm_ensure_f32(B);
            if (rc) return rc;
        }
        const int waves = B.sched.ntiles + B.sched.huge_count * (kBlock / kWaveSize);
        const int g = std::min(cus * 8, ((waves / (kBlock / kWaveSize) + 8) / 8) * 8);
        B.grid = std::max(8, (std::min(g, grid_cap) / 8) * 8);
        cb->dev[b] = B.dev();
        cb->sched[b] = B.sched;
        cb->grid[b] = B.grid;
    }
    return CG_OK;
}

}  // namespace

int dm_upload(DevMatrix &M, int32_t m, const int32_t *rp, const int32_t *ci, const double *val,
              int32_t pad_col_base) {
    dm_free(M);
    M.m = m;
    M.pad_col_base = pad_col_base;
    const int32_t base = m > 0 ? rp[0] : 0;
    M.nnz = m > 0 ? (int64_t)rp[m] - base : 0;
    try {
        M.h_rp.resize((size_t)m + 1);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i <= m; ++i) M.h_rp[i] = m > 0 ? rp[i] - base : 0;
        M.h_ci.resize((size_t)M.nnz);
        par_copy(M.h_ci.data(), ci + base, (size_t)M.nnz);
        M.h_val.clear();
        if (val) {
            M.h_val.resize((size_t)M.nnz);
            par_copy(M.h_val.data(), val + base, (size_t)M.nnz);
        }
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory");
    }
    hipError_t e = dmalloc(&M.d_rp, (size_t)m + 1);
    // padded: 16-byte stream-tile loads may run up to kStreamNnz entries past the end
    if (e == hipSuccess) e = dmalloc(&M.d_ci, (size_t)M.nnz + kStreamNnz);
    if (e == hipSuccess) e = dmalloc(&M.d_val, (size_t)M.nnz + kStreamNnz);
    if (e == hipSuccess) e = dmalloc(&M.d_rows, (size_t)m);
    if (e == hipSuccess)
        e = hipMemcpy(M.d_rp, M.h_rp.data(), sizeof(int32_t) * ((size_t)m + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && M.nnz)
        e = hipMemcpy(M.d_ci, M.h_ci.data(), sizeof(int32_t) * M.nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess && M.nnz) {
        if (val) e = hipMemcpy(M.d_val, M.h_val.data(), sizeof(double) * M.nnz, hipMemcpyHostToDevice);
        else e = hipMemset(M.d_val, 0, sizeof(double) * M.nnz);
    }
    // padding (and entry 0 of an empty block): column 0, value 0
    if (e == hipSuccess) e = hipMemset(M.d_ci + M.nnz, 0, sizeof(int32_t) * kStreamNnz);
    if (e == hipSuccess) e = hipMemset(M.d_val + M.nnz, 0, sizeof(double) * kStreamNnz);
    if (e != hipSuccess) {
        dm_free(M);
        return fail(CG_ENOMEM, "matrix upload failed: %s", hipGetErrorString(e));
    }
    return CG_OK;
}

int dm_ensure_f32(DevMatrix &M) {
    hipError_t e = hipSuccess;
    if (!M.d_val32) {
        const size_t nv = (size_t)M.nnz + kStreamNnz;
        std::vector<float> v32(nv, 0.0f);
        std::vector<double> dv;
        const double *hv = M.h_val.data();
        if (M.h_val.empty() && M.nnz) {   // values live on the device only
            dv.resize((size_t)M.nnz);
            e = hipMemcpy(dv.data(), M.d_val, sizeof(double) * dv.size(), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail(CG_EDEVICE, "float32 copies: %s", hipGetErrorString(e));
            hv = dv.data();
        }
        for (int64_t k = 0; k < M.nnz; ++k) v32[k] = (float)hv[k];
        e = dmalloc(&M.d_val32, nv);
        if (e == hipSuccess) e = hipMemcpy(M.d_val32, v32.data(), sizeof(float) * nv, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && M.d_sell_val && !M.d_sell_val32) {
        std::vector<double> sv(M.sell_slots);
        e = hipMemcpy(sv.data(), M.d_sell_val, sizeof(double) * sv.size(), hipMemcpyDeviceToHost);
        std::vector<float> sv32(sv.size());
        for (size_t k = 0; k < sv.size(); ++k) sv32[k] = (float)sv[k];
        if (e == hipSuccess) e = dmalloc(&M.d_sell_val32, sv32.size());
        if (e == hipSuccess)
            e = hipMemcpy(M.d_sell_val32, sv32.data(), sizeof(float) * sv32.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return fail(CG_ENOMEM, "float32 copies: %s", hipGetErrorString(e));
    return CG_OK;
}

int dm_schedule(DevMatrix &M, int kind_opt, int grid_opt, int cus, int grid_cap, bool need_f32,
                int32_t block_cols) {
    std::vector<int32_t> rows;
    // stencil slices (6) start from the dictionary choice and are upgraded below
    std::vector<int32_t> tiles;
    build_schedule(M, kind_opt == 6 ? 4 : kind_opt, M.sched, rows, false, &tiles);
    if (M.sched.kind == kTileStream) {
        const int rc = set_stream_tiles(M, M.sched, tiles);
        if (rc) return rc;
    }
    if (M.sched.kind == kTileColBlocked) {
        const int32_t bc = block_cols > 0 ? block_cols : kColBlockCols;
        if (M.cb && M.block_cols == bc && need_f32)
            for (int b = 0; b < M.cb->nb; ++b) {
                const int rc = dm_ensure_f32(M.blocks[b]);
                if (rc) return rc;
                M.cb->dev[b] = M.blocks[b].dev();
            }
        const int rc = build_blocks(M, bc, cus, grid_cap, need_f32);
        if (rc) return rc;
    }
    // stencil slices where every slice has at most 8 distinct column offsets
    // (float64); else the dictionary or plain slices.  Without host values
    // the slots hold zeros until the owner writes them on the device.
    if ((kind_opt == 0 || kind_opt == 6) && !need_f32 &&
        (M.sched.kind == kTileSlicedDict || M.sched.kind == kTileSliced) && M.sched.bins[0].lanes <= kSliceMaxWidth) {
        bool fits = false;
        const int rc = build_stencil(M, &fits);
        if (rc) return rc;
        if (fits) M.sched.kind = kTileStencil;
    }
    if (M.sched.kind == kTileSlicedDict && !M.d_sell_idx) {
        std::vector<int32_t> dict;
        std::vector<uint32_t> idx;
        bool ok = false;
        try {
            ok = build_dict(M, dict, idx);
        } catch (...) {
            return fail(CG_ENOMEM, "out of host memory");
        }
        if (ok) {
            hipError_t e = dmalloc(&M.d_sell_dict, dict.size());
            if (e == hipSuccess) e = dmalloc(&M.d_sell_idx, idx.size());
            if (e == hipSuccess)
                e = hipMemcpy(M.d_sell_dict, dict.data(), sizeof(int32_t) * dict.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(M.d_sell_idx, idx.data(), sizeof(uint32_t) * idx.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(CG_ENOMEM, "dictionary layout upload failed: %s", hipGetErrorString(e));
        } else {
            M.sched.kind = kTileSliced;   // too many distinct offsets: plain slices
        }
    }
    if (M.sched.kind == kTileSliced || M.sched.kind == kTileSlicedDict) {
        // the dictionary tiles read no columns from the sliced copy
        const int rc = build_sliced(M, M.sched.kind == kTileSliced);
        if (rc) return rc;
    }
    // gap-coded columns for the paired float64 tiles where the pattern allows
    M.use_gap = false;
    if (M.sched.kind == kTileSliced && (kind_opt == 0 || kind_opt == 7) &&
        M.sched.bins[0].lanes <= kSliceMaxWidth) {
        bool fits = false;
        const int rc = build_gaps(M, &fits);
        if (rc) return rc;
        M.use_gap = fits;
    }
    if (M.sched.kind == kTileStencil)
        M.sched.stream_nt = (int64_t)M.st_slots * (int64_t)sizeof(double) + (int64_t)M.m > kStreamNtBytes;
    else if (M.sched.kind == kTileSliced)
        M.sched.stream_nt = (int64_t)M.sell_slots * (int64_t)(sizeof(double) + (M.use_gap ? 2 : 4)) + M.m >
                            kStreamNtBytes;
    else
        M.sched.stream_nt = M.sched.kind == kTileSlicedDict &&
                            (int64_t)M.sell_slots * (int64_t)sizeof(double) + 4ll * M.m > kStreamNtBytes;
    if (!rows.empty()) {
        const hipError_t e = hipMemcpy(M.d_rows, rows.data(), sizeof(int32_t) * rows.size(),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(CG_EDEVICE, "row list upload failed: %s", hipGetErrorString(e));
    }
    if (need_f32) {
        const int rc = dm_ensure_f32(M);
        if (rc) return rc;
    }
    const int waves_needed = M.sched.ntiles + M.sched.huge_count * (kBlock / kWaveSize);
    const int auto_grid = ((waves_needed / (kBlock / kWaveSize) + 8) / 8) * 8;
    int g = grid_opt > 0 ? grid_opt : std::min(cus * 8, auto_grid);
    g = std::min(g, grid_cap);
    M.grid = std::max(8, (g / 8) * 8);
    return CG_OK;
}

void dm_free(DevMatrix &M) {
    free_blocks(M);
    (void)hipFree(M.d_tile_row);
    M.d_tile_row = nullptr;
    (void)hipFree(M.d_rp);
    (void)hipFree(M.d_ci);
    (void)hipFree(M.d_rows);
    (void)hipFree(M.d_val);
    (void)hipFree(M.d_val32);
    free_sliced(M);
    M.d_rp = M.d_ci = M.d_rows = nullptr;
    M.d_val = nullptr;
    M.d_val32 = nullptr;
    M.m = 0;
    M.nnz = 0;
    M.h_rp.clear();
    M.h_ci.clear();
    M.h_val.clear();
}

}  // namespace cgmi
