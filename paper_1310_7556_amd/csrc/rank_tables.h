// Host side of the rank form of the vote (Section 4, first step): the
// static tables built once per context from the azimuth offsets, and their
// layout, shared by the builder (rank_tables.cpp, plain C++) and the
// kernels (k_vote_rank.hip).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/hough.h"

namespace hough {

// Rank form of the vote: rows per tile (ranks fit a byte), workgroup size
// and the stride of a tile's sorted fine offsets per layer: 128 values +
// padding, then a search index (kRankIndexAt: the smallest and largest
// value, a shift, the count, and 257 byte counts of the values below each of
// 256 equal parts of [smallest, largest]).
constexpr uint32_t kRankTileRows = 128;
constexpr uint32_t kRankThreads = 512;
constexpr uint32_t kRankIndexAt = 132;
constexpr uint32_t kRankSortStride = kRankIndexAt + 4 + 68;

// Whole-event items rank each entry's interval once against all rows of its
// layer.  Per layer, the fine offsets of every row sorted (from
// kRankGlobAt), after a header (the smallest and largest value, a shift, the
// count) and 257 16-bit counts of the values below each of 256 equal parts
// of [smallest, largest]; per (tile, layer), the bytes cnt[k] = how many of
// the first k sorted values belong to the tile, k = 0..rows.  Both follow
// the per-tile tables in the same buffer; only grids of at most
// kRankEventRowsMax rows have them.
constexpr uint32_t kRankGlobAt = 4 + 129;
constexpr uint32_t kRankEventRowsMax = 1024;
struct RankGlobLayout {
    size_t glob_at, cnt_at, size;   // in 32-bit words from the buffer's start
    uint32_t gstride, cstride;      // per layer
};
inline RankGlobLayout rank_glob_layout(uint32_t rows, uint32_t L)
{
    RankGlobLayout y;
    const size_t n_tiles = (rows + kRankTileRows - 1) / kRankTileRows;
    y.gstride = (kRankGlobAt + rows + 3) & ~3u;
    y.cstride = (rows + 1 + 3) / 4;
    y.glob_at = n_tiles * L * kRankSortStride;
    y.cnt_at = y.glob_at + size_t(L) * y.gstride;
    y.size = rows <= kRankEventRowsMax ? y.cnt_at + n_tiles * L * y.cstride : y.glob_at;
    return y;
}

// Static per-row words of the rank tables: [0, 16) J | unreachable << 31 per
// layer, [16, 32) (0x80 + rank) in every byte per layer.
constexpr uint32_t kRankInvalid = 0x80000000u;

// The rank form applies to this spec (n_phi 256, 512 or 1024, at most 16
// layers).
bool rank_vote_form(const hough_grid_spec &g);
// From the offsets O and validity V ([l][r], rows r): the per-row words
// info ([rows][32]) and the sorted-offset, index and count tables (the
// per-tile tables, then RankGlobLayout's whole-event ones).
void build_rank_tables(const hough_grid_spec &g, uint32_t rows, uint32_t shift, const uint32_t *O, const uint8_t *V,
                       std::vector<uint32_t> &info, std::vector<uint32_t> &sorted);

}  // namespace hough
