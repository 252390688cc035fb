// The rank form's static tables (see rank_tables.h and k_vote_rank.hip).
#include "rank_tables.h"

#include <algorithm>
#include <utility>

namespace hough {

bool rank_vote_form(const hough_grid_spec &g)
{
    return (g.n_phi == 256 || g.n_phi == 512 || g.n_phi == 1024) && g.n_layers <= 16;
}

void build_rank_tables(const hough_grid_spec &g, uint32_t rows, uint32_t shift, const uint32_t *O, const uint8_t *V,
                       std::vector<uint32_t> &info, std::vector<uint32_t> &sorted)
{
    const uint32_t L = g.n_layers;
    const uint32_t wmask = (1u << shift) - 1u;
    const uint32_t n_tiles = (rows + kRankTileRows - 1) / kRankTileRows;
    const RankGlobLayout y = rank_glob_layout(rows, L);
    info.assign(size_t(rows) * 32, 0u);
    sorted.assign(y.size, 0xFFFFFFFFu);
    std::vector<uint32_t> f;
    for (uint32_t t = 0; t < n_tiles; ++t) {
        const uint32_t r0 = t * kRankTileRows, r1 = std::min(rows, r0 + kRankTileRows);
        for (uint32_t l = 0; l < L; ++l) {
            f.clear();
            for (uint32_t r = r0; r < r1; ++r) f.push_back(O[size_t(l) * rows + r] & wmask);
            std::sort(f.begin(), f.end());
            uint32_t *st = sorted.data() + (size_t(t) * L + l) * kRankSortStride;
            std::copy(f.begin(), f.end(), st);
            // the search index of these values (see rank_below)
            const uint32_t f0 = f.empty() ? 0u : f.front(), f1 = f.empty() ? 0u : f.back();
            uint32_t sh = 0;
            while (((f1 - f0) >> sh) > 255u) ++sh;
            st[kRankIndexAt] = f0;
            st[kRankIndexAt + 1] = f1;
            st[kRankIndexAt + 2] = sh;
            st[kRankIndexAt + 3] = uint32_t(f.size());
            uint8_t *ix = reinterpret_cast<uint8_t *>(st + kRankIndexAt + 4);
            for (uint32_t b = 0; b <= 256; ++b) {
                const uint64_t edge = uint64_t(f0) + (uint64_t(b) << sh);
                ix[b] = uint8_t(std::lower_bound(f.begin(), f.end(), edge,
                                                 [](uint32_t v, uint64_t e) { return uint64_t(v) < e; }) -
                                f.begin());
            }
            for (uint32_t r = r0; r < r1; ++r) {
                const uint32_t o = O[size_t(l) * rows + r];
                const uint32_t rank = uint32_t(std::lower_bound(f.begin(), f.end(), o & wmask) - f.begin());
                const uint32_t J = o >> shift;
                info[size_t(r) * 32 + l] = J | (V[size_t(l) * rows + r] ? 0u : kRankInvalid);
                info[size_t(r) * 32 + 16 + l] = (0x80u + rank) * 0x01010101u;
            }
        }
    }
    if (y.size == y.glob_at) return;                 // too many rows for whole-event items
    // per layer, every row's fine offset sorted with its tile, the search
    // index (see rank_all), and per tile the counts cnt[k] of its rows among
    // the first k sorted values
    std::vector<std::pair<uint32_t, uint32_t>> fa(rows);
    for (uint32_t l = 0; l < L; ++l) {
        for (uint32_t r = 0; r < rows; ++r) fa[r] = {O[size_t(l) * rows + r] & wmask, r / kRankTileRows};
        std::sort(fa.begin(), fa.end());
        uint32_t *gl = sorted.data() + y.glob_at + size_t(l) * y.gstride;
        for (uint32_t k = 0; k < rows; ++k) gl[kRankGlobAt + k] = fa[k].first;
        const uint32_t f0 = fa.front().first, f1 = fa.back().first;
        uint32_t sh = 0;
        while (((f1 - f0) >> sh) > 255u) ++sh;
        gl[0] = f0;
        gl[1] = f1;
        gl[2] = sh;
        gl[3] = rows;
        uint16_t *ix = reinterpret_cast<uint16_t *>(gl + 4);
        for (uint32_t b = 0; b <= 256; ++b) {
            const uint64_t edge = uint64_t(f0) + (uint64_t(b) << sh);
            uint32_t n = 0;
            while (n < rows && uint64_t(fa[n].first) < edge) ++n;
            ix[b] = uint16_t(n);
        }
        for (uint32_t t = 0; t < n_tiles; ++t) {
            uint8_t *cn = reinterpret_cast<uint8_t *>(sorted.data() + y.cnt_at + (size_t(t) * L + l) * y.cstride);
            std::fill(cn, cn + size_t(y.cstride) * 4, uint8_t(0));
            uint32_t run = 0;
            for (uint32_t k = 0; k < rows; ++k) {
                run += fa[k].second == t ? 1u : 0u;
                cn[k + 1] = uint8_t(run);
            }
        }
    }
}

}  // namespace hough
