// Test driver for a sanitizer build of the rank vote's host tables
// (rank_tables.cpp): reads a hough_grid_spec from a file, builds the azimuth
// offsets, then the rank tables, and checks every table against brute-force
// counts over the rows' fine offsets.  Prints the number of checks and
// exits 0; exit status 1 names the first mismatch, 3 an unusable spec.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rank_tables.h"
#include "tables.h"

using namespace hough;

static long checks = 0;

static bool fail(const char *what, unsigned l, unsigned t, unsigned long long x)
{
    std::printf("MISMATCH %s layer %u tile %u at %llu\n", what, l, t, x);
    return false;
}

// #{v in f : v < x} by a plain count
static unsigned below(const std::vector<unsigned> &f, unsigned long long x)
{
    unsigned n = 0;
    for (unsigned v : f) n += (unsigned long long)v < x ? 1u : 0u;
    return n;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    hough_grid_spec g;
    FILE *fp = std::fopen(argv[1], "rb");
    if (!fp || std::fread(&g, sizeof g, 1, fp) != 1) return 2;
    std::fclose(fp);
    if (!spec_valid(g) || !rank_vote_form(g)) return 3;
    const unsigned rows = g.n_d0 * g.n_qpt, L = g.n_layers;
    unsigned log2phi = 0;
    while ((1u << log2phi) < g.n_phi) ++log2phi;
    const unsigned shift = 32 - log2phi, wmask = (1u << shift) - 1u;
    std::vector<uint32_t> O(size_t(L) * rows);
    std::vector<uint8_t> V(O.size());
    build_offsets(g, O.data(), V.data());
    std::vector<uint32_t> info, sorted;
    build_rank_tables(g, rows, shift, O.data(), V.data(), info, sorted);
    const RankGlobLayout y = rank_glob_layout(rows, L);
    if (info.size() != size_t(rows) * 32 || sorted.size() != y.size) return fail("sizes", 0, 0, 0) ? 0 : 1;
    const unsigned n_tiles = (rows + kRankTileRows - 1) / kRankTileRows;
    for (unsigned l = 0; l < L; ++l) {
        std::vector<unsigned> all(rows);
        for (unsigned r = 0; r < rows; ++r) all[r] = O[size_t(l) * rows + r] & wmask;
        for (unsigned t = 0; t < n_tiles; ++t) {
            const unsigned r0 = t * kRankTileRows, r1 = std::min(rows, r0 + kRankTileRows);
            std::vector<unsigned> f(all.begin() + r0, all.begin() + r1);
            const uint32_t *st = sorted.data() + (size_t(t) * L + l) * kRankSortStride;
            std::vector<unsigned> s = f;
            std::sort(s.begin(), s.end());
            for (unsigned k = 0; k < s.size(); ++k, ++checks)
                if (st[k] != s[k]) return fail("tile sorted", l, t, k) ? 0 : 1;
            const unsigned f0 = st[kRankIndexAt], sh = st[kRankIndexAt + 2];
            if (f0 != s.front() || st[kRankIndexAt + 1] != s.back() || st[kRankIndexAt + 3] != s.size() ||
                ((s.back() - s.front()) >> sh) > 255u || (sh && ((s.back() - s.front()) >> (sh - 1)) <= 255u))
                return fail("tile header", l, t, 0) ? 0 : 1;
            const uint8_t *ix = reinterpret_cast<const uint8_t *>(st + kRankIndexAt + 4);
            for (unsigned b = 0; b <= 256; ++b, ++checks)
                if (ix[b] != below(f, (unsigned long long)f0 + ((unsigned long long)b << sh)))
                    return fail("tile index", l, t, b) ? 0 : 1;
            for (unsigned r = r0; r < r1; ++r, ++checks) {
                const uint32_t w = info[size_t(r) * 32 + l], R = info[size_t(r) * 32 + 16 + l];
                const uint32_t want = (O[size_t(l) * rows + r] >> shift) | (V[size_t(l) * rows + r] ? 0u : kRankInvalid);
                if (w != want || R != (0x80u + below(f, all[r])) * 0x01010101u) return fail("row words", l, t, r) ? 0 : 1;
            }
        }
        if (y.size == y.glob_at) continue;            // no whole-event tables past kRankEventRowsMax rows
        const uint32_t *gl = sorted.data() + y.glob_at + size_t(l) * y.gstride;
        std::vector<unsigned> s = all;
        std::sort(s.begin(), s.end());
        for (unsigned k = 0; k < rows; ++k, ++checks)
            if (gl[kRankGlobAt + k] != s[k]) return fail("all sorted", l, 0, k) ? 0 : 1;
        const unsigned f0 = gl[0], sh = gl[2];
        if (f0 != s.front() || gl[1] != s.back() || gl[3] != rows || ((s.back() - s.front()) >> sh) > 255u)
            return fail("all header", l, 0, 0) ? 0 : 1;
        const uint16_t *ix = reinterpret_cast<const uint16_t *>(gl + 4);
        for (unsigned b = 0; b <= 256; ++b, ++checks)
            if (ix[b] != below(all, (unsigned long long)f0 + ((unsigned long long)b << sh)))
                return fail("all index", l, 0, b) ? 0 : 1;
        // a tile's count at g(x) is the tile's rows below x, for x at every
        // offset, one past it and one before it
        for (unsigned t = 0; t < n_tiles; ++t) {
            const unsigned r0 = t * kRankTileRows, r1 = std::min(rows, r0 + kRankTileRows);
            std::vector<unsigned> f(all.begin() + r0, all.begin() + r1);
            const uint8_t *cn = reinterpret_cast<const uint8_t *>(sorted.data() + y.cnt_at + (size_t(t) * L + l) * y.cstride);
            for (unsigned q = 0; q < rows; ++q)
                for (int dx = -1; dx <= 1; ++dx, ++checks) {
                    const long long xx = (long long)all[q] + dx;
                    if (xx < 0) continue;
                    const unsigned gx = below(all, (unsigned long long)xx);
                    if (cn[gx] != below(f, (unsigned long long)xx)) return fail("tile counts", l, t, q) ? 0 : 1;
                }
        }
    }
    std::printf("ok %ld\n", checks);
    return 0;
}
