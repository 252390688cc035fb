// Test driver for a sanitizer build of the library's host table code
// (tables.cpp): reads a hough_grid_spec from a file, validates it, builds
// the azimuth offsets, validity flags and z shifts, and writes them as raw
// arrays (O uint32, V uint8, Z int32, in that order) to the output file.
// Exit status 3 when the spec is invalid.
#include <cstdio>
#include <vector>

#include "tables.h"

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    hough_grid_spec g;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f || std::fread(&g, sizeof g, 1, f) != 1) return 2;
    std::fclose(f);
    if (!hough::spec_valid(g)) return 3;
    const size_t rows = size_t(g.n_d0) * g.n_qpt, nov = size_t(g.n_layers) * rows;
    std::vector<uint32_t> O(nov);
    std::vector<uint8_t> V(nov);
    hough::build_offsets(g, O.data(), V.data());
    std::vector<int32_t> Z(g.n_z0 ? size_t(g.n_qpt) * g.n_layers * g.n_cot : 0);
    if (g.n_z0) hough::build_zshift(g, Z.data());
    f = std::fopen(argv[2], "wb");
    if (!f) return 2;
    if (!O.empty()) std::fwrite(O.data(), sizeof(uint32_t), O.size(), f);
    if (!V.empty()) std::fwrite(V.data(), 1, V.size(), f);
    if (!Z.empty()) std::fwrite(Z.data(), sizeof(int32_t), Z.size(), f);
    std::fclose(f);
    return 0;
}
