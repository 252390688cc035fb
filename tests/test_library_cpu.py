"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
symbol the header declares, validates specs like the oracle, builds tables
bit-identical to the oracle's independent ones, and its exact-division
helper matches integer division."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth
from paper_1310_7556_amd import hough

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hough.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hough_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hough.load_library()
    names = declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(hough.EXPORTED) == names


@pytest.mark.parametrize("name", list(synth.CONFIGS))
def test_tables_bit_identical_to_oracle(name):
    spec = synth.grid_spec(name)
    O, V, Z = hough.build_tables(spec)
    tab = oracle.Tables(spec)
    np.testing.assert_array_equal(O, tab.O)
    np.testing.assert_array_equal(V, tab.V)
    np.testing.assert_array_equal(Z, tab.Z)


def test_tables_displaced_unreachable_rows():
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    spec.update(n_d0=16, d0_lo_mm=-120.0, d0_hi_mm=120.0, n_qpt=32)
    O, V, _ = hough.build_tables(spec)
    tab = oracle.Tables(spec)
    np.testing.assert_array_equal(O, tab.O)
    np.testing.assert_array_equal(V, tab.V)
    assert not V.all() and V.any()


@pytest.mark.parametrize("mut", [
    {}, {"n_phi": 48}, {"n_phi": 1}, {"n_layers": 0}, {"n_qpt": 0},
    {"layer_r_mm": [40.0, 30.0] + [50.0 + i for i in range(8)]},
    {"n_z0": 256, "z0_lo_um": 5, "z0_hi_um": 5, "n_cot": 4},
    {"n_z0": 256, "z0_lo_um": -5, "z0_hi_um": 5, "n_cot": 0},
    {"n_z0": 256, "z0_lo_um": -5, "z0_hi_um": 5, "n_cot": 4, "n_d0": 2},
    {"n_z0": 256, "z0_lo_um": -5, "z0_hi_um": 5, "n_cot": 4},
])
def test_spec_validation_agrees_with_oracle(mut):
    spec = synth.grid_spec("c1_single_100trk")
    spec.update(mut)
    assert hough.check_spec(spec) == oracle.check_spec(spec)


def test_fastdiv_exact(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(r'''
#include "fastdiv.h"
#include <cstdio>
#include <random>
int main() {
    std::mt19937_64 rng(7);
    const uint32_t ds[] = {1u, 2u, 3u, 7u, 1562u, 400000u, 3125u, 65535u, 0x7FFFFFFFu,
                           0x80000000u, 0x80000001u, 0xFFFFFFFFu, 641u, 6700417u};
    for (uint32_t d : ds) {
        hough::FastDiv32 f = hough::make_fastdiv32(d);
        for (int i = 0; i < 200000; ++i) {
            uint32_t n = uint32_t(rng());
            if (i < 64) n = i; else if (i < 128) n = 0xFFFFFFFFu - (i - 64);
            else if (i < 192) n = d * uint32_t(i - 128);
            if (hough::fastdiv32(n, f) != n / d) { printf("bad %u %u\n", n, d); return 1; }
        }
    }
    for (int i = 0; i < 2000; ++i) {
        uint32_t d = uint32_t(rng()) | 1u;
        hough::FastDiv32 f = hough::make_fastdiv32(d);
        for (int j = 0; j < 500; ++j) {
            uint32_t n = uint32_t(rng());
            if (hough::fastdiv32(n, f) != n / d) { printf("bad %u %u\n", n, d); return 1; }
        }
    }
    return 0;
}
''')
    exe = tmp_path / "t"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_1310_7556_amd", "csrc"), str(src), "-o", str(exe)])
    subprocess.check_call([str(exe)])


def test_binmagic_exact(tmp_path):
    src = tmp_path / "b.cpp"
    src.write_text(r'''
#include "fastdiv.h"
#include <cstdio>
#include <random>
int main() {
    std::mt19937_64 rng(11);
    struct C { uint64_t span; uint32_t n; };
    const C cs[] = {{400000, 256}, {1, 1}, {3, 2}, {1000, 7}, {65535, 65535}, {4000000, 3},
                    {2000000001ull, 256}, {4294967295ull, 1}, {123457, 65535}};
    int tested = 0;
    for (int variant = 0; variant < 2; ++variant)
    for (C c : cs) {
        // the proven shift, and the smallest shift whose step ends check out
        hough::BinMagic b = variant ? hough::make_binmagic_min(c.span, c.n) : hough::make_binmagic(c.span, c.n);
        if (!b.ok) continue;
        if (variant && c.span == 400000 && b.s != 0) { printf("no shift-free magic for 400000/256\n"); return 3; }
        tested++;
        auto check = [&](uint64_t u) {
            const uint64_t want = (unsigned __int128)u * c.n / c.span;
            if (hough::binmagic_apply(uint32_t(u), b.m, b.s) != want) { printf("bad %llu %llu %u\n",
                (unsigned long long)u, (unsigned long long)c.span, c.n); return false; }
            return true;
        };
        if (c.span <= 5000000) { for (uint64_t u = 0; u < c.span; ++u) if (!check(u)) return 1; }
        else for (int i = 0; i < 2000000; ++i) if (!check(rng() % c.span)) return 1;
        for (uint64_t k = 0; k <= c.n; ++k) {          // bin edges and their neighbours
            uint64_t e = ((unsigned __int128)k * c.span + c.n - 1) / c.n;
            for (int64_t d = -1; d <= 1; ++d) { int64_t u = int64_t(e) + d; if (u >= 0 && uint64_t(u) < c.span && !check(u)) return 1; }
            if (k > 4096) break;
        }
    }
    return tested >= 8 ? 0 : 2;   // 400000/256, 3/2, 1000/7, 4e6/3 admit a 32-bit multiplier
}
''')
    exe = tmp_path / "b"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_1310_7556_amd", "csrc"), str(src), "-o", str(exe)])
    subprocess.check_call([str(exe)])


@pytest.mark.parametrize("cot", [(-1.2, 1.2), (1.2, -1.2), (0.5, 0.5)])
def test_z_shift_monotone_in_cot_bin(cot):
    """The rz kernel leaves a member out of a pass of cot bins when its z
    lies outside [min, max + span) of the pass's end values, which is exact
    only if Z[k][l][j] is monotone in j; it is (linear cot centres, a
    positive arc length, monotone rounding) for rising, falling and flat
    cot ranges."""
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    spec.update(cot_lo=cot[0], cot_hi=cot[1])
    _, _, Z = hough.build_tables(spec)
    d = np.diff(Z.astype(np.int64), axis=2)
    assert (d >= 0).all() or (d <= 0).all()
