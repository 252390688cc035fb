"""The library's host table code (FP64 offsets, validity and z shifts) built
with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only,
every finding fatal) and run on every workload's grid spec and on invalid
specs; the tables it writes must equal the oracle's bit for bit."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1310_7556_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "host_tables")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC,
           os.path.join(CSRC, "tables.cpp"), os.path.join(ROOT, "tests", "host_tables_main.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return out


def run(driver, tmp_path, spec):
    from paper_1310_7556_amd import hough
    s = hough.make_spec(spec)
    src, dst = tmp_path / "spec.bin", tmp_path / "tables.bin"
    src.write_bytes(bytes(memoryview(s)))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, str(src), str(dst)], capture_output=True, text=True, env=env, timeout=120)
    return r, dst


@pytest.mark.parametrize("name", list(synth.CONFIGS))
def test_sanitized_host_tables_equal_the_oracle(driver, tmp_path, name):
    spec = synth.grid_spec(name)
    r, dst = run(driver, tmp_path, spec)
    assert r.returncode == 0, r.stderr[-2000:]
    tab = oracle.Tables(spec)
    raw = dst.read_bytes()
    nO = tab.O.size
    O = np.frombuffer(raw, np.uint32, nO)
    V = np.frombuffer(raw, np.uint8, nO, offset=4 * nO)
    Z = np.frombuffer(raw, np.int32, offset=5 * nO)
    np.testing.assert_array_equal(O, tab.O.reshape(-1))
    np.testing.assert_array_equal(V, tab.V.reshape(-1))
    np.testing.assert_array_equal(Z, tab.Z.reshape(-1))


@pytest.mark.parametrize("kw", [dict(n_phi=3), dict(n_layers=0), dict(n_layers=17), dict(n_qpt=0),
                                dict(z0_lo_um=5, z0_hi_um=5), dict(n_cot=0)])
def test_sanitized_host_code_rejects_invalid_specs(driver, tmp_path, kw):
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    spec.update(kw)
    if kw.get("n_layers") == 0:
        spec["layer_r_mm"] = []
    r, _ = run(driver, tmp_path, spec)
    assert r.returncode == 3, (r.returncode, r.stderr[-2000:])


@pytest.fixture(scope="module")
def rank_driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan_rank") / "host_rank_tables")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC,
           os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "rank_tables.cpp"),
           os.path.join(ROOT, "tests", "host_rank_tables_main.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return out


RANK_TABLE_SPECS = [dict(), dict(n_qpt=300, n_phi=256), dict(n_qpt=1024, n_phi=512, n_layers=13,
                    layer_r_mm=[40.0 + 63.0 * i for i in range(13)]),
                    dict(n_qpt=64, n_phi=256, n_d0=8, d0_lo_mm=-120.0, d0_hi_mm=120.0), dict(n_qpt=1, n_phi=1024)]


@pytest.mark.parametrize("kw", RANK_TABLE_SPECS)
def test_sanitized_rank_tables_equal_brute_force(rank_driver, tmp_path, kw):
    """The rank vote's static tables (per tile: sorted fine offsets, their
    search index, each row's J, validity and rank; per event: all rows'
    sorted offsets, their 16-bit index and each tile's counts) against plain
    counts over the rows' fine offsets, under ASan and UBSan: the c4 grid,
    a ragged last tile, 13 layers and 1024 rows, a displaced grid with
    unreachable rows and 512 rows, and a single row."""
    from paper_1310_7556_amd import hough
    spec = synth.grid_spec("c4_batch_4096")
    spec.update(kw)
    s = hough.make_spec(spec)
    src = tmp_path / "spec.bin"
    src.write_bytes(bytes(memoryview(s)))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([rank_driver, str(src)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
    assert r.stdout.startswith("ok ") and int(r.stdout.split()[1]) > 1000
