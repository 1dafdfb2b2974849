"""Host-side checks of the C ABI (no GPU needed): the built library loads,
exports every function include/nmc.h declares, and its pure host entry
points (period, footprint, argument validation) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(nmc_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2301_06763_amd import nmc
    if not os.path.exists(nmc.LIB_PATH):
        pytest.fail("libnmc.so is not built (run __graft_entry__.build())")
    return nmc.lib()


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("nmc_create", "nmc_destroy", "nmc_solve", "nmc_solve_batch", "nmc_footprint_bytes",
                 "nmc_serve_submit", "nmc_serve_poll", "nmc_serve_tick", "nmc_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_period(lib):
    assert lib.nmc_period(4) == 8
    assert lib.nmc_period(12) == 32
    assert lib.nmc_period(32) == 64
    assert lib.nmc_period(64) == 128
    assert lib.nmc_period(256) == 512
    for bad in (0, 2, 6, 258, 260, -4):
        assert lib.nmc_period(bad) == 0


def test_footprint(lib):
    from paper_2301_06763_amd import nmc
    import torch
    # per full grid: A = N*N*(P/2) and B = N*P*(P/2) complex values; L full grids and
    # L-1 smaller child-region boxes
    N, L = 64, 5
    P = 128
    grid = (N * N * (P // 2) + N * P * (P // 2)) * 16
    fp = nmc.footprint_bytes(N, L, torch.float64)
    assert (2 * L - 1) * grid <= fp < (2 * L - 1) * grid * 1.05  # hole grids below N = 128
    N2, P2 = 128, 256
    grid2 = (N2 * N2 * (P2 // 2) + N2 * P2 * (P2 // 2)) * 16
    fp2 = nmc.footprint_bytes(N2, L, torch.float64)
    assert L * grid2 < fp2 < (2 * L - 1) * grid2  # smaller child-region boxes from N = 128
    assert nmc.footprint_bytes(N, L, torch.float32) < fp
    out = ctypes.c_size_t()
    assert lib.nmc_footprint_bytes(6, 2, 0, ctypes.byref(out)) == nmc.NMC_EINVAL
    assert lib.nmc_footprint_bytes(8, 0, 0, ctypes.byref(out)) == nmc.NMC_EINVAL
    assert lib.nmc_footprint_bytes(8, 17, 0, ctypes.byref(out)) == nmc.NMC_EINVAL
    assert lib.nmc_footprint_bytes(260, 2, 0, ctypes.byref(out)) == nmc.NMC_EUNSUPPORTED
    assert lib.nmc_footprint_bytes(8, 2, 7, ctypes.byref(out)) == nmc.NMC_EINVAL
    assert lib.nmc_footprint_bytes(8, 2, 0, None) == nmc.NMC_EINVAL


def test_footprint_of_the_modified_method(lib):
    from paper_2301_06763_amd import nmc
    import torch
    # L full-size grids (L-1 hole grids and the finest level) plus L-1 doubled
    # grids of period 2P: A = N^2 P (x half spectra) and B = N (2P) P
    # (N z rows) complex values each
    N, L, P = 32, 4, 64
    grid = (N * N * (P // 2) + N * P * (P // 2)) * 16
    dbl = (N * N * P + N * (2 * P) * P) * 16
    fp = nmc.footprint_bytes(N, L, torch.float64, nmc.NMC_MODIFIED)
    assert L * grid + (L - 1) * dbl <= fp < (L * grid + (L - 1) * dbl) * 1.05
    assert fp > nmc.footprint_bytes(N, L, torch.float64)
    assert nmc.footprint_bytes(N, L, torch.float64, 0) == nmc.footprint_bytes(N, L, torch.float64)
    out = ctypes.c_size_t()
    # doubled period 2P <= 1024: every N up to 256
    assert lib.nmc_footprint_bytes_flags(128, 3, 0, nmc.NMC_MODIFIED, ctypes.byref(out)) == nmc.NMC_OK
    assert lib.nmc_footprint_bytes_flags(256, 3, 0, nmc.NMC_MODIFIED, ctypes.byref(out)) == nmc.NMC_OK
    assert lib.nmc_footprint_bytes_flags(260, 3, 0, nmc.NMC_MODIFIED, ctypes.byref(out)) == nmc.NMC_EUNSUPPORTED
    assert lib.nmc_footprint_bytes_flags(132, 3, 0, 0, ctypes.byref(out)) == nmc.NMC_OK
    # the three-level scheme adds L-2 quadrupled grids of period 4P: A = N^2 (2P)
    # and B = N (4P) (2P) complex values; 4P <= 1024 needs N <= 128 from L = 3
    qdp = (N * N * 2 * P + N * 4 * P * 2 * P) * 16
    fp3 = nmc.footprint_bytes(N, L, torch.float64, nmc.NMC_MODIFIED3)
    assert fp + (L - 2) * qdp <= fp3 < (fp + (L - 2) * qdp) * 1.05
    assert lib.nmc_footprint_bytes_flags(128, 3, 0, nmc.NMC_MODIFIED3, ctypes.byref(out)) == nmc.NMC_OK
    assert lib.nmc_footprint_bytes_flags(132, 3, 0, nmc.NMC_MODIFIED3, ctypes.byref(out)) == nmc.NMC_EUNSUPPORTED
    assert lib.nmc_footprint_bytes_flags(256, 2, 0, nmc.NMC_MODIFIED3, ctypes.byref(out)) == nmc.NMC_OK


def test_null_context_is_rejected(lib):
    from paper_2301_06763_amd import nmc
    assert lib.nmc_solve(None, None, None, 8, 2, 0.1, 2, 1.0, 0, 0, None) == nmc.NMC_EINVAL
    assert lib.nmc_serve_tick(None, None) == nmc.NMC_EINVAL
    assert lib.nmc_last_error(None) == b"null context"
    lib.nmc_destroy(None)  # no-op


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2301_06763_amd import nmc
    h = ctypes.c_void_p()
    rc = lib.nmc_create(ctypes.byref(h), 0, 0)
    assert rc == nmc.NMC_EINVAL and not h.value


def test_pass_names(lib):
    names = [lib.nmc_pass_name(i).decode() for i in range(13)]
    assert names == ["restrict", "x", "y", "z", "inv_y", "inv_x_second", "carry", "inv_x_full",
                     "xy", "inv_yx_second", "inv_yx_full", "acceleration", "inv_x_doubled"]
    assert lib.nmc_pass_name(99) == b"?"


def test_scratch_size_matches_binding():
    from paper_2301_06763_amd import nmc
    src = open(HEADER).read()
    m = re.search(r"#define NMC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m, "NMC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == nmc.NMC_SCRATCH_BYTES


def test_noalloc_rejects_null_context(lib):
    assert lib.nmc_solve_noalloc(None, None, None, 8, 2, 1.0, 2, 1.0, 0, 0, None) == -1
