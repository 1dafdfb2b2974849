"""Parity of the modified (dipole-preserving) method of Sect. 7 / Appendix B
on the HIP path (flag NMC_MODIFIED, through the C ABI) with the CPU oracle's
solve_modified.

Tolerances as for the original method: FP64 <= 1e-12 pointwise relative,
FP32 <= 1e-5 relative to the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_06763_amd import inputs

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_06763_amd import nmc
    c = nmc.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def MOD():
    from paper_2301_06763_amd import nmc
    return nmc.NMC_MODIFIED


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    return np.abs(got - ref) / np.abs(ref)


def run(ctx, rho_np, h0, flags, dtype=torch.float64, G=1.0):
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to("cuda", dtype)
    phi = ctx.solve(rho, h0, G, flags)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy()


def tol_of(dtype):
    return F64_TOL if dtype == torch.float64 else F32_TOL


# (N, L): pyramid restriction where N is a multiple of 2^L, the cascaded one
# otherwise; N = 12, 20 have periods P above 2N (doubled period 2P above 4N);
# L = 2 has no carry, L >= 3 one carry launch, L = 6 at N = 16 two.
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,L", [(4, 2), (8, 2), (8, 3), (12, 3), (16, 4), (16, 6), (20, 3), (32, 4)])
def test_modified_random_levels(ctx, MOD, dtype, N, L):
    w = inputs.random_levels(N, L, seed=500 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0, G=0.7)
    got = run(ctx, rho, w.h0, MOD, dtype=dtype, G=0.7)
    assert np.max(rel_err(got, ref)) < tol_of(dtype), (N, L)


def test_modified_single_level_is_the_original(ctx, MOD):
    """One level has no doubled grid: the modified solve is the plain one."""
    w = inputs.random_levels(16, 1, seed=9)
    rho = w.rho.numpy()
    a = run(ctx, rho, w.h0, MOD)
    b = run(ctx, rho, w.h0, 0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modified_no_restrict(ctx, MOD, dtype):
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(16, 3, seed=12)
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0, restrict=False)
    got = run(ctx, rho, w.h0, MOD | nmc.NMC_NO_RESTRICT, dtype=dtype)
    assert np.max(rel_err(got, ref)) < tol_of(dtype)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("N,L", [(8, 3), (16, 4), (32, 3)])
def test_modified_fused_planes_match_separate(ctx, MOD, dtype, N, L):
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(N, L, seed=600 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0)
    fused = run(ctx, rho, w.h0, MOD, dtype=dtype)
    sep = run(ctx, rho, w.h0, MOD | nmc.NMC_NO_FUSED_PLANES, dtype=dtype)
    assert np.max(rel_err(fused, ref)) < tol_of(dtype)
    assert np.max(rel_err(sep, ref)) < tol_of(dtype)


def test_modified_fp32_uncompensated_within_tolerance(ctx, MOD):
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(32, 5, seed=21)
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0)
    got = run(ctx, rho, w.h0, MOD | nmc.NMC_F32_UNCOMPENSATED, dtype=torch.float32)
    assert np.max(rel_err(got, ref)) < F32_TOL


def test_modified_keeps_the_dipole_the_original_loses(ctx, MOD):
    """Sect. 7, Fig. 15: a +/- mass pair inside one coarse cell restricts to
    zero, so the original method's coarse level sees nothing of it; the
    modified method's coarse level sees the dipole field."""
    N, L, h0 = 16, 2, 1.0 / 16
    rho = np.zeros((L, N, N, N))
    c = N // 2
    rho[1, c, c, c - 2] = 1.0
    rho[1, c, c, c - 1] = -1.0
    orig = run(ctx, rho, h0, 0)
    mod = run(ctx, rho, h0, MOD)
    ref = oracle.solve_modified(rho, h0)
    assert np.max(np.abs(orig[0])) < 1e-18
    assert np.max(np.abs(mod[0])) > 1e-4  # the oracle's largest is 2.1e-4
    assert np.max(np.abs(mod - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modified_plummer32(ctx, MOD, dtype):
    w = inputs.plummer32()
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0)
    got = run(ctx, rho, w.h0, MOD, dtype=dtype)
    assert np.max(rel_err(got, ref)) < tol_of(dtype)


@pytest.fixture(scope="module")
def ellipsoid64_mod():
    w = inputs.ellipsoid64()
    rho = w.rho.numpy()
    return w, rho, oracle.solve_modified(rho, w.h0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modified_ellipsoid64(ctx, MOD, ellipsoid64_mod, dtype):
    w, rho, ref = ellipsoid64_mod
    got = run(ctx, rho, w.h0, MOD, dtype=dtype)
    e = rel_err(got, ref)
    for l in range(w.L):
        print(f"level {l}: max {e[l].max():.3e} rms {np.sqrt((e[l] ** 2).mean()):.3e}")
    assert np.max(e) < tol_of(dtype)


@pytest.fixture(scope="module")
def binary128_mod():
    w = inputs.binary128()
    rho = w.rho.numpy()
    return w, rho, oracle.solve_modified(rho, w.h0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modified_binary128_largest_n(ctx, MOD, binary128_mod, dtype):
    """N = 128, the largest N of the modified method (doubled period 512)."""
    w, rho, ref = binary128_mod
    got = run(ctx, rho, w.h0, MOD, dtype=dtype)
    assert np.max(rel_err(got, ref)) < tol_of(dtype)


def test_modified_rejects_n_above_128(ctx, MOD):
    from paper_2301_06763_amd import nmc
    rho = torch.zeros(2, 132, 132, 132, device="cuda", dtype=torch.float32)
    with pytest.raises(nmc.NmcError) as e:
        ctx.solve(rho, 1.0, 1.0, MOD)
    assert e.value.code == nmc.NMC_EUNSUPPORTED


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modified_batch_and_graph_equal_alone(ctx, MOD, dtype):
    """Modified and original requests in one batch (separate groups), and a
    captured-graph replay of a modified solve, equal their direct solves."""
    from paper_2301_06763_amd import nmc
    items = []
    for i, (N, L) in enumerate(((16, 3), (16, 4), (32, 3), (16, 3))):
        w = inputs.random_levels(N, L, seed=700 + i)
        items.append((w.rho.to("cuda", dtype), w.h0, 1.0, MOD if i % 2 == 0 else 0))
    alone = [ctx.solve(r, h, G, f | nmc.NMC_NO_GRAPH).clone() for r, h, G, f in items]
    batch = ctx.solve_batch(items)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a, b)
    r, h, G, f = items[0]
    out = torch.empty_like(r)
    for _ in range(3):  # the second and later calls replay a captured graph
        ctx.solve(r, h, G, f, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, alone[0])
