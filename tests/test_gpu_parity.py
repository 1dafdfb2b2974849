"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 path: pointwise relative error <= 1e-12 (the zero-padded convolution is
exact; both sides only differ by rounding).  FP32 path: <= 1e-5 relative to
the FP64 oracle.  All inputs are seeded and shared by both sides.
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


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    return np.abs(got - ref) / np.abs(ref)


def run(ctx, rho_np, h0, dtype=torch.float64, G=1.0, flags=0):
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to("cuda", dtype)
    phi = ctx.solve(rho, h0, G, flags)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy()


# --- FFT core and Green spectrum ---------------------------------------------

@pytest.mark.parametrize("P", [8, 16, 32, 64, 128, 256, 512])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fft_lines_match_numpy(ctx, P, dtype):
    rng = np.random.default_rng(P)
    n = 37
    x = rng.standard_normal((n, P)) + 1j * rng.standard_normal((n, P))
    xt = torch.from_numpy(x).to("cuda", dtype)
    fwd = ctx.fft_lines(xt, -1).cpu().numpy()
    inv = ctx.fft_lines(xt, +1).cpu().numpy()
    ref_f = np.fft.fft(x, axis=1)
    ref_i = np.fft.ifft(x, axis=1) * P
    tol = 1e-14 if dtype == torch.complex128 else 2e-6
    for got, ref in ((fwd, ref_f), (inv, ref_i)):
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < tol * np.log2(P), (P, err)


@pytest.mark.parametrize("N", [4, 12, 32, 64])
def test_green_spectrum_matches_oracle(ctx, N):
    from scipy import fft as sfft
    P = 8
    while P < 2 * N:
        P *= 2
    H = P // 2 + 1
    ref = sfft.rfftn(oracle.green_periodic(P)).real[:H, :H, :H]
    got = ctx.green_spectrum(N, torch.float64).cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err < 1e-14
    got32 = ctx.green_spectrum(N, torch.float32).cpu().numpy()
    assert np.array_equal(got32, got.astype(np.float32))


# --- single and nested solves, FP64 -----------------------------------------

# (N, L) with N a multiple of 2^L take the block-mean pyramid restriction,
# the others the cascaded one; L >= 7 below N = 128 needs two carry launches;
# N = 48 and 64 (P = 128) take the z pass with separate column-0 workgroups
# (N = 48 with input and output rows below the period's half).
@pytest.mark.parametrize("N,L", [(4, 1), (4, 2), (4, 3), (8, 1), (8, 3), (8, 4), (12, 1), (12, 2),
                                 (16, 3), (16, 5), (16, 7), (20, 2), (32, 4), (32, 5), (48, 3), (64, 2)])
def test_random_levels_fp64(ctx, N, L):
    w = inputs.random_levels(N, L, seed=100 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, G=1.3)
    got = run(ctx, rho, w.h0, G=1.3)
    assert np.max(rel_err(got, ref)) < F64_TOL


# N in (128, 256) with period 512: the z pass's wavefront kernel with input
# and output rows below the period's half, child-region boxes, both the
# one- and two-stream schedules.
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,L,flags", [(132, 2, 0), (200, 2, 0), (144, 3, 1 << 4)])
def test_period512_partial_grids(ctx, dtype, N, L, flags):
    w = inputs.random_levels(N, L, seed=150 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, G=0.7)
    got = run(ctx, rho, w.h0, G=0.7, dtype=dtype, flags=flags)
    e = rel_err(got, ref)
    print(f"N={N} L={L} {dtype}: max rel err {np.max(e):.3e}", flush=True)
    assert np.max(e) < (F64_TOL if dtype == torch.float64 else F32_TOL)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restriction_modes_in_one_batch(ctx, dtype):
    """One group mixing pyramid (L = 3, 4) and cascaded (L = 5, 6)
    restrictions and one or two carry launches: each request matches the
    oracle and its own solve alone."""
    items, refs = [], []
    for i, L in enumerate((3, 5, 4, 6)):
        w = inputs.random_levels(16, L, seed=300 + i)
        items.append((w.rho.to("cuda", dtype), w.h0, 1.0 + 0.1 * i))
        refs.append(oracle.solve(w.rho.numpy(), w.h0, G=1.0 + 0.1 * i))
    alone = [ctx.solve(r, h, G).clone() for r, h, G in items]
    batch = ctx.solve_batch(items)
    torch.cuda.synchronize()
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    for a, b, ref in zip(alone, batch, refs):
        assert torch.equal(a, b)
        assert np.max(rel_err(b.double().cpu().numpy(), ref)) < tol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("N,L", [(4, 2), (8, 3), (12, 3), (16, 4), (32, 4)])
def test_fused_plane_passes_match_separate(ctx, dtype, N, L):
    """Up to P = 64 X+Y and I2+I1 run as fused plane passes (one z plane
    per workgroup, kept in LDS); the separate passes (NMC_NO_FUSED_PLANES)
    do the same line transforms, so both agree to rounding and both match
    the oracle."""
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(N, L, seed=400 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0)
    fused = run(ctx, rho, w.h0, dtype=dtype)
    sep = run(ctx, rho, w.h0, dtype=dtype, flags=nmc.NMC_NO_FUSED_PLANES)
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    assert np.max(rel_err(fused, ref)) < tol
    assert np.max(rel_err(sep, ref)) < tol
    agree = 1e-14 if dtype == torch.float64 else 1e-6
    assert np.max(np.abs(fused - sep) / np.abs(sep)) < agree


def test_deep_hierarchy_fp32(ctx):
    """Seven levels of 32^3 in FP32: cascaded restriction and a carry
    cascade split over two launches, with compensated sums."""
    w = inputs.random_levels(32, 7, seed=17)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0)
    got = run(ctx, rho, w.h0, dtype=torch.float32)
    assert np.max(rel_err(got, ref)) < F32_TOL


def test_random12_brute_force(ctx):
    """The 12^3 single-level brute-force check (N=12 runs on a 32^3 period)."""
    w = inputs.random12()
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, method="direct")
    got = run(ctx, rho, w.h0)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_nested_brute_force_12(ctx):
    w = inputs.random_levels(12, 3, seed=7)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, method="direct")
    got = run(ctx, rho, w.h0)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_no_restrict_flag(ctx):
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(16, 3, seed=3)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, restrict=False)
    got = run(ctx, rho, w.h0, flags=nmc.NMC_NO_RESTRICT)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_point_mass(ctx):
    N, L = 16, 3
    rho = np.zeros((L, N, N, N))
    rho[2, 5, 9, 3] = 1.0
    rho[0, 1, 14, 2] = 0.5
    ref = oracle.solve(rho, 0.25)
    got = run(ctx, rho, 0.25)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_zero_density_gives_zero(ctx):
    got = run(ctx, np.zeros((3, 8, 8, 8)), 0.1)
    assert np.all(got == 0)


def test_plummer32_fp64(ctx):
    w = inputs.plummer32()
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0)
    got = run(ctx, rho, w.h0)
    assert np.max(rel_err(got, ref)) < F64_TOL


@pytest.fixture(scope="module")
def ellipsoid64():
    w = inputs.ellipsoid64()
    rho = w.rho.numpy()
    return w, rho, oracle.solve(rho, w.h0)


def test_ellipsoid64_fp64(ctx, ellipsoid64):
    w, rho, ref = ellipsoid64
    got = run(ctx, rho, w.h0)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_ellipsoid64_fp32(ctx, ellipsoid64):
    w, rho, ref = ellipsoid64
    got = run(ctx, rho, w.h0, dtype=torch.float32)
    e = rel_err(got, ref)
    for l in range(w.L):
        print(f"level {l}: max {e[l].max():.3e} rms {np.sqrt((e[l] ** 2).mean()):.3e}")
    assert np.max(e) < F32_TOL


@pytest.fixture(scope="module")
def binary128():
    w = inputs.binary128()
    rho = w.rho.numpy()
    return w, rho, oracle.solve(rho, w.h0)


def test_binary128_fp64(ctx, binary128):
    w, rho, ref = binary128
    got = run(ctx, rho, w.h0)
    assert np.max(rel_err(got, ref)) < F64_TOL


def test_binary128_fp32(ctx, binary128):
    w, rho, ref = binary128
    got = run(ctx, rho, w.h0, dtype=torch.float32)
    e = rel_err(got, ref)
    for l in range(w.L):
        print(f"level {l}: max {e[l].max():.3e} rms {np.sqrt((e[l] ** 2).mean()):.3e}")
    assert np.max(e) < F32_TOL


def test_fp32_uncompensated_still_within_tolerance(ctx, binary128):
    from paper_2301_06763_amd import nmc
    w, rho, ref = binary128
    got = run(ctx, rho, w.h0, dtype=torch.float32, flags=nmc.NMC_F32_UNCOMPENSATED)
    assert np.max(rel_err(got, ref)) < F32_TOL


def _sample_points(L, N, rng, k=3):
    pts = []
    for l in range(L):
        for _ in range(k):
            pts.append((l, *[int(v) for v in rng.integers(0, N, size=3)]))
        # a cell next to the child-region boundary and a corner
        pts.append((l, N // 4 - 1, N // 2, 3 * N // 4))
        pts.append((l, 0, N - 1, 0))
    return pts


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_clumps256_sampled(ctx, dtype):
    """Full-size 256^3 x 6 levels: sampled cells against the direct sum."""
    w = inputs.clumps256(device="cuda")
    rho = w.rho.to(dtype)
    phi = ctx.solve(rho, w.h0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    pts = _sample_points(w.L, w.N, rng, k=1)
    ref = oracle.solve_points(w.rho.cpu().numpy(), w.h0, pts)
    got = np.array([phi[p].item() for p in pts])
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    assert np.max(rel_err(got, ref)) < tol


# --- determinism, batching, serving -------------------------------------------

def test_repeat_determinism(ctx):
    w = inputs.random_levels(32, 3, seed=5)
    rho = w.rho.cuda()
    a = ctx.solve(rho, w.h0).clone()
    b = ctx.solve(rho, w.h0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _mixed(n, dtype=torch.float64):
    out = []
    for i in range(n):
        N = [8, 16, 12, 32][i % 4]
        L = 1 + (i % 4)
        w = inputs.random_levels(N, L, seed=200 + i)
        out.append((w.rho.to("cuda", dtype), w.h0 * (1 + 0.1 * i), 1.0 + 0.05 * i))
    return out


def test_batch_equals_alone(ctx):
    items = _mixed(9)
    alone = [ctx.solve(r, h, G).clone() for r, h, G in items]
    batch = ctx.solve_batch(items)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_serving_mix_equals_alone(dtype):
    """Requests solved in the continuous-batching mix give bitwise the same
    result as alone (grids are independent; kernels are deterministic)."""
    from paper_2301_06763_amd import nmc
    items = _mixed(12, dtype)
    c = nmc.Context(budget_bytes=256 << 20)
    try:
        alone = [c.solve(r, h, G).clone() for r, h, G in items]
        tickets = []
        for k, (r, h, G) in enumerate(items):
            tickets.append(c.submit(r, h, G))
            if k % 3 == 0:
                c.tick()
        c.drain()
        for tk, a in zip(tickets, alone):
            assert c.poll(tk)
            assert torch.equal(tk.phi, a)
        st = c.stats()
        assert st["completed"] == len(items) and st["inflight"] == 0
        assert st["peak_inflight_bytes"] <= 256 << 20
    finally:
        c.close()


def test_serving_request_larger_than_the_ring():
    """Under a budget the serving batches share one allocation used as a
    ring, sized from what the budget leaves; a request larger than the ring
    but within the budget releases it, runs on workspace of its own and
    gives the result it gives alone; the ring is back for the next batch."""
    from paper_2301_06763_amd import nmc
    N, L = 64, 10
    fp = nmc.footprint_bytes(N, L, torch.float64)
    budget = int(fp * 1.04) + (4 << 20)  # the ring (budget less 1/16) is smaller than fp
    w = inputs.random_levels(N, L, seed=32)
    rho = w.rho.to("cuda", torch.float64).contiguous()
    free = nmc.Context()
    try:
        alone = free.solve(rho, w.h0, flags=nmc.NMC_NO_GRAPH).clone()
    finally:
        free.close()
    small = inputs.random_levels(16, 2, seed=31)
    r0 = small.rho.to("cuda", torch.float64).contiguous()
    c = nmc.Context(budget_bytes=budget)
    try:
        c.submit(r0, small.h0)
        c.drain()
        ring = c.stats()["arena_bytes"]
        assert 0 < ring < fp, (ring, fp)
        tk = c.submit(rho, w.h0)
        c.drain()
        assert c.poll(tk)
        assert torch.equal(tk.phi, alone)
        tk2 = c.submit(r0, small.h0)
        c.drain()
        assert c.poll(tk2)
        st = c.stats()
        assert st["arena_bytes"] > 0 and st["completed"] == 3
    finally:
        c.close()


def test_serving_ring_wraps_at_the_budget():
    """Many requests under a budget a few times their footprint: the
    batches' workspace regions wrap around the ring many times, batches
    wait for room instead of failing, and every result equals the same
    request solved alone."""
    from paper_2301_06763_amd import nmc
    shapes = [(32, 3), (64, 4), (32, 5), (64, 2), (48, 3), (64, 5)]
    items = []
    for i in range(48):
        N, L = shapes[i % len(shapes)]
        w = inputs.random_levels(N, L, seed=2000 + i)
        items.append((w.rho.to("cuda", torch.float32).contiguous(), w.h0))
    big = max(nmc.footprint_bytes(r.shape[1], r.shape[0], torch.float32) for r, _ in items)
    budget = 6 * big + (64 << 20)
    c = nmc.Context(budget_bytes=budget)
    try:
        alone = [c.solve(r, h, flags=nmc.NMC_NO_GRAPH).clone() for r, h in items]
        torch.cuda.synchronize()
        tickets = [c.submit(r, h) for r, h in items]
        c.drain()
        for k, (tk, a) in enumerate(zip(tickets, alone)):
            assert c.poll(tk)
            assert torch.equal(tk.phi, a), k
        st = c.stats()
        assert st["completed"] == len(items) and st["inflight"] == 0
        assert 0 < st["arena_bytes"] < budget
        assert st["peak_inflight_bytes"] <= st["arena_bytes"]
        assert st["batches"] >= 4
    finally:
        c.close()


# --- boundary errors ------------------------------------------------------------

def test_invalid_arguments(ctx):
    from paper_2301_06763_amd import nmc
    rho = torch.zeros((2, 8, 8, 8), dtype=torch.float64, device="cuda")
    out = torch.full_like(rho, 7.0)
    L = nmc.lib()
    s = torch.cuda.current_stream().cuda_stream
    h = ctx._h
    assert L.nmc_solve(h, rho.data_ptr(), out.data_ptr(), 6, 2, 0.1, 2, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, rho.data_ptr(), out.data_ptr(), 8, 0, 0.1, 2, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, rho.data_ptr(), out.data_ptr(), 8, 2, -1.0, 2, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, rho.data_ptr(), out.data_ptr(), 8, 2, 0.1, 3, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, rho.data_ptr(), rho.data_ptr(), 8, 2, 0.1, 2, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, None, out.data_ptr(), 8, 2, 0.1, 2, 1.0, 0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_solve(h, rho.data_ptr(), out.data_ptr(), 260, 2, 0.1, 2, 1.0, 0, 0, s) == nmc.NMC_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # untouched on error


def test_budget_rejects_oversized_request():
    from paper_2301_06763_amd import nmc
    c = nmc.Context(budget_bytes=8 << 20)
    try:
        rho = torch.zeros((4, 64, 64, 64), dtype=torch.float64, device="cuda")
        with pytest.raises(nmc.NmcError) as ei:
            c.submit(rho, 0.1)
        assert ei.value.code == nmc.NMC_ENOMEM
        with pytest.raises(nmc.NmcError) as ei:
            c.solve(rho, 0.1)
        assert ei.value.code == nmc.NMC_ENOMEM
    finally:
        c.close()


def test_graph_replay_matches_direct(ctx):
    """Repeated identical calls replay a captured graph; it must read the
    current input each time and match the direct launch bitwise."""
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(32, 3, seed=21)
    rho = w.rho.cuda()
    out = torch.empty_like(rho)
    for k in range(4):
        rho.mul_(1.0 + 0.25 * k)  # new contents, same pointer
        ctx.solve(rho, w.h0, out=out)
        ref = ctx.solve(rho, w.h0, flags=nmc.NMC_NO_GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
    # replays on another stream are ordered after the previous replay
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.solve(rho, w.h0, out=out, stream=s)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


# --- gravitational acceleration (Sect. 2 stencil, Appendix A methods A, B) --

def _accel_tol(phi_ref, h0, bound):
    """Per-level bound on |g - g_ref| implied by a pointwise relative bound on
    the potential: every stencil value is a convex combination of potential
    values, so |dg| <= 2 * bound * max|Phi_l| / (2 h_l)."""
    L = phi_ref.shape[0]
    return [bound * np.max(np.abs(phi_ref[l])) / oracle.level_spacing(h0, l) for l in range(L)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,L", [(8, 1), (8, 3), (12, 3), (16, 4), (32, 3)])
def test_acceleration_stencil_matches_oracle(ctx, dtype, N, L):
    """The GPU stencil applied to the oracle's potential equals the oracle's
    stencil of the same potential (FP64: rounding only; FP32: the input
    rounded to FP32 once)."""
    w = inputs.random_levels(N, L, seed=500 + N + L)
    phi = oracle.solve(w.rho.numpy(), w.h0)
    ref = oracle.acceleration(phi, w.h0)
    g = ctx.acceleration(torch.from_numpy(phi).to("cuda", dtype), w.h0)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    bound = 1e-13 if dtype == torch.float64 else 2e-7
    for l, tol in enumerate(_accel_tol(phi, w.h0, bound)):
        assert np.max(np.abs(g[l] - ref[l])) < tol, l


def test_acceleration_exact_on_linear_potential(ctx):
    """Every rule of the stencil (central, one-sided faces, methods A and
    B) is exact for a linear potential sampled on all levels."""
    N, L = 16, 4
    h0 = 1.0 / N
    a, b, c = 0.3, -1.2, 0.7
    phi = np.zeros((L, N, N, N))
    for l in range(L):
        x = oracle.cell_centres(N, oracle.level_spacing(h0, l))
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        phi[l] = a * X + b * Y + c * Z + 2.0
    g = ctx.acceleration(torch.from_numpy(phi).cuda(), h0).cpu().numpy()
    assert np.max(np.abs(g[:, 0] + a)) < 1e-12
    assert np.max(np.abs(g[:, 1] + b)) < 1e-12
    assert np.max(np.abs(g[:, 2] + c)) < 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_solve_then_acceleration_matches_oracle(ctx, dtype):
    """The whole path (GPU solve, GPU acceleration) against the oracle's,
    within the bound the potential's tolerance implies through the stencil."""
    w = inputs.ellipsoid64()
    rho = w.rho.numpy()
    phi_ref = oracle.solve(rho, w.h0)
    ref = oracle.acceleration(phi_ref, w.h0)
    phi = ctx.solve(w.rho.to("cuda", dtype), w.h0)
    g = ctx.acceleration(phi, w.h0)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    bound = F64_TOL if dtype == torch.float64 else F32_TOL
    for l, tol in enumerate(_accel_tol(phi_ref, w.h0, bound)):
        assert np.max(np.abs(g[l] - ref[l])) < tol, l


def test_acceleration_rejects_bad_arguments(ctx):
    from paper_2301_06763_amd import nmc
    L = nmc.lib()
    phi = torch.zeros((2, 8, 8, 8), dtype=torch.float64, device="cuda")
    g = torch.full((2, 3, 8, 8, 8), 5.0, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    h = ctx._h
    assert L.nmc_acceleration(h, phi.data_ptr(), g.data_ptr(), 6, 2, 0.1, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_acceleration(h, phi.data_ptr(), g.data_ptr(), 8, 0, 0.1, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_acceleration(h, phi.data_ptr(), g.data_ptr(), 8, 2, 0.0, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_acceleration(h, phi.data_ptr(), phi.data_ptr(), 8, 2, 0.1, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_acceleration(h, None, g.data_ptr(), 8, 2, 0.1, 0, s) == nmc.NMC_EINVAL
    assert L.nmc_acceleration(h, phi.data_ptr(), g.data_ptr(), 260, 2, 0.1, 0, s) == nmc.NMC_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(g == 5.0)


# --- the tensor-product carry rule (NMC_PROLONG_TRILINEAR) -------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,L,extra", [(8, 3, 0), (12, 3, 0), (16, 4, 0), (16, 6, 0), (32, 4, 0), (32, 4, 1)])
def test_trilinear_carry(ctx, dtype, N, L, extra):
    """Hole-grid formulation with the tensor-product carry (one cascade
    launch per level), fused plane passes and (extra) the separate ones."""
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(N, L, seed=1200 + N + L)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, trilinear=True)
    flags = nmc.NMC_PROLONG_TRILINEAR | (nmc.NMC_NO_FUSED_PLANES if extra else 0)
    got = run(ctx, rho, w.h0, dtype=dtype, flags=flags)
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    assert np.max(rel_err(got, ref)) < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_trilinear_carry_child_region_boxes(ctx, dtype):
    """N = 128: child-region boxes, S_l = Phi(Omega^l) - C_l left by each
    level's last pass with the tensor-product carry."""
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(128, 3, seed=1300)
    rho = w.rho.numpy()
    ref = oracle.solve(rho, w.h0, trilinear=True)
    got = run(ctx, rho, w.h0, dtype=dtype, flags=nmc.NMC_PROLONG_TRILINEAR)
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    assert np.max(rel_err(got, ref)) < tol


@pytest.mark.parametrize("scheme", ["pairs", "triples"])
def test_trilinear_carry_modified(ctx, scheme):
    from paper_2301_06763_amd import nmc
    w = inputs.random_levels(16, 4, seed=1400)
    rho = w.rho.numpy()
    ref = oracle.solve_modified(rho, w.h0, scheme=scheme, trilinear=True)
    f = nmc.NMC_MODIFIED if scheme == "pairs" else nmc.NMC_MODIFIED3
    for dtype, tol in ((torch.float64, F64_TOL), (torch.float32, F32_TOL)):
        got = run(ctx, rho, w.h0, dtype=dtype, flags=f | nmc.NMC_PROLONG_TRILINEAR)
        assert np.max(rel_err(got, ref)) < tol


def test_trilinear_and_default_in_one_batch(ctx):
    """Requests with either carry rule in one batch fall into separate
    groups; each equals its solve alone."""
    from paper_2301_06763_amd import nmc
    items = []
    for i in range(4):
        w = inputs.random_levels(16, 4, seed=1500 + i)
        items.append((w.rho.to("cuda", torch.float32), w.h0, 1.0, nmc.NMC_PROLONG_TRILINEAR if i % 2 else 0))
    alone = [ctx.solve(r, h, G, f | nmc.NMC_NO_GRAPH).clone() for r, h, G, f in items]
    batch = ctx.solve_batch(items)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a, b)
    assert not torch.equal(alone[0], ctx.solve(items[0][0], items[0][1], 1.0, nmc.NMC_PROLONG_TRILINEAR))


def test_green_cache_evicted_under_budget():
    """The budget covers the workspace and the cached Green tables: with room
    for one three-level 64^3 solve and its tables (periods 128, 256, 512)
    but not for the period-64 tables as well, alternating it with a 32^3
    solve evicts and rebuilds those tables, and every result equals the
    unlimited context's."""
    from paper_2301_06763_amd import nmc
    wv = inputs.random_levels(32, 1, seed=1600)
    wy = inputs.random_levels(64, 3, seed=1601)
    V = (wv.rho.to("cuda", torch.float32), wv.h0, 1.0, 0)
    Y = (wy.rho.to("cuda", torch.float32), wy.h0, 1.0, nmc.NMC_MODIFIED3)
    free = nmc.Context()
    try:
        ref_v = free.solve(*V).clone()
        ref_y = free.solve(*Y).clone()
    finally:
        free.close()
    only_y = nmc.Context()
    try:
        only_y.solve(*Y)
        torch.cuda.synchronize()
        green_y = only_y.stats()["green_cache_bytes"]
    finally:
        only_y.close()
    ws_y = nmc.footprint_bytes(64, 3, torch.float32, nmc.NMC_MODIFIED3)
    ws_y = (ws_y + (2 << 20) - 1) // (2 << 20) * (2 << 20)
    budget = ws_y + green_y + (512 << 10)
    c = nmc.Context(budget_bytes=budget)
    try:
        greens = []
        # direct solves and (repeated calls) captured graphs, which hold workspace
        for (r, h, G, f), ref in ((V, ref_v), (Y, ref_y), (V, ref_v), (Y, ref_y), (Y, ref_y), (V, ref_v)):
            out = c.solve(r, h, G, f)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            g = c.stats()["green_cache_bytes"]
            assert g <= budget
            greens.append(g)
        assert greens[1] == green_y and greens[3] == green_y  # the period-64 tables were evicted
        assert greens[2] > green_y and greens[5] > green_y     # and rebuilt for the 32^3 solve
    finally:
        c.close()
