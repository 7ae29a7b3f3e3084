"""Full-size parity on the large workloads (3-leg Hubbard m=400, 4-leg Heisenberg m=1000).

Every element of w = Hv is compared with the oracle's matrix-form product at the
real superblock size (N = 3e7 .. 4e7), in the launch configuration the
benchmark uses (autotuned tiles); ground energies against the reference
energies written by the oracle.
"""
import numpy as np
import pytest

import workloads as W
from helpers import GpuProblem, assert_parity, oracle_superblock, reference_energy
from test_gpu_hv import bf16_bits, oracle_hv_bf16_operands

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_0707_0159_amd import d2d
    assert torch.cuda.is_available(), "GPU tests need a device"
    c = d2d.d2d_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    d2d.d2d_ctx_destroy(c)


@pytest.fixture(scope="module", params=[W.HUBBARD_3X12_M400.name, W.HEISENBERG_4X16_M1000.name])
def problem(request, ctx):
    wl = W.WORKLOADS[request.param]
    print(f"building {wl.name}", flush=True)
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl, prec_mask=15)
    yield wl, osb, prob
    prob.close()


def hv(ctx, prob, prec, v):
    from paper_0707_0159_amd import d2d
    with torch.cuda.stream(ctx.stream):
        if prec == d2d.D2D_BF16:
            vd = torch.as_tensor(bf16_bits(v).view(np.int16)).to("cuda")
            wd = torch.empty(v.size, dtype=torch.float32, device="cuda")
        else:
            vd = torch.as_tensor(v, dtype=torch.float64 if prec == 0 else torch.float32).to("cuda")
            wd = torch.empty_like(vd)
        d2d.d2d_hv(prob.sb, prec, vd, wd)
    ctx.stream.synchronize()
    out = wd.double().cpu().numpy()
    del vd, wd
    return out


def test_full_size_hv(ctx, problem):
    from paper_0707_0159_amd import d2d
    wl, osb, prob = problem
    assert prob.info["n"] == osb.N
    qL, dL, dR, off = d2d.d2d_sb_sectors(prob.sb)
    assert [tuple(q) for q in qL] == [s[0] for s in osb.sectors]
    for prec in (0, 1, 2, 3):
        d2d.d2d_sb_autotune(prob.sb, prec, reps=3)
    v = W.random_vector(osb.N, 1000)
    ref = osb.hv_factored(v)
    bound = osb.hv_abs_bound(v)
    secs = osb.sector_table()
    print(f"{wl.name}: N={osb.N}", flush=True)
    assert_parity(hv(ctx, prob, 0, v), ref, bound, 1e-12, secs, f"{wl.name} fp64")
    assert_parity(hv(ctx, prob, 1, v), ref, bound, 1e-5, secs, f"{wl.name} fp32")
    w16 = hv(ctx, prob, 2, v)
    assert_parity(w16, ref, bound, 2e-2, None, f"{wl.name} bf16 vs exact")
    ref_b = oracle_hv_bf16_operands(osb, v)
    bound_b = oracle_hv_bf16_operands(osb, v, absolute=True)
    assert_parity(w16, ref_b, bound_b, 1e-5, secs, f"{wl.name} bf16 vs bf16-operand oracle")
    del ref_b, bound_b, w16
    assert_parity(hv(ctx, prob, 3, v), ref, bound, 1e-4, secs, f"{wl.name} bf16x3 vs exact")


def test_full_size_skipped_k_steps(ctx, problem):
    """At the real sizes the sector operators are block sparse: the K steps
    left out remove a good share of the dense-sector flops, and the product
    equals, bit for bit, the one that runs every step (in the autotuned
    configuration, its K-loops unhalved)."""
    from paper_0707_0159_amd import d2d
    wl, osb, prob = problem
    v = W.random_vector(osb.N, 1300)
    for prec in (0, 1, 2, 3):
        tile, _ = d2d.d2d_sb_autotune(prob.sb, prec, reps=3)
        t = tile & ~d2d.D2D_TILE_SPLIT4 & ~d2d.D2D_TILE_DENSE
        d2d.d2d_sb_set_tile(prob.sb, prec, t | d2d.D2D_TILE_DENSE)
        fd = d2d.d2d_sb_gemm_flops(prob.sb, prec)
        wd = hv(ctx, prob, prec, v)
        d2d.d2d_sb_set_tile(prob.sb, prec, t)
        fs = d2d.d2d_sb_gemm_flops(prob.sb, prec)
        ws = hv(ctx, prob, prec, v)
        d2d.d2d_sb_set_tile(prob.sb, prec, tile)
        print(f"{wl.name} prec {prec} tile {t:#x}: flops {fs:.4e} of {fd:.4e} ({fs / fd:.3f})")
        assert abs(fd - prob.info["flops_exec"]) <= 1e-9 * fd
        assert np.array_equal(wd, ws)
        assert fs <= 0.8 * fd


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_full_size_energy(ctx, problem, prec):
    from paper_0707_0159_amd import d2d
    wl, osb, prob = problem
    E0 = reference_energy(wl.name)
    n = prob.info["n"]
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(n, wl.seed)).to("cuda")
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=prec, k_in=24, max_restarts=400, tol_res=1e-8, use_graph=1)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
    print(f"{wl.name} prec {prec}: E={e:.14f} ref {E0:.14f} dE {(e - E0) / abs(E0):.2e} "
          f"restarts {stats['restarts']} hv {stats['hv_count']} {stats['seconds']:.3f}s")
    assert st == 0
    assert abs(e - E0) <= 1e-10 * abs(E0)
