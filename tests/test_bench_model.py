"""The benchmark's time-to-energy bound (host arithmetic only, no GPU): the
per-step and per-restart byte counts and the per-product bound, recomputed
by hand for small cases."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_basis_bytes(bench):
    # precision index: 0 FP64, 1 FP32, 2 BF16, 3 BF16x3
    assert [bench.basis_bytes(p, 0) for p in range(4)] == [8, 4, 2, 4]
    assert [bench.basis_bytes(p, 1) for p in range(4)] == [8, 8, 8, 8]
    assert [bench.basis_bytes(p, 2) for p in range(4)] == [8, 4, 4, 4]


def test_fp32_solve_bound(bench):
    n, k, win = 1000, 11, 3
    stats = {"hv_count": [5, 40, 0, 0], "restarts": 4}
    flops = {"fp64": 2e9, "fp32": 3e9, "bf16": 3e9, "bf16x3": 3e9}
    byts = {"fp64": 4e6, "fp32": 2e6, "bf16": 1e6, "bf16x3": 2e6}
    pk = bench.PEAK
    t = bench.solve_time_parts(stats, n, k, win, 0, flops, byts)
    hv = 5 * max(2e9 / pk["fp64"], 4e6 / pk["hbm"]) + 40 * max(3e9 / pk["fp32"], 2e6 / pk["hbm"])
    assert t["hv_s"] == pytest.approx(hv)
    assert t["hv_flop_s"] == pytest.approx(5 * 2e9 / pk["fp64"] + 40 * 3e9 / pk["fp32"])
    assert t["hv_byte_s"] == pytest.approx((5 * 4e6 + 40 * 2e6) / pk["hbm"])
    # 40 FP32 steps: product 4 B read twice, window of 3 FP32 vectors read twice,
    # the next vector written, no input copy; 5 restarts at N (88 + 12 x 4)
    step = 40 * n * (2 * 4 + 2 * 3 * 4 + 4) / pk["hbm"]
    restart = 5 * n * (88 + 12 * 4) / pk["hbm"]
    assert t["vec_s"] == pytest.approx(step + restart)


def test_fp64_solve_counts_only_inner_steps(bench):
    # an FP64 solve's count includes one residual product per restart and the first
    n, k = 500, 9
    stats = {"hv_count": [1 + 3 * 9, 0, 0, 0], "restarts": 3}
    f = {x: 1.0 for x in bench.PREC_NAMES}
    t = bench.solve_time_parts(stats, n, k, 3, 0, f, f)
    steps = 3 * 8
    assert t["vec_s"] == pytest.approx((steps * n * (16 + 48 + 8) + 4 * n * (88 + 10 * 8)) / bench.PEAK["hbm"])


@pytest.mark.parametrize("basis,bq,ci", [(0, 2, 0), (1, 8, 2), (2, 4, 2)])
def test_bf16_step_bytes_follow_the_basis(bench, basis, bq, ci):
    n, k = 100, 5
    stats = {"hv_count": [3, 0, 8, 0], "restarts": 2}
    f = {x: 0.0 for x in bench.PREC_NAMES}
    t = bench.solve_time_parts(stats, n, k, 3, basis, f, f)
    expect = (8 * n * (2 * 4 + 2 * 3 * bq + bq + ci) + 3 * n * (88 + 6 * bq)) / bench.PEAK["hbm"]
    assert t["vec_s"] == pytest.approx(expect)


def test_one_kernel_step_reads_product_and_window_once(bench):
    # FP32 solve, window 3, FP32 basis: the one-kernel form reads the product
    # (4 B) and the window (3 x 4 B) once instead of twice per step
    n, k = 1000, 7
    stats = {"hv_count": [2, 30, 0, 0], "restarts": 1}
    f = {x: 0.0 for x in bench.PREC_NAMES}
    two = bench.solve_time_parts(stats, n, k, 3, 0, f, f)
    one = bench.solve_time_parts(stats, n, k, 3, 0, f, f, step_reads=1)
    restart = 2 * n * (88 + 8 * 4) / bench.PEAK["hbm"]
    assert two["vec_s"] == pytest.approx((30 * n * (2 * (4 + 12) + 4) / bench.PEAK["hbm"]) + restart)
    assert one["vec_s"] == pytest.approx((30 * n * ((4 + 12) + 4) / bench.PEAK["hbm"]) + restart)


def test_tile_desc(bench):
    """The bench line's description of a launch configuration (host only: a
    made-up shape table of (precision, BM, BN, BK, prefetch depth) rows)."""
    from paper_0707_0159_amd import d2d
    shapes = [(1, 64, 64, 16, 2), (1, 64, 256, 16, 2), (1, 256, 64, 16, 2)]
    d = bench.tile_desc(1 | d2d.D2D_TILE_ASYM, shapes)
    assert d["split_k_loops"] == "asymmetric" and d["BMxBNxBK"] == "64x256x16 + 256x64x16"
    d = bench.tile_desc(0 | d2d.D2D_TILE_SPLIT4 | d2d.D2D_TILE_PERSIST, shapes)
    assert d["split_k_loops"] == "halves" and d["persistent"] and d["BMxBNxBK"] == "64x64x16"
    d = bench.tile_desc(0 | d2d.D2D_TILE_SPLIT | d2d.D2D_TILE_XCD | d2d.D2D_TILE_FUSED, shapes)
    assert d["split_k_loops"] is True and d["xcd_order"] and d["central_in_gemm_launch"] and not d["persistent"]
    assert bench.split_words("asymmetric").startswith(", asymmetric")
