"""Hv parity: the HIP grouped-GEMM path against the oracle, element by element.

Bars: every element within tol x (the oracle's sum of the magnitudes of the
terms of that element, ``hv_abs_bound``), and every sector block within tol in
relative 2-norm; tol = 1e-12 for FP64, 1e-5 for FP32 (inputs rounded to FP32
once, FP32 accumulation).  The global relative 2-norm is printed.
"""
import numpy as np
import pytest

import workloads as W
from helpers import GpuProblem, asym_shapes, assert_parity, oracle_superblock, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_0707_0159_amd import d2d
    assert torch.cuda.is_available(), "GPU tests need a device"
    c = d2d.d2d_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    d2d.d2d_ctx_destroy(c)


def gpu_hv(ctx, prob, prec, v):
    from paper_0707_0159_amd import d2d
    dt = torch.float64 if prec == d2d.D2D_FP64 else torch.float32
    with torch.cuda.stream(ctx.stream):
        vd = torch.as_tensor(v, dtype=dt).to("cuda")
        wd = torch.full_like(vd, float("nan"))
        d2d.d2d_hv(prob.sb, prec, vd, wd)
    ctx.stream.synchronize()
    return wd.double().cpu().numpy()


def test_heisenberg_2x6_all_sectors_fp64_and_fp32(ctx):
    """2x6 Heisenberg, exact m=16 blocks, every S_z sector of the 4096 space."""
    from paper_0707_0159_amd import d2d
    wl = W.HEISENBERG_2X6_M16
    worst = {0: 0.0, 1: 0.0}
    total = 0
    for nup in range(0, 13):
        osb = oracle_superblock(wl, (nup, 0))
        prob = GpuProblem(ctx, wl, (nup, 0))
        assert prob.info["n"] == osb.N
        qL, dL, dR, off = d2d.d2d_sb_sectors(prob.sb)
        assert [tuple(q) for q in qL] == [s[0] for s in osb.sectors]
        assert list(off) == [s[3] for s in osb.sectors]
        H = osb.explicit()
        Habs = osb.explicit(absolute=True)
        secs = osb.sector_table()
        nvec = 1000 // 13 + 1
        for i in range(nvec):
            v = W.random_vector(osb.N, 1000 + total + i)
            ref = H @ v
            bound = Habs @ np.abs(v)
            for prec in (0, 1):
                w = gpu_hv(ctx, prob, prec, v)
                rep = assert_parity(w, ref, bound, 1e-12 if prec == 0 else 1e-5, secs,
                                    f"2x6 sz {nup} vec {i} prec {prec}") if i < 2 else None
                if rep is None:
                    from helpers import parity
                    rep = parity(w, ref, bound, 1e-12 if prec == 0 else 1e-5, secs)
                    assert rep["n_bad"] == 0 and rep["worst_sector"] <= (1e-12 if prec == 0 else 1e-5)
                worst[prec] = max(worst[prec], rep["rel_norm"])
        total += nvec
        prob.close()
    print("heisenberg_2x6 worst rel err", worst)
    assert worst[0] <= 1e-12
    assert worst[1] <= 1e-5


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_hubbard_2x16_every_tile_shape(ctx, prec, tol):
    """2x16 Hubbard m=256: 47 sector pairs of ragged size, every tile shape."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl)
    assert prob.info["n"] == osb.N
    shapes = [i | sp for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == prec
              for sp in (0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_SPLIT4,
                         d2d.D2D_TILE_XCD, d2d.D2D_TILE_SPLIT | d2d.D2D_TILE_XCD,
                         d2d.D2D_TILE_SPLIT4 | d2d.D2D_TILE_XCD)]
    shapes += [i | d2d.D2D_TILE_ASYM | x for i in asym_shapes(d2d, prec) for x in (0, d2d.D2D_TILE_XCD)]
    assert any(sh & d2d.D2D_TILE_ASYM for sh in shapes)
    secs = osb.sector_table()
    for k in range(3):
        v = W.random_vector(osb.N, 1000 + k)
        ref = osb.hv_factored(v)
        bound = osb.hv_abs_bound(v)
        for sh in shapes:
            d2d.d2d_sb_set_tile(prob.sb, prec, sh)
            w = gpu_hv(ctx, prob, prec, v)
            assert_parity(w, ref, bound, tol, secs, f"prec {prec} shape {sh} vec {k}")
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_persistent_launch_is_bitwise_plain(ctx, prec):
    """D2D_TILE_PERSIST: a grid of resident work-groups taking the work items
    from a counter gives the plain launch's product bit for bit, for every
    tile shape of the precision, unsplit, split, halved and asymmetric; the
    counters the last work-group clears make back-to-back persistent launches
    (and plain ones in between) agree too.  Checked against the oracle as
    well (2x16 Hubbard m=256, 47 sector pairs of ragged size)."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl, prec_mask=15)
    cfgs = [i | sp for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == prec
            for sp in (0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_SPLIT4)]
    cfgs += [i | d2d.D2D_TILE_ASYM for i in asym_shapes(d2d, prec)]
    v = W.random_vector(osb.N, 77)
    # FP64 and FP32 also against the oracle (the BF16 forms have their own parity tests)
    ref = osb.hv_factored(v) if prec in (0, 1) else None
    bound = osb.hv_abs_bound(v) if prec in (0, 1) else None
    secs = osb.sector_table()
    for cfg in cfgs:
        d2d.d2d_sb_set_tile(prob.sb, prec, cfg)
        plain = gpu_hv_prec(ctx, prob, prec, v)
        d2d.d2d_sb_set_tile(prob.sb, prec, cfg | d2d.D2D_TILE_PERSIST)
        first = gpu_hv_prec(ctx, prob, prec, v)
        second = gpu_hv_prec(ctx, prob, prec, v)
        assert np.array_equal(first, plain), f"cfg {cfg}"
        assert np.array_equal(second, plain), f"cfg {cfg} second launch"
        if ref is not None:
            assert_parity(first, ref, bound, 1e-12 if prec == 0 else 1e-5, secs, f"persistent prec {prec} cfg {cfg}")
    with pytest.raises(RuntimeError):   # a persistent launch takes no XCD order
        d2d.d2d_sb_set_tile(prob.sb, prec, cfgs[0] | d2d.D2D_TILE_PERSIST | d2d.D2D_TILE_XCD)
    prob.close()


def gpu_hv_prec(ctx, prob, prec, v):
    """d2d_hv with the input in the precision's storage type (BF16 inputs are
    the FP32 values rounded by torch)."""
    from paper_0707_0159_amd import d2d
    dt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float32}[prec]
    with torch.cuda.stream(ctx.stream):
        vd = torch.as_tensor(np.asarray(v, dtype=np.float64)).to("cuda").to(dt)
        wd = torch.full(vd.shape, float("nan"), dtype=torch.float64 if prec == 0 else torch.float32, device="cuda")
        d2d.d2d_hv(prob.sb, prec, vd, wd)
    ctx.stream.synchronize()
    return wd.double().cpu().numpy()


def test_sector_table_matches_oracle(ctx):
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl)
    qL, dL, dR, off = d2d.d2d_sb_sectors(prob.sb)
    assert [tuple(q) for q in qL] == [s[0] for s in osb.sectors]
    assert list(dL) == [s[1].size for s in osb.sectors]
    assert list(dR) == [s[2].size for s in osb.sectors]
    assert list(off) == [s[3] for s in osb.sectors]
    prob.close()


def test_repeatable_bitwise(ctx):
    """No atomics in the accumulation: repeated products are bit-identical."""
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl)
    v = W.random_vector(prob.info["n"], 7)
    for prec in (0, 1):
        for sp in (0, 1 << 16):
            d2d_set = __import__("paper_0707_0159_amd.d2d", fromlist=["d2d"])
            d2d_set.d2d_sb_set_tile(prob.sb, prec, (4 if prec else 1) | sp)
            a = gpu_hv(ctx, prob, prec, v)
            for _ in range(5):
                assert np.array_equal(a, gpu_hv(ctx, prob, prec, v))
    prob.close()


def bf16_round(x):
    """float64 -> float32 (RNE) -> bfloat16 (RNE), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def oracle_hv_bf16_operands(osb, v, absolute=False):
    """The oracle's matrix form with H_l, H_r sectors and v rounded to bfloat16
    (with ``absolute``: the same on the absolute values of every operand, the
    element-wise bound of that product)."""
    f = np.abs if absolute else (lambda a: a)
    vb = f(bf16_round(v))
    w = np.zeros_like(vb)
    for (q, r, c, o), (hl, hr) in zip(osb.sectors, osb.dense_sectors()):
        dL, dR = r.size, c.size
        V = vb[o:o + dL * dR].reshape(dR, dL).T
        W = f(bf16_round(hl)) @ V + V @ f(bf16_round(hr)).T
        w[o:o + dL * dR] = W.T.reshape(-1)
    for hc, pidx in osb.central_groups():
        w[pidx] += f(hc) @ vb[pidx]
    return w


def bf16x3_parts(x):
    """float64 -> float32, then hi = bf16(x), lo = bf16(x - hi) (each RNE), as float64."""
    f = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = bf16_round(f)
    return hi, bf16_round(f - hi)          # f - hi is exact in float32


def oracle_hv_bf16x3_operands(osb, v):
    """The oracle's matrix form with every GEMM product formed as hi*hi + hi*lo +
    lo*hi of the bf16 parts (lo*lo dropped); the central term on float32(v)."""
    vh, vl = bf16x3_parts(v)
    vf = np.asarray(v, dtype=np.float32).astype(np.float64)
    w = np.zeros_like(vf)
    for (q, r, c, o), (hl, hr) in zip(osb.sectors, osb.dense_sectors()):
        dL, dR = r.size, c.size
        Vh = vh[o:o + dL * dR].reshape(dR, dL).T
        Vl = vl[o:o + dL * dR].reshape(dR, dL).T
        Lh, Ll = bf16x3_parts(hl)
        Rh, Rl = bf16x3_parts(hr)
        W = Lh @ Vh + Lh @ Vl + Ll @ Vh + Vh @ Rh.T + Vh @ Rl.T + Vl @ Rh.T
        w[o:o + dL * dR] = W.T.reshape(-1)
    for hc, pidx in osb.central_groups():
        w[pidx] += hc @ vf[pidx]
    return w


def gpu_hv_bf16(ctx, prob, v):
    from paper_0707_0159_amd import d2d
    with torch.cuda.stream(ctx.stream):
        vd = torch.as_tensor(bf16_bits(v).view(np.int16)).to("cuda")
        wd = torch.full((v.size,), float("nan"), dtype=torch.float32, device="cuda")
        d2d.d2d_hv(prob.sb, d2d.D2D_BF16, vd, wd)
    ctx.stream.synchronize()
    return wd.double().cpu().numpy()


@pytest.mark.parametrize("name", [W.HEISENBERG_2X6_M16.name, W.HUBBARD_2X16_M256.name])
def test_bf16_every_tile_shape(ctx, name):
    """BF16 operands, FP32 accumulation: equal to the oracle on bf16-rounded
    operands up to FP32 accumulation (<= 1e-5), and within 2e-2 of the exact product."""
    from paper_0707_0159_amd import d2d
    wl = W.WORKLOADS[name]
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl, prec_mask=7)
    shapes = [i | sp for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == d2d.D2D_BF16
              for sp in (0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_SPLIT4,
                         d2d.D2D_TILE_XCD, d2d.D2D_TILE_SPLIT | d2d.D2D_TILE_XCD,
                         d2d.D2D_TILE_SPLIT4 | d2d.D2D_TILE_XCD)]
    shapes += [i | d2d.D2D_TILE_ASYM | x for i in asym_shapes(d2d, d2d.D2D_BF16) for x in (0, d2d.D2D_TILE_XCD)]
    assert shapes
    secs = osb.sector_table()
    for k in range(2):
        v = W.random_vector(osb.N, 1000 + k)
        ref_b = oracle_hv_bf16_operands(osb, v)
        bound_b = oracle_hv_bf16_operands(osb, v, absolute=True)
        ref = osb.hv_factored(v)
        bound = osb.hv_abs_bound(v)
        for sh in shapes:
            d2d.d2d_sb_set_tile(prob.sb, d2d.D2D_BF16, sh)
            w = gpu_hv_bf16(ctx, prob, v)
            assert_parity(w, ref_b, bound_b, 1e-5, secs, f"{name} bf16 shape {sh} vs bf16-operand oracle")
            assert_parity(w, ref, bound, 2e-2, None, f"{name} bf16 shape {sh} vs exact")
    prob.close()


@pytest.mark.parametrize("name,target", [(W.HEISENBERG_2X6_M16.name, (6, 0)), (W.HEISENBERG_2X6_M16.name, (3, 0)), (W.HUBBARD_2X16_M256.name, None)])
def test_pack_unpack_full_space(ctx, name, target):
    """d2d_pack / d2d_unpack against the oracle's index map of the paper's
    vector order (pure data movement: equal bit for bit; unpack zero-fills
    outside the target sector)."""
    from paper_0707_0159_amd import d2d
    wl = W.WORKLOADS[name]
    osb = oracle_superblock(wl, target)
    prob = GpuProblem(ctx, wl, target)
    D = osb.m * osb.n
    x = W.random_vector(D * D, 77)
    with torch.cuda.stream(ctx.stream):
        xd = torch.as_tensor(x).to("cuda")
        pd = torch.full((osb.N,), float("nan"), dtype=torch.float64, device="cuda")
        fd = torch.full((D * D,), float("nan"), dtype=torch.float64, device="cuda")
        d2d.d2d_pack(prob.sb, xd, pd)
        d2d.d2d_unpack(prob.sb, pd, fd)
    ctx.stream.synchronize()
    packed = osb.pack(x)
    assert np.array_equal(pd.cpu().numpy(), packed)
    assert np.array_equal(fd.cpu().numpy(), osb.unpack(packed))
    del xd, pd, fd
    prob.close()


@pytest.mark.parametrize("name", [W.HEISENBERG_2X6_M16.name, W.HUBBARD_2X16_M256.name])
def test_bf16x3_every_tile_shape(ctx, name):
    """BF16x3 (hi/lo bf16 parts of FP32 operands, three products, FP32
    accumulation): equal to the oracle computing the same three products in
    float64 up to FP32 accumulation (<= 1e-5), and within 1e-4 of the exact product."""
    from paper_0707_0159_amd import d2d
    wl = W.WORKLOADS[name]
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl, prec_mask=15)
    shapes = [i | sp for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == d2d.D2D_BF16X3
              for sp in (0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_SPLIT4, d2d.D2D_TILE_XCD)]
    shapes += [i | d2d.D2D_TILE_ASYM | x for i in asym_shapes(d2d, d2d.D2D_BF16X3) for x in (0, d2d.D2D_TILE_XCD)]
    assert shapes
    worst = 0.0
    secs = osb.sector_table()
    for k in range(2):
        v = W.random_vector(osb.N, 1000 + k)
        ref3 = oracle_hv_bf16x3_operands(osb, v)
        ref = osb.hv_factored(v)
        bound = osb.hv_abs_bound(v)
        for sh in shapes:
            d2d.d2d_sb_set_tile(prob.sb, d2d.D2D_BF16X3, sh)
            w = gpu_hv(ctx, prob, d2d.D2D_BF16X3, v)
            assert_parity(w, ref3, bound, 1e-5, secs, f"{name} bf16x3 shape {sh} vs split-operand oracle")
            rep = assert_parity(w, ref, bound, 1e-4, None, f"{name} bf16x3 shape {sh} vs exact")
            worst = max(worst, rep["rel_norm"])
    print("worst vs exact", worst)
    prob.close()


def sector_step_flops(osb, BM, BN, BK, dense):
    """The grouped GEMM's flops for one tile shape, from the oracle's dense
    sector operators: per output tile and K step of BK, 2 x rows x columns x
    (K columns in the step), every step (dense) or only the steps whose
    operator tile holds a nonzero in 16 x 16 cells (the library's granularity).
    The sector operators the grouped GEMM carries are the halves without the
    explicit columns' own off-diagonal terms (those go with the central term)."""
    total = 0.0
    for (q, r, c, o), (hl, hr) in zip(osb.sectors, osb.dense_sectors(column_offdiagonal=False)):
        dL, dR = r.size, c.size
        for H, d, dout, B in ((hl, dL, dR, BM), (hr, dR, dL, BN)):
            # nonzero 16 x 16 cells of H (rows: output rows of the product, columns: K)
            nc = -(-d // 16)
            P = np.zeros((nc * 16, nc * 16), dtype=bool)
            P[:d, :d] = H != 0
            cells = P.reshape(nc, 16, nc, 16).any(axis=(1, 3))
            for t0 in range(0, d, B):
                rows = min(B, d - t0)
                for k0 in range(0, d, BK):
                    keep = dense or cells[t0 // 16:-(-min(t0 + B, d) // 16), k0 // 16:-(-min(k0 + BK, d) // 16)].any()
                    if keep:
                        # each tile's rows meet every output tile of the other dimension
                        total += 2.0 * rows * min(BK, d - k0) * dout
    return total


def aligned_step_flops(osb, shape0, shape1, dense, padded):
    """The asymmetric split's flops from the oracle's dense sector operators:
    H_l V items on segments of at most BM0 rows inside each run of one
    column-2 state, every BN0 columns; V H_r^T items on segments of at most
    BN1 columns inside each run of one column-3 state, every BM1 rows; a K
    step of BK runs when its 16-column cells hold a nonzero in the segment's
    own rows (columns) of the operator (every step with dense); 2 x segment
    x other extent x the step's K columns inside the block.  K runs over the
    length padded to a multiple of 8 for the BF16 operands (padded)."""
    (BM0, BN0, BK), (BM1, BN1, _) = shape0, shape1
    m = osb.m
    total = 0.0
    for (q, r, c, o), (hl, hr) in zip(osb.sectors, osb.dense_sectors(column_offdiagonal=False)):
        dL, dR = r.size, c.size
        for H, idx, dout, SEG, OTHER in ((hl, r, dR, BM0, BN0), (hr, c, dL, BN1, BM1)):
            d = idx.size
            KL = -(-d // 8) * 8 if padded else d
            nc = -(-d // 16)
            P = np.zeros((d, nc * 16), dtype=bool)
            P[:, :d] = H != 0
            cells = P.reshape(d, nc, 16).any(axis=2)          # per row of H: its nonzero 16-column cells
            a = idx // m
            starts = [0] + [i for i in range(1, d) if a[i] != a[i - 1]] + [d]
            ntiles = -(-dout // OTHER)
            for s0, s1 in zip(starts[:-1], starts[1:]):
                for t0 in range(s0, s1, SEG):
                    t1 = min(s1, t0 + SEG)
                    rows = cells[t0:t1].any(axis=0)
                    for k0 in range(0, KL, BK):
                        c0, c1 = k0 // 16, min(-(-(k0 + BK) // 16), nc)
                        if dense or (c0 < c1 and rows[c0:c1].any()):
                            kk = max(0, min(BK, d - k0))
                            for j in range(ntiles):
                                total += 2.0 * (t1 - t0) * min(OTHER, dout - j * OTHER) * kk
    return total


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_skipped_k_steps_add_nothing(ctx, prec):
    """K steps whose operator tile is zero are left out: the product is bit
    for bit the one that runs every step (unhalved K-loops; every shape, with
    split K-loops and the XCD order too), and the flops the library reports
    for either are the oracle's count over the same steps."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl, prec_mask=15)
    v = W.random_vector(osb.N, 1200 + prec)
    run = gpu_hv_bf16 if prec == d2d.D2D_BF16 else (lambda c, p, x: gpu_hv(c, p, prec, x))
    fewer = 0
    for i, s in enumerate(d2d.d2d_tile_shapes()):
        if s[0] != prec:
            continue
        dense_f = sector_step_flops(osb, s[1], s[2], s[3], True)
        skip_f = sector_step_flops(osb, s[1], s[2], s[3], False)
        for sp in (0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_XCD) + ((d2d.D2D_TILE_ASYM,) if i in asym_shapes(d2d, prec) else ()):
            if sp == d2d.D2D_TILE_ASYM:
                # run-aligned items in the lead shape and its transposed partner:
                # every step and only the nonzero ones agree bit for bit, and
                # the library's flops are the oracle's count of the same steps
                sh0, sh1 = d2d.d2d_tile_shapes()[i][1:4], d2d.d2d_tile_shapes()[i + 1][1:4]
                padded = prec in (d2d.D2D_BF16, d2d.D2D_BF16X3)
                d2d.d2d_sb_set_tile(prob.sb, prec, i | sp | d2d.D2D_TILE_DENSE)
                fd = d2d.d2d_sb_gemm_flops(prob.sb, prec)
                wd = run(ctx, prob, v)
                d2d.d2d_sb_set_tile(prob.sb, prec, i | sp)
                fs = d2d.d2d_sb_gemm_flops(prob.sb, prec)
                ws = run(ctx, prob, v)
                ad = aligned_step_flops(osb, sh0, sh1, True, padded)
                asf = aligned_step_flops(osb, sh0, sh1, False, padded)
                print(f"prec {prec} shape {i} asym: flops every step {fd:.4e}, skipping {fs:.4e} "
                      f"({fs / prob.info['flops_nnz']:.3f} of F_nnz)")
                assert np.array_equal(wd, ws)
                assert abs(fd - ad) <= 1e-9 * ad and abs(fs - asf) <= 1e-9 * ad
                # the XCD order moves the same items: same product, same flops
                d2d.d2d_sb_set_tile(prob.sb, prec, i | sp | d2d.D2D_TILE_XCD)
                assert d2d.d2d_sb_gemm_flops(prob.sb, prec) == fs
                assert np.array_equal(run(ctx, prob, v), ws)
                continue
            d2d.d2d_sb_set_tile(prob.sb, prec, i | sp | d2d.D2D_TILE_DENSE)
            fd = d2d.d2d_sb_gemm_flops(prob.sb, prec)
            wd = run(ctx, prob, v)
            d2d.d2d_sb_set_tile(prob.sb, prec, i | sp)
            fs = d2d.d2d_sb_gemm_flops(prob.sb, prec)
            ws = run(ctx, prob, v)
            print(f"prec {prec} shape {i} flags {sp:#x}: flops dense {fd:.4e} skipping {fs:.4e} ({fs / fd:.3f})")
            assert np.array_equal(wd, ws)
            assert abs(fd - dense_f) <= 1e-9 * dense_f and abs(fs - skip_f) <= 1e-9 * dense_f
        assert abs(dense_f - prob.info["flops_exec"]) <= 1e-9 * dense_f
        fewer += skip_f < dense_f
    assert fewer >= 1
    d2d.d2d_sb_set_tile(prob.sb, prec, -1)
    prob.close()
