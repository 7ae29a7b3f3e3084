"""Ground energy of the HIP restarted Lanczos against the oracle (|dE| <= 1e-10 relative)."""
import numpy as np
import pytest

import workloads as W
from helpers import GpuProblem, oracle_superblock, reference_energy

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


def run(ctx, prob, prec, seed, k_in=24, graph=1, tol=1e-9, window=0, separate=0, plain=0, basis=0, one=0):
    from paper_0707_0159_amd import d2d
    n = prob.info["n"]
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(n, seed)).to("cuda")
        psi = torch.zeros_like(v0)
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=prec, k_in=k_in, max_restarts=300, tol_res=tol, use_graph=graph,
                            reorth_window=window, separate_central=separate, plain_cgs2=plain,
                            basis=basis, one_kernel_step=one)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0, psi)
    ctx.stream.synchronize()
    return st, e, stats, psi.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("graph", [0, 1])
def test_heisenberg_2x6_energy(ctx, prec, graph):
    wl = W.HEISENBERG_2X6_M16
    prob = GpuProblem(ctx, wl)
    st, e, stats, psi = run(ctx, prob, prec, wl.seed, graph=graph)
    E0 = reference_energy(wl.name)
    print("heisenberg_2x6", prec, graph, e, E0, stats["restarts"], stats["hv_count"])
    assert st == 0
    assert abs(e - E0) <= 1e-10 * abs(E0)
    # psi is an eigenvector of the oracle's operator
    osb = oracle_superblock(wl)
    r = osb.hv_explicit(psi) - e * psi
    assert np.linalg.norm(r) <= 1e-8 * abs(E0)
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("window,plain", [(0, 0), (3, 0), (3, 1), (2, 0), (4, 0)])
def test_hubbard_2x16_energy(ctx, prec, window, plain):
    """Full reorthogonalisation, and windows of 2..4 in the two-kernel Gram form
    and the three-kernel two-pass form."""
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    st, e, stats, psi = run(ctx, prob, prec, wl.seed, window=window, plain=plain)
    E0 = reference_energy(wl.name)
    print("hubbard_2x16", prec, window, plain, e, E0, (e - E0) / abs(E0), stats["restarts"], stats["hv_count"],
          stats["seconds"])
    assert st == 0
    assert abs(e - E0) <= 1e-10 * abs(E0)
    assert e >= E0 - 1e-10 * abs(E0)          # Rayleigh quotient is variational
    prob.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("window", [0, 3])
def test_basis_storage(ctx, prec, window):
    """The inner basis in the products' input precision (the default: FP32,
    BF16 for BF16 products), in FP64 and in FP32: every low precision reaches
    the oracle's energy, and the Ritz vector is an eigenvector of the oracle's
    operator to the residual bar (the start vector enters the Ritz vector in
    FP64, so the storage rounding only touches the correction)."""
    wl = W.HEISENBERG_2X6_M16
    prob = GpuProblem(ctx, wl, prec_mask=15)
    E0 = reference_energy(wl.name)
    osb = oracle_superblock(wl)
    for basis in (0, 1, 2):
        st, e, stats, psi = run(ctx, prob, prec, wl.seed, window=window, basis=basis)
        print("basis", prec, window, basis, e, E0, stats["restarts"], stats["hv_count"])
        assert st == 0
        assert abs(e - E0) <= 1e-10 * abs(E0)
        r = osb.hv_explicit(psi) - e * psi
        assert np.linalg.norm(r) <= 1e-8 * abs(E0)
    prob.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_odd_length_basis(ctx, prec):
    """An odd packed length (the 2x6 ladder's blocks in the 8-up sector, 495
    states): basis vectors of 2 or 4 bytes start on padded strides, and the
    BF16 central-term gathers read whole aligned words; the energy equals the
    lowest eigenvalue of the oracle's explicit matrix of that sector."""
    wl = W.HEISENBERG_2X6_M16
    tgt = (8, 0)
    prob = GpuProblem(ctx, wl, target=tgt, prec_mask=15)
    assert prob.info["n"] == 495
    E0 = float(np.linalg.eigvalsh(oracle_superblock(wl, tgt).explicit().toarray())[0])
    for basis in (0, 2):
        st, e, stats, _ = run(ctx, prob, prec, wl.seed, window=3, tol=1e-9, basis=basis)
        print("odd length", prec, basis, e, E0, stats["restarts"], stats["hv_count"])
        assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    prob.close()


@pytest.mark.parametrize("basis", [0, 1, 2])
def test_hubbard_2x16_bf16_basis(ctx, basis):
    """The 2x16 Hubbard ladder in BF16 with each basis storage: the oracle's energy, with
    the default fitted cycles and the window of the benchmark."""
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    E0 = reference_energy(wl.name)
    st, e, stats, _ = run(ctx, prob, 2, wl.seed, window=3, tol=1e-8, basis=basis)
    print("hubbard_2x16 bf16 basis", basis, e, stats["restarts"], stats["hv_count"], stats["log_prec"])
    assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    prob.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_krylov_size_limits(ctx, prec):
    """With a window, k_in runs up to 128 (here 64, window 3); full
    reorthogonalisation projects on at most 32 basis vectors, so it takes k_in
    up to 32.  k_in 33 with it, k_in 129, and a window of 33 are refused before
    any launch."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl)
    E0 = reference_energy(wl.name)
    for k, win in ((64, 3), (32, 0)):
        st, e, stats, _ = run(ctx, prob, prec, wl.seed, k_in=k, window=win, tol=1e-8)
        print("k_in", prec, k, win, e, stats["restarts"], stats["hv_count"])
        assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    for k, win in ((33, 0), (129, 3), (24, 33)):
        with pytest.raises(d2d.D2DError, match="k_in"):
            run(ctx, prob, prec, wl.seed, k_in=k, window=win)
    prob.close()


def test_bf16_cycles_use_their_own_krylov_size(ctx):
    """k_in_bf16 sets the length of the BF16 cycles only: every BF16 restart
    adds k_in_bf16 - 1 products, any other precision k_in - 1, and the solve
    reaches the oracle's energy."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(prob.info["n"], wl.seed)).to("cuda")
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=2, k_in=48, k_in_bf16=16, max_restarts=300, tol_res=1e-8, reorth_window=3,
                            fixed_cycles=1)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
    E0 = reference_energy(wl.name)
    hv = stats["hv_count"]
    print("k_in_bf16", e, stats["restarts"], hv, stats["log_prec"])
    assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    assert hv[2] > 0 and hv[2] % 15 == 0 and hv[1] % 47 == 0 and hv[3] % 47 == 0
    assert hv[2] // 15 + hv[1] // 47 + hv[3] // 47 == stats["restarts"]
    assert hv[0] == stats["restarts"] + 1
    prob.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_last_cycle_fits_the_residual_bar(ctx, prec):
    """With fixed_cycles 0 a cycle stops early when the previous cycle's
    residual rate reaches the bar sooner: the solve meets the oracle's energy
    with fewer products than full cycles, and the inner products are no
    longer a multiple of k_in - 1; fixed_cycles 1 keeps every cycle full."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl)
    E0 = reference_energy(wl.name)
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(prob.info["n"], wl.seed)).to("cuda")
    ctx.stream.synchronize()
    out = {}
    for fixed in (0, 1):
        opts = d2d.lanczos_opts(prec=prec, k_in=64, max_restarts=300, tol_res=1e-8, reorth_window=3,
                                fixed_cycles=fixed)
        st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
        inner = sum(stats["hv_count"]) - (stats["restarts"] + 1)
        print("fixed_cycles", prec, fixed, e, stats["restarts"], stats["hv_count"], stats["log_rho"])
        assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
        assert stats["residual"] <= 1e-8 * abs(e)
        out[fixed] = (inner, stats["restarts"])
    assert out[1][0] == 63 * out[1][1]
    assert out[0][0] % 63 != 0 and out[0][0] < out[1][0]
    prob.close()


def test_fp64_solve_ignores_basis_option(ctx):
    """At FP64 the basis is FP64 whatever the basis option says: identical iterates."""
    wl = W.HEISENBERG_2X6_M16
    prob = GpuProblem(ctx, wl)
    out = [run(ctx, prob, 0, wl.seed, window=3, basis=b) for b in (0, 1, 2)]
    for s1, e1, st1, p1 in out:
        assert s1 == 0 and e1 == out[0][1]
        assert np.array_equal(np.asarray(st1["log_theta"]), np.asarray(out[0][2]["log_theta"]))
        assert np.array_equal(p1, out[0][3])
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_one_kernel_step_is_bitwise_two_kernels(ctx, prec):
    """The Gram step as one cooperative kernel (sums, grid barrier, update
    from registers) against the two kernels, direct launches on the 2x16
    Hubbard ladder (412 blocks of at most 2048 elements): the same iterates
    bit for bit."""
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    out = [run(ctx, prob, prec, wl.seed, k_in=48, graph=0, window=3, tol=1e-8, one=o) for o in (1, 0)]
    (s0, e0, st0, p0), (s1, e1, st1, p1) = out
    print("one kernel", prec, e0, e1, st0["restarts"], st0["hv_count"], "cooperative steps", st0["coop_steps"])
    assert s0 == 0 and s1 == 0
    assert st0["coop_steps"] > 0 and st1["coop_steps"] == 0   # the cooperative path ran, and only when asked
    assert e0 == e1
    assert st0["hv_count"] == st1["hv_count"]
    assert np.array_equal(np.asarray(st0["log_theta"]), np.asarray(st1["log_theta"]))
    assert np.array_equal(np.asarray(st0["log_rho"]), np.asarray(st1["log_rho"]))
    assert np.array_equal(p0, p1)
    E0 = reference_energy(wl.name)
    assert abs(e0 - E0) <= 1e-10 * abs(E0)
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("split", [0, 1, 2, 3])
def test_fused_central_is_bitwise_separate(ctx, prec, split):
    """One launch for GEMM + central term (parts added by the first step kernel)
    gives the same iterates bit for bit as the central term launched after the
    GEMM: same energies, restart logs and Ritz vector; for unsplit, split,
    halved and asymmetric K-loops (two GEMM launches, the central term on the
    second)."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    shape = next(i for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == prec)
    if split == 3:
        from helpers import asym_shapes
        shape = asym_shapes(d2d, prec)[0]
    flag = [0, d2d.D2D_TILE_SPLIT, d2d.D2D_TILE_SPLIT4, d2d.D2D_TILE_ASYM][split]
    d2d.d2d_sb_set_tile(prob.sb, prec, shape | flag | d2d.D2D_TILE_FUSED)
    out = [run(ctx, prob, prec, wl.seed, window=3, tol=1e-8, separate=sep) for sep in (0, 1)]
    (s0, e0, st0, p0), (s1, e1, st1, p1) = out
    assert s0 == 0 and s1 == 0
    assert e0 == e1
    assert st0["restarts"] == st1["restarts"]
    assert np.array_equal(np.asarray(st0["log_theta"]), np.asarray(st1["log_theta"]))
    assert np.array_equal(p0, p1)
    prob.close()


def test_seeded_start_vector(ctx):
    """v0 = NULL: the device draws the SplitMix64 / Box-Muller start vector; the
    same vector generated on the host gives the same solve (same restarts,
    energies within rounding of the two log/cos implementations)."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl)
    n = prob.info["n"]
    E0 = reference_energy(wl.name)
    opts = d2d.lanczos_opts(prec=1, k_in=24, max_restarts=300, tol_res=1e-8, reorth_window=3, seed=11)
    st0, e0, s0 = d2d.d2d_lanczos(prob.sb, opts, None)
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.splitmix_normal(n, 11)).to("cuda")
    ctx.stream.synchronize()
    st1, e1, s1 = d2d.d2d_lanczos(prob.sb, opts, v0)
    print("seeded", e0, e1, s0["restarts"], s1["restarts"])
    assert st0 == 0 and st1 == 0
    assert abs(e0 - E0) <= 1e-10 * abs(E0)
    assert abs(e0 - e1) <= 1e-12 * abs(E0)
    assert abs(s0["log_theta"][0] - s1["log_theta"][0]) <= 1e-12 * abs(s1["log_theta"][0])
    prob.close()


def test_energy_change_stop(ctx):
    """tol_rel_e: stop on successive FP64 Rayleigh quotients (residual bar out of reach)."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl)
    E0 = reference_energy(wl.name)
    n = prob.info["n"]
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(n, wl.seed)).to("cuda")
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=1, k_in=24, max_restarts=300, tol_res=1e-300, reorth_window=3, tol_rel_e=1e-13)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
    th = stats["log_theta"]
    print("tol_rel_e", e, stats["restarts"], th[-2:], stats["residual"])
    assert st == 0
    assert abs(th[-1] - th[-2]) <= 1e-13 * abs(th[-1])
    assert abs(e - E0) <= 1e-10 * abs(E0)
    prob.close()


def test_no_escalation_when_the_krylov_space_is_slow(ctx):
    """Poor progress alone does not raise the precision: with the threshold at
    1e-6 every restart counts as poor, but on this workload the BF16 restarts
    lower the Rayleigh quotient and reach the residual the recurrence
    predicts, so BF16 is kept to the end."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(prob.info["n"], wl.seed)).to("cuda")
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=2, k_in=24, max_restarts=300, tol_res=1e-8, reorth_window=3, escalate=1e-6,
                            fixed_cycles=1)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
    E0 = reference_energy(wl.name)
    ratios = [r / max(p, 1e-300) for r, p in zip(stats["log_rho"][1:], stats["log_pred"][1:])]
    print("no escalation", set(stats["log_prec"]), stats["hv_count"], e, "true/pred", ratios)
    assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    assert set(stats["log_prec"]) == {2}
    assert stats["hv_count"][3] == 0 and stats["hv_count"][1] == 0
    assert stats["log_pred"][0] == 0.0 and all(p > 0 for p in stats["log_pred"][1:])
    prob.close()


def test_escalation_from_bf16_on_a_rising_energy(ctx):
    """A 12-site ladder (dimension 924) in BF16 with an FP64 inner basis: a
    restart's Ritz vector has a higher FP64 Rayleigh quotient than its start,
    which only the BF16 error can cause, so the precision moves on to BF16x3;
    the energy still meets the bar.  (With an FP32 basis this seed's BF16
    restarts happen not to rise, and the solve stays in BF16.)"""
    from paper_0707_0159_amd import d2d
    wl = W.batch64(6)[15]       # the 6-column variant of batch problem 15: 924 states
    prob = GpuProblem(ctx, wl, prec_mask=15)
    assert prob.info["n"] == 924
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(prob.info["n"], wl.seed)).to("cuda")
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=2, k_in=24, max_restarts=300, tol_res=1e-8, reorth_window=3, basis=1,
                            fixed_cycles=1)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0)
    E0 = reference_energy(wl.name)
    seen = list(dict.fromkeys(stats["log_prec"]))
    th = stats["log_theta"]
    print("escalation", seen, stats["hv_count"], e, "theta", th)
    assert st == 0 and abs(e - E0) <= 1e-10 * abs(E0)
    assert seen[:2] == [2, 3]
    # entry j logs the precision of the restart that produced it; the decision
    # to escalate follows the entry before the first BF16x3 one
    first = stats["log_prec"].index(3)
    assert first >= 2 and th[first - 1] > th[first - 2]
    prob.close()


def test_ferromagnetic_sector_breakdown(ctx):
    """1-dimensional sector: the start vector is an eigenvector, rho = 0 at once."""
    wl = W.HEISENBERG_2X6_M16
    prob = GpuProblem(ctx, wl, target=(12, 0))
    assert prob.info["n"] == 1
    st, e, stats, psi = run(ctx, prob, 0, 3)
    assert st == 0 and abs(e - 4.0) < 1e-13        # J * 16 bonds / 4
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_graphs_replayed_across_calls(ctx, prec):
    """Restarts captured as hipGraphs by one d2d_lanczos call are replayed by
    the next calls on the same superblock (no new capture), with iterates bit
    for bit those of direct launches; a new launch configuration (another
    tile) is captured anew and still meets the energy."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    try:
        direct = run(ctx, prob, prec, wl.seed, k_in=48, graph=0, window=3, tol=1e-8)
        calls = [run(ctx, prob, prec, wl.seed, k_in=48, graph=1, window=3, tol=1e-8) for _ in range(3)]
        caps = [c[2]["graph_captures"] for c in calls]
        print("graph captures per call", prec, caps, "restarts", direct[2]["restarts"])
        assert caps[0] >= 1 and caps[1] == 0 and caps[2] == 0
        for st, e, stats, psi in calls:
            assert st == 0 and e == direct[1]
            assert np.array_equal(np.asarray(stats["log_theta"]), np.asarray(direct[2]["log_theta"]))
            assert np.array_equal(psi, direct[3])
        shape = [i for i, sh in enumerate(d2d.d2d_tile_shapes()) if sh[0] == prec][-1]
        d2d.d2d_sb_set_tile(prob.sb, prec, shape)
        st, e, stats, _ = run(ctx, prob, prec, wl.seed, k_in=48, graph=1, window=3, tol=1e-8)
        assert st == 0 and stats["graph_captures"] >= 1
        E0 = reference_energy(wl.name)
        assert abs(e - E0) <= 1e-10 * abs(E0)
    finally:
        d2d.d2d_sb_set_tile(prob.sb, prec, -1)
        prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_persistent_launch_in_captured_graphs(ctx, prec):
    """The inner steps' grouped launch as a persistent launch (D2D_TILE_PERSIST,
    central term fused, split K-loops) inside captured graphs replayed across
    calls: its counters are left zero by every launch, so every replay takes
    every work item, and the solve is bit for bit the plain launch's (same
    energy, restart log and Ritz vector)."""
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    prob = GpuProblem(ctx, wl, prec_mask=15)
    try:
        shape = [i for i, s in enumerate(d2d.d2d_tile_shapes()) if s[0] == prec][0]
        cfg = shape | d2d.D2D_TILE_SPLIT | d2d.D2D_TILE_FUSED
        d2d.d2d_sb_set_tile(prob.sb, prec, cfg)
        plain = run(ctx, prob, prec, wl.seed, k_in=48, graph=0, window=3, tol=1e-8)
        d2d.d2d_sb_set_tile(prob.sb, prec, cfg | d2d.D2D_TILE_PERSIST)
        calls = [run(ctx, prob, prec, wl.seed, k_in=48, graph=g, window=3, tol=1e-8) for g in (0, 1, 1)]
        print("persistent", prec, "restarts", plain[2]["restarts"], "captures",
              [c[2]["graph_captures"] for c in calls])
        assert calls[1][2]["graph_captures"] >= 1 and calls[2][2]["graph_captures"] == 0
        for st, e, stats, psi in calls:
            assert st == 0 and e == plain[1]
            assert np.array_equal(np.asarray(stats["log_theta"]), np.asarray(plain[2]["log_theta"]))
            assert np.array_equal(psi, plain[3])
        E0 = reference_energy(wl.name)
        assert abs(plain[1] - E0) <= 1e-10 * abs(E0)
    finally:
        d2d.d2d_sb_set_tile(prob.sb, prec, -1)
        prob.close()
