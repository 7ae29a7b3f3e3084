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


def run(ctx, prob, prec, seed, k_in=24, graph=1, tol=1e-9):
    from paper_0707_0159_amd import d2d
    n = prob.info["n"]
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(n, seed)).to("cuda")
        psi = torch.zeros_like(v0)
    ctx.stream.synchronize()
    opts = d2d.lanczos_opts(prec=prec, k_in=k_in, max_restarts=300, tol_res=tol, use_graph=graph)
    st, e, stats = d2d.d2d_lanczos(prob.sb, opts, v0, psi)
    ctx.stream.synchronize()
    return st, e, stats, psi.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("graph", [0, 1])
def test_config1_energy(ctx, prec, graph):
    wl = W.CONFIGS[1]
    prob = GpuProblem(ctx, wl)
    st, e, stats, psi = run(ctx, prob, prec, wl.seed, graph=graph)
    E0 = reference_energy(wl.name)
    print("config1", prec, graph, e, E0, stats["restarts"], stats["hv_count"])
    assert st == 0
    assert abs(e - E0) <= 1e-10 * abs(E0)
    # psi is an eigenvector of the oracle's operator
    osb = oracle_superblock(wl)
    r = osb.hv_explicit(psi) - e * psi
    assert np.linalg.norm(r) <= 1e-8 * abs(E0)
    prob.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_config2_energy(ctx, prec):
    wl = W.CONFIGS[2]
    prob = GpuProblem(ctx, wl, prec_mask=7)
    st, e, stats, psi = run(ctx, prob, prec, wl.seed)
    E0 = reference_energy(wl.name)
    print("config2", prec, e, E0, (e - E0) / abs(E0), stats["restarts"], stats["hv_count"], stats["seconds"])
    assert st == 0
    assert abs(e - E0) <= 1e-10 * abs(E0)
    assert e >= E0 - 1e-10 * abs(E0)          # Rayleigh quotient is variational
    prob.close()


def test_ferromagnetic_sector_breakdown(ctx):
    """1-dimensional sector: the start vector is an eigenvector, rho = 0 at once."""
    wl = W.CONFIGS[1]
    prob = GpuProblem(ctx, wl, target=(12, 0))
    assert prob.info["n"] == 1
    st, e, stats, psi = run(ctx, prob, 0, 3)
    assert st == 0 and abs(e - 4.0) < 1e-13        # J * 16 bonds / 4
    prob.close()
