"""Stream capture: cp_power, cp_power_batch and cp_propagate issue only
kernels (coefficients and ids travel as kernel arguments, zeroing is a fill
kernel) and no synchronisation without CP_Q_STATS / CP_Q_TIMING, so a caller
can record them into a HIP graph.  Each graph here is replayed several
times, with eager library work and synchronisations between the replays,
and every replay must equal the eager result bit for bit.  Each Graph
object keeps one workspace, so each capture uses its own Graph object (the
captured workspace must stay allocated while the HIP graph lives)."""

import pytest

import synth
from gpu_util import gpu_graph, require_gpu

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def graph():
    return synth.chung_lu(60_000, 500_000, 2.3, seed=19)


def _replays(torch, hg, outs, refs, eager):
    for rep in range(4):
        for o in outs:
            o.fill_(-7.0)
        eager()  # other library work on the eager stream between replays
        torch.cuda.synchronize()
        hg.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r), rep


@pytest.mark.parametrize("stripes", [False, True])
def test_capture_single_source(torch, graph, stripes):
    g = graph
    srcs = [int(s) for s in synth.sources(g, 3, seed=5)]
    G = gpu_graph(g, stripes=stripes, reorder=not stripes)
    other = gpu_graph(g)
    y1 = torch.empty(g.n, dtype=torch.float32, device="cuda")
    y2 = torch.empty(g.n, dtype=torch.float32, device="cuda")
    ref1 = G.power("hkpr", 5.0, srcs[0], tol=1e-7, prec="f32", y=y1).y.clone()
    ref2 = G.power("ppr", 0.15, srcs[1], tol=1e-7, prec="f32", y=y2).y.clone()
    _case("capture single", stripes)
    hg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hg):
        st = torch.cuda.current_stream().cuda_stream
        G.power("hkpr", 5.0, srcs[0], tol=1e-7, prec="f32", y=y1, stream=st)
        G.power("ppr", 0.15, srcs[1], tol=1e-7, prec="f32", y=y2, stream=st)
    _replays(torch, hg, [y1, y2], [ref1, ref2],
             lambda: other.power("ppr", 0.2, srcs[2], tol=1e-6, prec="f32"))


def test_capture_batch_and_propagate(torch, graph):
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    srcs = [int(s) for s in synth.sources(g, 21, seed=6)]
    qs = [cp.make_query("ppr" if i % 2 else "hkpr", 0.2 if i % 2 else 3.0, s, 1e-7,
                        method="power" if i % 3 == 2 else "cheby") for i, s in enumerate(srcs)]
    Gb = gpu_graph(g, reorder=True)
    Gp = gpu_graph(g, reorder=True)
    other = gpu_graph(g)
    Gb.set_batch_width(len(qs), "f32", 16)
    Yb = torch.empty((g.n, len(qs)), dtype=torch.float32, device="cuda")
    refb = Gb.power_batch(qs, prec="f32", Y=Yb)[0].clone()
    X = (torch.rand((g.n, 9), generator=torch.Generator().manual_seed(3), dtype=torch.float32) - 0.5).cuda()
    Z = torch.empty_like(X)
    refz = Gp.propagate(X, "ppr", 0.1, a=0.5, kmode="fixed", K=12, prec="f32", Z=Z, method="clenshaw")[0].clone()
    _case("capture batch + propagate")
    hb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hb):
        st = torch.cuda.current_stream().cuda_stream
        Gb.power_batch(qs, prec="f32", Y=Yb, stream=st)
        Gp.propagate(X, "ppr", 0.1, a=0.5, kmode="fixed", K=12, prec="f32", Z=Z, method="clenshaw", stream=st)
    _replays(torch, hb, [Yb, Z], [refb, refz],
             lambda: other.power_batch(qs[:5], prec="f32"))
