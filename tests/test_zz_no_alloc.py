"""cp_power_noalloc (the workspace is the library's static device array)
against cp_power (caller workspace), through the C ABI: bitwise equal
results on two calls in a row, the second on a smaller graph, for the
single-CSR and XCD-striped layouts in FP64, FP32 (double and float
arithmetic) and BF16; a graph whose
workspace exceeds the array is refused with CP_EWORKSPACE, and CP_Q_TIMING
with CP_EINVAL."""

import numpy as np
import pytest

import synth
from gpu_util import gpu_graph, require_gpu

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("stripes", [False, True])
def test_noalloc_equals_power_on_two_calls_second_smaller(torch, stripes):
    from paper_2412_10789_amd import chebyprop as cp

    big = synth.chung_lu(300_000, 3_000_000, 2.1, seed=41)
    small = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    Gb, Gs = gpu_graph(big, stripes=stripes), gpu_graph(small, stripes=stripes)
    for prec in ("f64", "f32", "f32f", "bf16"):
        for g, G, s, kind, param in ((big, Gb, int(synth.sources(big, 1, seed=2)[0]), "hkpr", 5.0),
                                     (small, Gs, int(synth.sources(small, 1, seed=3)[0]), "ppr", 0.2)):
            _case("noalloc", stripes, prec, g.n, kind, s)
            ref = G.power(kind, param, s, tol=1e-7, prec=prec, flags=cp.CP_Q_STATS)
            y = torch.full((g.n,), -7.0, dtype=ref.y.dtype, device="cuda")
            info = G.power_noalloc(kind, param, s, y, tol=1e-7, prec=prec, flags=cp.CP_Q_STATS)
            torch.cuda.synchronize()
            assert info["K"] == ref.info["K"] and info["steps"] == ref.info["steps"]
            assert info["mass"] == ref.info["mass"]
            assert torch.equal(y, ref.y), (stripes, prec, g.n)
    Gb.close()
    Gs.close()


def test_noalloc_limits(torch):
    from paper_2412_10789_amd import chebyprop as cp

    # a graph whose FP64 workspace exceeds the static array: 3M isolated nodes around a small core
    core = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    n = 3_000_000
    rp = np.concatenate([core.row_ptr, np.full(n - core.n, core.nnz, dtype=np.int64)])
    G = cp.Graph(rp, core.col_idx)
    s = int(synth.sources(core, 1, seed=3)[0])
    assert 3 * 8 * n > cp.CP_NOALLOC_SCRATCH_BYTES > 16 * n + (1 << 20)  # FP64 vectors do not fit, FP32 do
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    _case("noalloc too large")
    with pytest.raises(cp.ChebypropError) as ei:
        G.power_noalloc("ppr", 0.2, s, y, prec="f64")
    assert ei.value.status == cp.CP_EWORKSPACE
    # FP32 fits (16 bytes per node): the same query runs
    y32 = torch.empty(n, dtype=torch.float32, device="cuda")
    _case("noalloc f32 3M nodes")
    G.power_noalloc("ppr", 0.2, s, y32, prec="f32")
    ref = G.power("ppr", 0.2, s, prec="f32")
    assert torch.equal(y32, ref.y)
    with pytest.raises(cp.ChebypropError) as ei:
        G.power_noalloc("ppr", 0.2, s, y32, prec="f32", flags=cp.CP_Q_TIMING)
    assert ei.value.status == cp.CP_EINVAL
    G.close()
