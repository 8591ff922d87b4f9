"""Host-side parts of bench.py: the algorithmic byte counts of the roofline,
the validity rule of the committed counter traffic, and the one-GPU
contract (more GPUs exit with a message before anything touches a GPU)."""

import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_step_bytes_per_precision():
    b = _bench()
    n, nnz = 1000, 17000
    # column ids + row offsets + per node five vector terms at the storage
    # width: gather, z read + write, estimate read + write
    assert b.step_bytes(n, nnz, "f32") == 4 * nnz + 8 * (n + 1) + 5 * n * 4
    assert b.step_bytes(n, nnz, "f64") == 4 * nnz + 8 * (n + 1) + 5 * n * 8
    assert b.step_bytes(n, nnz, "bf16") == 4 * nnz + 8 * (n + 1) + 5 * n * 2
    # batched: the index stream is shared, the vector terms scale with sources
    assert b.step_bytes(n, nnz, "f32", 64) - b.step_bytes(n, nnz, "f32", 0) == 64 * n * 20
    # the implementation keeps a double estimate for FP32 storage
    assert b.impl_step_bytes(n, nnz, "f32") == 4 * nnz + 8 * (n + 1) + n * (3 * 4 + 2 * 8)
    assert b.impl_step_bytes(n, nnz, "bf16") == b.step_bytes(n, nnz, "bf16") + n * 2 * 2
    # Clenshaw: no estimate stream, one read of the start vector
    assert b.clenshaw_step_bytes(n, nnz, "f32", 8) == 4 * nnz + 8 * (n + 1) + 8 * n * 4 * 4


def test_batch_launch_bytes_count_active_sources():
    b = _bench()
    n, nnz = 1000, 17000
    Ks = [3, 5, 5]
    # launches k = 1..4: sources with K > k are active: 3, 3, 2, 2
    want = sum(b.step_bytes(n, nnz, "f32", a) for a in (3, 3, 2, 2))
    assert b.batch_launch_bytes(n, nnz, "f32", Ks) == want


def test_roofline_fraction():
    b = _bench()
    r = b.roofline(8e9, 2.0, "k")  # 8 GB in 2 ms = 4 TB/s
    assert r["achieved"] == 4000.0 and r["frac"] == 0.5 and r["peak"] == 8000.0 and r["bound"] == "hbm"


def test_traffic_only_for_current_kernels():
    b = _bench()
    with open(os.path.join(ROOT, "profiles", "step_traffic.json")) as fh:
        rec = json.load(fh)
    for key, e in rec.items():
        files = b.BATCH_SOURCES if key.endswith(":batch") else b.SINGLE_SOURCES
        got = b.measured_traffic(key, files)
        if e["kernel_hash"] == b.kernel_hash(files):
            assert got == e["bytes_per_launch"] and got > 0
        else:
            assert got is None
    assert b.measured_traffic("no such workload") is None


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_oracle_checks_run_on_mixed_queries():
    """The bench's accuracy helpers on a small graph: the converged vectors
    of PPR (small alpha) and HKPR (large t) queries, with either rule for
    PPR, match each other and the certificate; checks of exact inputs report
    errors at rounding level and the certificate bounds the PPR error."""
    import numpy as np

    import synth

    b = _bench()
    b.np = np
    g = synth.chung_lu(5_000, 30_000, 2.3, seed=3)
    srcs = [int(s) for s in synth.sources(g, 4, seed=4)]
    kinds, params = ["ppr", "hkpr", "ppr", "hkpr"], [0.1, 10.0, 0.2, 3.0]
    e1 = b.exact_vectors(g, kinds, params, srcs)
    e2 = b.exact_vectors(g, kinds, params, srcs, chebyshev_for_ppr=True)
    assert np.abs(e1 - e2).sum(axis=0).max() <= 1e-11
    Ks = [40, 30, 30, 20]
    rows, _ = b.check_same_k_and_exact(g, e1, kinds, params, srcs, Ks, chebyshev_for_ppr=True)
    for r in rows:
        assert r["l1_vs_exact"] <= 1e-11 and abs(r["mass"] - 1.0) <= 1e-11
        assert r["l1_vs_same_K"] <= 1e-4  # the truncated series at these K
    cert, _ = b.check_ppr_certificate(g, e1[:, [0, 2]], [srcs[0], srcs[2]], [0.1, 0.2])
    assert all(c["l1_bound_vs_exact"] <= 1e-9 for c in cert)
