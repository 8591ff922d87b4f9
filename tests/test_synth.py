"""The seeded input generators: determinism and CSR validity (CPU only)."""

import numpy as np
import pytest

import synth


def _check_simple_symmetric(g):
    n = g.n
    rp, ci = g.row_ptr, g.col_idx
    assert rp.dtype == np.int64 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    assert ci.min() >= 0 and ci.max() < n
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(rows == ci), "self-loop"
    key = rows.astype(np.int64) * n + ci
    assert np.all(np.diff(key) > 0), "rows must be sorted and duplicate-free"
    tkey = ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(tkey), key), "not symmetric"


def test_chung_lu_valid_and_deterministic():
    a = synth.chung_lu(5000, 25000, 2.5, seed=7)
    b = synth.chung_lu(5000, 25000, 2.5, seed=7, threads=3)
    c = synth.chung_lu(5000, 25000, 2.5, seed=8)
    _check_simple_symmetric(a)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
    assert not np.array_equal(a.col_idx[:100], c.col_idx[:100])
    assert np.all(a.degrees > 0), "isolated nodes must be dropped"
    assert abs(a.nnz / 2 / 25000 - 1) < 0.01


def test_chung_lu_power_law_shape():
    g = synth.chung_lu(100_000, 850_000, 2.3, seed=3)
    d = g.degrees
    # hub degree near the structural cutoff sqrt(2m)
    assert 0.3 * np.sqrt(g.nnz) < d.max() < 3 * np.sqrt(g.nnz)
    # complementary CDF slope ~ -(gamma - 1) over the middle decades
    xs = np.array([30, 60, 120, 240])
    ccdf = np.array([(d >= x).mean() for x in xs])
    slope = np.polyfit(np.log(xs), np.log(ccdf), 1)[0]
    assert -1.8 < slope < -0.9, slope


def test_weight_order_relabel():
    g = synth.chung_lu(3000, 15000, 2.5, seed=1, relabel="none")
    d = g.degrees
    # heaviest nodes first: the first 1% hold far more than 1% of the arcs
    assert d[:30].sum() > 0.05 * d.sum()


def test_small_graphs():
    for g in (synth.star(4), synth.cycle(6), synth.path(5), synth.complete(5),
              synth.erdos_renyi(30, 0.2, seed=1), synth.barbell_with_tail(4, 3)):
        _check_simple_symmetric(g)
    assert list(synth.star(3).degrees) == [3, 1, 1, 1]


def test_splitmix_matches_native():
    lib = synth._load()
    for seed, ctr in [(0, 0), (1, 5), (2**63 + 11, 123456789)]:
        assert synth.splitmix64_at(seed, ctr) == lib.synth_splitmix64_at(seed, ctr)
    # published first output of SplitMix64 seeded with 0
    assert synth.splitmix64_at(0, 0) == 0xE220A8397B1DCDAF


def test_sources_and_tolerances():
    g = synth.chung_lu(2000, 8000, 2.5, seed=2)
    s1 = synth.sources(g, 16, seed=5)
    assert np.array_equal(s1, synth.sources(g, 16, seed=5))
    assert np.all(g.degrees[s1] > 0)
    tol = synth.tolerance_choice(3, 64, [1e-4, 1e-6, 1e-7])
    assert set(np.unique(tol)) <= {1e-4, 1e-6, 1e-7} and len(np.unique(tol)) == 3
    lt = synth.tolerance_loguniform(4, 1000, 1e-7, 1e-4)
    assert lt.min() >= 1e-7 and lt.max() <= 1e-4


def test_bad_parameters():
    with pytest.raises(RuntimeError):
        synth.chung_lu(1, 10, 2.5, seed=1)
