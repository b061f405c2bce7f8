"""Input generators (CPU): CSR well-formed, symmetric, deterministic in the
seed and independent of the thread count; attributes symmetric per edge."""
import os

import numpy as np
import pytest

import oracle
import synth


def _sym_check(g):
    off, adj = g.offsets.astype(np.int64), g.adj.astype(np.int64)
    src = np.repeat(np.arange(g.n_vertices), np.diff(off))
    key = src * g.n_vertices + adj
    rkey = adj * g.n_vertices + src
    assert np.array_equal(np.sort(key), np.sort(rkey))
    assert not np.any(src == adj)
    return src


@pytest.mark.parametrize("permute", [False, True])
def test_rmat_wellformed(permute):
    g = synth.rmat(10, 8, seed=3, permute=permute)
    assert oracle.validate(g) == oracle.OK
    _sym_check(g)


def test_chung_lu_wellformed():
    g = synth.chung_lu(5000, 40000, 2.1, 4.0, seed=9)
    assert oracle.validate(g) == oracle.OK
    _sym_check(g)
    d = g.degrees()
    assert d.max() > 20 * max(d.mean(), 1)


def test_deterministic_across_threads(monkeypatch):
    monkeypatch.setenv("FW_SYNTH_THREADS", "1")
    a = synth.rmat(11, 4, seed=5)
    wa = synth.weights_zipf(a, 1.2, 65535, 3)
    monkeypatch.setenv("FW_SYNTH_THREADS", "7")
    b = synth.rmat(11, 4, seed=5)
    wb = synth.weights_zipf(b, 1.2, 65535, 3)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.adj, b.adj)
    assert np.array_equal(wa, wb)


def test_attributes_symmetric_and_in_range():
    g = synth.rmat(10, 8, seed=4)
    src = np.repeat(np.arange(g.n_vertices), np.diff(g.offsets).astype(np.int64))
    for w in (synth.weights_uniform(g, 1, 255, 1), synth.weights_zipf(g, 1.2, 65535, 2),
              synth.labels_uniform(g, 5, 3)):
        key = np.minimum(src, g.adj) * g.n_vertices + np.maximum(src, g.adj)
        order = np.argsort(key, kind="stable")
        ks, ws = key[order], w[order]
        pairs = ks[0::2] == ks[1::2]
        assert pairs.all() and np.array_equal(ws[0::2], ws[1::2])
    u = synth.weights_uniform(g, 1, 255, 1)
    assert u.min() >= 1 and u.max() <= 255
    lab = synth.labels_uniform(g, 5, 3)
    assert set(np.unique(lab).tolist()) == {0, 1, 2, 3, 4}


def test_zipf_tail_mass():
    """Zipf(1.2) clipped at 65535: P(k >= 65535) = zeta(1.2, 65535)/zeta(1.2)
    (about 9.7%) and P(k = 1) = 1/zeta(1.2)."""
    from scipy.special import zeta
    g = synth.rmat(14, 16, seed=8)
    w = synth.weights_zipf(g, 1.2, 65535, 4)
    n = w.shape[0] // 2
    tail = zeta(1.2, 65535) / zeta(1.2)
    one = 1 / zeta(1.2)
    assert abs((w == 65535).mean() - tail) < 5 * np.sqrt(tail * (1 - tail) / n)
    assert abs((w == 1).mean() - one) < 5 * np.sqrt(one * (1 - one) / n)


def test_uniform_ids():
    ids = synth.uniform_ids(100000, 1000, 7)
    assert ids.max() < 1000
    from scipy.stats import chisquare
    assert chisquare(np.bincount(ids, minlength=1000)).pvalue > 1e-4
