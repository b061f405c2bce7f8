"""The regrouping of Eq. 2 that the persistent node2vec walker uses when
N(prev) is much shorter than N(cur) (CPU): for every group of consecutive
entries of N(cur),

    T_g = f_out * sum(w_i) + (f_in - f_out) * sum(w_i : u_i in N(prev), u_i != prev)
                           + (f_ret - f_out) * sum(w_i : u_i == prev)

computed modulo 2^64, where the middle sum takes every entry of N(cur)
whose id occurs in N(prev) (once per entry of N(cur), however often the id
repeats in N(prev)).  Checked against the oracle's per-entry transition
weights on rows with parallel edges, self-loops and prev repeated, for
factors that make f_in - f_out and f_ret - f_out negative."""
import numpy as np
import pytest

import oracle
from helpers import csr_from_edges

M64 = (1 << 64) - 1


def _graph(seed):
    rng = np.random.default_rng(seed)
    cur, prev, nv = 0, 1, 400
    edges = [(cur, int(v), int(rng.integers(1, 60_000)), 0) for v in rng.integers(2, nv, 300)]
    edges += [(cur, prev, 7, 0), (cur, prev, 9, 0), (cur, cur, 4, 0)]      # prev twice, self-loop
    edges += [(prev, int(v), 1, 0) for v in rng.integers(2, nv, 40)]       # repeats likely
    edges += [(prev, prev, 3, 0), (prev, cur, 5, 0)]
    return csr_from_edges(nv, edges, labels=False), cur, prev


def _regrouped(g, cur, prev, f, gsz):
    o, e = int(g.offsets[cur]), int(g.offsets[cur + 1])
    po, pe = int(g.offsets[prev]), int(g.offsets[prev + 1])
    ids, w = g.adj[o:e].astype(np.int64), g.weights[o:e].astype(np.int64)
    in_prev = set(int(x) for x in g.adj[po:pe]) - {prev}
    f_ret, f_in, f_out = f
    out = []
    for b in range(0, e - o, gsz):
        gi, gw = ids[b:b + gsz], w[b:b + gsz]
        t = (f_out * int(gw.sum())) & M64
        t = (t + ((f_in - f_out) & M64) * int(gw[np.isin(gi, list(in_prev))].sum())) & M64
        t = (t + ((f_ret - f_out) & M64) * int(gw[gi == prev].sum())) & M64
        out.append(t)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("f", [(1, 2, 4), (4, 2, 1), (3, 0, 5), (0, 7, 2), (2, 2, 1)])
@pytest.mark.parametrize("gsz", [1, 7, 64, 1000])
def test_regrouped_group_totals_equal_the_oracle(seed, f, gsz):
    g, cur, prev = _graph(seed)
    wts = oracle.transition_weights(g, "node2vec", oracle.params(*f), prev, cur, 1)
    exp = [int(wts[b:b + gsz].sum()) for b in range(0, len(wts), gsz)]
    assert _regrouped(g, cur, prev, f, gsz) == exp
