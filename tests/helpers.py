"""Test helpers: tiny hand-built graphs and an exact enumeration of walk
probabilities written from the paper's definitions in terms of graph distance
(Eq. 2) and edge labels (Eq. 1), independent of the oracle's code."""
from __future__ import annotations

import json
from fractions import Fraction
from pathlib import Path
from types import SimpleNamespace

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

GOLDEN = Path(__file__).resolve().parent / "golden"
END = 0xFFFFFFFF


def csr_from_edges(nv, edges, symmetric=True, weights=True, labels=True):
    """edges: iterable of (u, v, w, label).  Returns a namespace with the CSR
    arrays (rows sorted ascending)."""
    rows = [[] for _ in range(nv)]
    for (u, v, w, lab) in edges:
        rows[u].append((v, w, lab))
        if symmetric:
            rows[v].append((u, w, lab))
    off = [0]
    adj, ws, ls = [], [], []
    for r in rows:
        r.sort()
        for (v, w, lab) in r:
            adj.append(v)
            ws.append(w)
            ls.append(lab)
        off.append(len(adj))
    return SimpleNamespace(
        offsets=np.array(off, dtype=np.uint64), adj=np.array(adj, dtype=np.uint32),
        weights=np.array(ws, dtype=np.uint32) if weights else None,
        labels=np.array(ls, dtype=np.uint8) if labels else None,
        n_vertices=nv, n_edges=len(adj))


def tiny6(weighted=True, labelled=True):
    spec = json.loads((GOLDEN / "tiny6.json").read_text())
    return csr_from_edges(spec["n_vertices"], spec["edges"], weights=weighted,
                          labels=labelled), spec


def hop_distances(g) -> np.ndarray:
    """All-pairs hop distance on the directed CSR (scipy's BFS)."""
    nv = g.n_vertices
    rows = np.repeat(np.arange(nv), np.diff(g.offsets).astype(np.int64))
    m = csr_matrix((np.ones(g.n_edges), (rows, g.adj.astype(np.int64))), shape=(nv, nv))
    return shortest_path(m, directed=True, unweighted=True)


def chances(g, dist, algo, cur, prev, t, factors=(1, 1, 1), schema=()):
    """Relative chance of each neighbour of cur (section 2.1): weight times
    Eq. 2's value chosen by dist(prev, u), or times Eq. 1's label indicator."""
    b, e = int(g.offsets[cur]), int(g.offsets[cur + 1])
    out = []
    for i in range(b, e):
        u = int(g.adj[i])
        w = int(g.weights[i]) if g.weights is not None else 1
        if algo == "node2vec" and t > 0:
            dd = dist[prev, u]
            f = {0: factors[0], 1: factors[1], 2: factors[2]}.get(int(dd) if np.isfinite(dd) else -1, 0)
            w *= f
        elif algo == "metapath":
            w *= 1 if int(g.labels[i]) == schema[t % len(schema)] else 0
        out.append(w)
    return out


def path_distribution(g, algo, start, length, factors=(1, 1, 1), schema=()):
    """Exact probability of every length-`length` path row from `start`
    (early ends padded with END), as Fractions."""
    dist = hop_distances(g)
    res = {}

    def rec(path, p):
        t = len(path) - 1
        if t == length:
            res[tuple(path)] = res.get(tuple(path), 0) + p
            return
        cur = path[-1]
        prev = path[-2] if t > 0 else None
        c = chances(g, dist, algo, cur, prev, t, factors, schema)
        tot = sum(c)
        if tot == 0:
            row = tuple(path + [END] * (length - t))
            res[row] = res.get(row, 0) + p
            return
        b = int(g.offsets[cur])
        for i, ci in enumerate(c):
            if ci:
                rec(path + [int(g.adj[b + i])], p * Fraction(ci, tot))

    rec([start], Fraction(1))
    return res


def chi2_pvalue(rows: np.ndarray, dist: dict) -> float:
    """Pearson chi-square of observed path rows against exact probabilities."""
    from scipy.stats import chisquare
    keys = list(dist.keys())
    index = {k: i for i, k in enumerate(keys)}
    counts = np.zeros(len(keys))
    for r in map(tuple, rows.tolist()):
        assert r in index, f"impossible path {r}"
        counts[index[r]] += 1
    n = rows.shape[0]
    exp = np.array([float(dist[k]) * n for k in keys])
    if len(keys) == 1:
        return 1.0
    return float(chisquare(counts, exp).pvalue)


def reservoir_pick(weights, rng) -> int:
    """Sequential weighted reservoir sampling (Algorithm 2, section 2.2):
    keep element i with probability W[i] / (W[1] + ... + W[i])."""
    total, sel = 0, -1
    for i, w in enumerate(weights):
        total += w
        if w and rng.random() < w / total:
            sel = i
    return sel
