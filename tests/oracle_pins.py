"""Pins of the CPU oracle to things other than itself.

Each pin checks the oracle against a fact fixed outside its code: a published
Philox known answer and numpy's independent Philox implementation; closed
forms for the 64-bit scaling computed with Python integers; brute-force
enumeration for the inverse-CDF pick; hand-worked transition weights; exact
path distributions computed from graph distances (scipy's BFS) for Eq. 2 and
from labels for Eq. 1, against which 10^6 oracle draws are chi-square tested;
algorithm identities; and walk invariants.  The same pins run against planted
mistakes in the oracle (test_oracle_mutants) to show that they catch them.
"""
from __future__ import annotations

import numpy as np

import oracle
from helpers import END, chi2_pvalue, csr_from_edges, path_distribution, tiny6

M64 = (1 << 64) - 1


def _numpy_philox_block(ctr, key):
    """numpy's Philox increments its 256-bit counter before each block, so
    start it one below."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & M64 for i in range(4)]
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                         counter=np.array(words, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


def pin_philox_kat():
    # Published known answer for Philox4x64-10 at counter 0, key 0 (Random123
    # distribution of Salmon et al., SC 2011).
    got = [int(x) for x in oracle.philox4x64_10([0, 0, 0, 0], [0, 0])]
    assert got == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B,
                   0x7E68B68AEC7BA23B], [hex(x) for x in got]


def pin_philox_numpy(cases=200):
    rng = np.random.default_rng(7)
    for i in range(cases):
        ctr = [int(x) for x in rng.integers(0, 1 << 63, 4, dtype=np.uint64)]
        if i % 4 == 0:
            ctr[2] = ctr[3] = 0
        if i % 5 == 0:
            ctr[0] = M64
        key = [int(x) for x in rng.integers(0, 1 << 63, 2, dtype=np.uint64)]
        got = [int(x) for x in oracle.philox4x64_10(ctr, key)]
        assert got == _numpy_philox_block(ctr, key), (ctr, key)


def pin_draw_keying(cases=100):
    """The step draw is word 0 of the block at counter (qid, t, 0, 0) and key
    (seed, 0)."""
    rng = np.random.default_rng(11)
    for _ in range(cases):
        seed, qid, t = (int(x) for x in rng.integers(0, 1 << 40, 3))
        t %= 1000
        assert oracle.draw(seed, qid, t) == _numpy_philox_block([qid, t, 0, 0], [seed, 0])[0]


def pin_scale_closed_form():
    """floor(u*T/2^64) == r exactly on the interval [ceil(r 2^64 / T),
    ceil((r+1) 2^64 / T)), whose length is floor or ceil of 2^64/T."""
    rng = np.random.default_rng(3)
    totals = [1, 2, 3, 5, 7, 255, 1 << 20, (1 << 38) + 12345, (1 << 63) + 1, M64]
    totals += [int(x) for x in rng.integers(1, 1 << 62, 20, dtype=np.uint64)]
    two64 = 1 << 64
    for T in totals:
        for r in {0, 1, T // 2, T - 1, int(rng.integers(0, 1 << 62)) % T}:
            if r >= T:
                continue
            lo = -(-r * two64 // T)
            hi = -(-(r + 1) * two64 // T)
            assert hi - lo in (two64 // T, -(-two64 // T))
            assert oracle.scale(lo, T) == r, (T, r)
            assert oracle.scale(hi - 1, T) == r, (T, r)
            if lo > 0:
                assert oracle.scale(lo - 1, T) == r - 1, (T, r)
        assert oracle.scale(M64, T) == T - 1
        assert oracle.scale(0, T) == 0


def pin_pick_bruteforce():
    """Enumerating every r in [0, T) hits index i exactly w_i times, and
    index order follows r (inverse CDF in list order)."""
    rng = np.random.default_rng(5)
    vectors = [[1], [3], [0, 2], [2, 0], [1, 1, 1], [0, 0, 5, 0], [4, 0, 0, 1, 3]]
    vectors += [list(rng.integers(0, 20, int(rng.integers(1, 40)))) for _ in range(30)]
    for w in vectors:
        T = int(sum(w))
        if T == 0:
            assert oracle.pick(w, 0) == -1
            continue
        picks = [oracle.pick(w, r) for r in range(T)]
        assert picks == sorted(picks)
        counts = np.bincount(picks, minlength=len(w))
        assert counts.tolist() == [int(x) for x in w], (w, counts)
        assert oracle.pick(w, T) == -1


def _prm(case):
    if case["algo"] == "node2vec":
        return oracle.params(*case["factors"])
    if case["algo"] == "metapath":
        return oracle.params(schema=case["schema"])
    return oracle.params()


def pin_hand_weights():
    for case in tiny6()[1]["cases"]:
        g, _ = tiny6(weighted=case["weighted"])
        prev = case["prev"] if case["prev"] is not None else 0xFFFFFFFF
        got = oracle.transition_weights(g, case["algo"], _prm(case), prev, case["cur"], case["t"])
        assert got.tolist() == case["expect"], (case, got)


def _chi2_case(g, algo, start, length, factors=(1, 1, 1), schema=(), n=1_000_000, seed=2024):
    dist = path_distribution(g, algo, start, length, factors, schema)
    prm = oracle.params(*factors, schema=schema)
    rows = oracle.walk(g, algo, prm, np.full(n, start, dtype=np.uint32), length, seed)
    p = chi2_pvalue(rows, dist)
    assert p > 1e-4, (algo, start, length, factors, schema, p)
    return p


def pin_chi2_paths(n=1_000_000):
    """10^6 oracle walks of length 3 from one start (query ids 0..n-1 give
    independent draws) against the exact path distribution."""
    g, _ = tiny6()
    _chi2_case(g, "deepwalk", 0, 3, n=n)
    _chi2_case(g, "node2vec", 2, 3, factors=(1, 2, 4), n=n)
    _chi2_case(g, "node2vec", 3, 3, factors=(4, 2, 1), n=n)
    _chi2_case(g, "metapath", 1, 3, schema=(0, 1), n=n)
    gu, _ = tiny6(weighted=False)
    _chi2_case(gu, "metapath", 3, 3, schema=(1, 0, 2), n=n)


def _python_walk(g, dist, algo, start, qid, length, seed, factors, schema):
    """A walk rebuilt from independent parts: numpy's Philox for the draw,
    Python integers for the scaling, chances from graph distances/labels."""
    from helpers import chances
    row = [start]
    for t in range(length):
        cur = row[-1]
        prev = row[-2] if t > 0 else None
        c = chances(g, dist, algo, cur, prev, t, factors, schema)
        tot = sum(c)
        if tot == 0:
            return row + [END] * (length - t)
        u = _numpy_philox_block([qid, t, 0, 0], [seed, 0])[0]
        r = (u * tot) >> 64
        acc = 0
        for i, ci in enumerate(c):
            acc += ci
            if acc > r:
                break
        row.append(int(g.adj[int(g.offsets[cur]) + i]))
    return row


def pin_walk_rebuilt():
    """Whole walks equal the rebuilt ones, for query ids with an offset."""
    from helpers import hop_distances
    g, _ = tiny6()
    dist = hop_distances(g)
    seed, L, base = 123456789, 6, 1000
    starts = np.arange(40, dtype=np.uint32) % 6
    for algo, f, sch in [("deepwalk", (1, 1, 1), ()), ("node2vec", (1, 2, 4), ()),
                         ("metapath", (1, 1, 1), (0, 1))]:
        rows = oracle.walk(g, algo, oracle.params(*f, schema=sch), starts, L, seed,
                           qid_base=base)
        for i, s in enumerate(starts):
            exp = _python_walk(g, dist, algo, int(s), base + i, L, seed, f, sch)
            assert rows[i].tolist() == exp, (algo, i, rows[i], exp)



def pin_walk_ids_rebuilt():
    """Walks of a chosen list of query ids (the form behind every sampled
    parity check and the CPU baseline): row j is the walk of query qids[j]
    from starts[qids[j]], keyed by that id, rebuilt from independent parts,
    for a shuffled, non-contiguous id list whose start vertices differ from
    the ids; the threaded form returns the same rows in the same order."""
    from helpers import hop_distances
    g, _ = tiny6()
    dist = hop_distances(g)
    seed, L, n = 987654321, 5, 90
    starts = ((np.arange(n) * 5 + 3) % 6).astype(np.uint32)
    qids = np.random.default_rng(4).permutation(n)[:30].astype(np.uint64)
    for algo, f, sch in [("deepwalk", (1, 1, 1), ()), ("node2vec", (1, 2, 4), ()),
                         ("metapath", (1, 1, 1), (1, 0))]:
        prm = oracle.params(*f, schema=sch)
        rows = oracle.walk_ids(g, algo, prm, starts, qids, L, seed)
        for j, q in enumerate(qids):
            exp = _python_walk(g, dist, algo, int(starts[q]), int(q), L, seed, f, sch)
            assert rows[j].tolist() == exp, (algo, j, int(q), rows[j], exp)
        thr = oracle.walk_ids_threaded(g, algo, prm, starts, qids, L, seed, 4)
        assert np.array_equal(thr, rows), algo


def pin_walk_ids_rmat12():
    """On R-MAT-12 (node2vec p=2 q=1/2, 20 hops) the rows of a shuffled id
    list equal the same rows of the whole query set, single-threaded and
    threaded."""
    import synth
    g = synth.load_recipe_graph("rmat12_n2v", use_cache=False)
    n = g.n_vertices
    starts = ((np.arange(n, dtype=np.uint64) * 2654435761) % n).astype(np.uint32)
    prm = oracle.params(1, 2, 4)
    full = oracle.walk(g, "node2vec", prm, starts, 20, 42)
    qids = np.random.default_rng(8).permutation(n)[:700].astype(np.uint64)
    rows = oracle.walk_ids(g, "node2vec", prm, starts, qids, 20, 42)
    assert np.array_equal(rows, full[qids.astype(np.int64)])
    thr = oracle.walk_ids_threaded(g, "node2vec", prm, starts, qids, 20, 42, 8)
    assert np.array_equal(thr, rows)


def pin_identities():
    """node2vec with equal factors is DeepWalk; MetaPath whose schema matches
    every label is unit-weight DeepWalk; both bit-exact."""
    g, _ = tiny6()
    starts = np.arange(6, dtype=np.uint32).repeat(50)
    a = oracle.walk(g, "deepwalk", oracle.params(), starts, 12, 9)
    for f in [(1, 1, 1), (3, 3, 3)]:
        b = oracle.walk(g, "node2vec", oracle.params(*f), starts, 12, 9)
        assert np.array_equal(a, b), f
    gl = csr_from_edges(6, [(u, v, w, 3) for (u, v, w, _) in tiny6()[1]["edges"]],
                        weights=False)
    gu = csr_from_edges(6, tiny6()[1]["edges"], weights=False, labels=False)
    a = oracle.walk(gu, "deepwalk", oracle.params(), starts, 12, 9)
    b = oracle.walk(gl, "metapath", oracle.params(schema=[3]), starts, 12, 9)
    assert np.array_equal(a, b)


def pin_regular_uniform(n=200_000):
    """Unweighted DeepWalk on a k-regular graph picks each neighbour with
    probability 1/k (circulant graph C_12(1, 2, 5): 6-regular)."""
    nv, k = 12, 6
    edges = {tuple(sorted((i, (i + s) % nv))) for i in range(nv) for s in (1, 2, 5)}
    g = csr_from_edges(nv, [(u, v, 1, 0) for (u, v) in sorted(edges)], weights=False)
    rows = oracle.walk(g, "deepwalk", oracle.params(), np.zeros(n, np.uint32), 1, 77)
    counts = np.bincount(rows[:, 1], minlength=nv)
    nb = g.adj[int(g.offsets[0]):int(g.offsets[1])]
    assert set(np.nonzero(counts)[0].tolist()) == set(nb.tolist())
    from scipy.stats import chisquare
    assert chisquare(counts[nb]).pvalue > 1e-4
    assert len(nb) == k


def pin_path_graph_edges():
    """On a weighted path graph an interior vertex moves left with
    probability w_left / (w_left + w_right)."""
    edges = [(0, 1, 1, 0), (1, 2, 3, 0), (2, 3, 5, 0), (3, 4, 7, 0)]
    g = csr_from_edges(5, edges)
    n = 400_000
    rows = oracle.walk(g, "deepwalk", oracle.params(), np.full(n, 2, np.uint32), 1, 5)
    left = float((rows[:, 1] == 1).mean())
    assert abs(left - 3 / 8) < 5 * np.sqrt(3 / 8 * 5 / 8 / n)


def walk_invariants(g, algo, prm_tuple, starts, paths, schema=()):
    """path[0] = start; each hop is an edge; MetaPath hops carry the schema
    label; an early end happens exactly where no neighbour has positive
    chance (degree 0 for DeepWalk/node2vec with positive factors; no label
    match for MetaPath), and is padded to the end."""
    off, adj = g.offsets, g.adj
    L = paths.shape[1] - 1
    assert np.array_equal(paths[:, 0], np.asarray(starts, dtype=np.uint32))
    for row in paths:
        for t in range(L):
            cur, nxt = int(row[t]), int(row[t + 1])
            if cur == END:
                assert nxt == END
                continue
            b, e = int(off[cur]), int(off[cur + 1])
            nb = adj[b:e]
            if algo == "metapath":
                ok = g.labels[b:e] == schema[t % len(schema)]
                if g.weights is not None:
                    ok &= g.weights[b:e] > 0
            else:
                ok = np.ones(e - b, bool) if g.weights is None else g.weights[b:e] > 0
            if nxt == END:
                assert not ok.any(), (row, t)
            else:
                j = np.searchsorted(nb, nxt)
                assert j < e - b and nb[j] == nxt and ok[j], (row, t)


def pin_invariants_rmat12():
    import synth
    g = synth.load_recipe_graph("rmat12_n2v", use_cache=False)
    starts = np.arange(g.n_vertices, dtype=np.uint32)
    paths = oracle.walk(g, "node2vec", oracle.params(1, 2, 4), starts, 20, 42)
    walk_invariants(g, "node2vec", (1, 2, 4), starts, paths)
    labels = synth.labels_uniform(g, 5, 99)
    g.labels = labels
    sch = (0, 1, 2, 3, 4)
    paths = oracle.walk(g, "metapath", oracle.params(schema=sch), starts, 20, 42)
    walk_invariants(g, "metapath", None, starts, paths, schema=sch)


def pin_errors():
    g, _ = tiny6()
    ok = oracle.params(1, 2, 4)
    rc, _ = oracle.walk_status(g, "node2vec", ok, [6], 3, 1)
    assert rc == oracle.EINVAL
    rc, _ = oracle.walk_status(g, "node2vec", oracle.params(0, 0, 0), [0], 3, 1)
    assert rc == oracle.EINVAL
    gnl, _ = tiny6(labelled=False)
    rc, _ = oracle.walk_status(gnl, "metapath", oracle.params(schema=[0]), [0], 3, 1)
    assert rc == oracle.EINVAL
    rc, _ = oracle.walk_status(g, "metapath", oracle.params(), [0], 3, 1)
    assert rc == oracle.EINVAL
    big = csr_from_edges(3, [(0, 1, 0xFFFFFFFF, 0), (0, 2, 1, 0)])
    rc, _ = oracle.walk_status(big, "node2vec", oracle.params(0xFFFFFFFF, 1, 1), [0], 2, 1)
    assert rc == oracle.EOVERFLOW
    rc, _ = oracle.walk_status(big, "deepwalk", oracle.params(), [0], 2, 1)
    assert rc == oracle.OK
    bad = csr_from_edges(3, [(0, 1, 1, 0), (0, 2, 1, 0)])
    bad.adj = bad.adj[[1, 0, 2, 3]].copy()
    assert oracle.validate(bad) == oracle.EINVAL
    assert oracle.validate(g) == oracle.OK


def pin_zero_length_and_dead_ends():
    g, _ = tiny6()
    rows = oracle.walk(g, "deepwalk", oracle.params(), np.arange(6), 0, 1)
    assert rows.shape == (6, 1) and rows[:, 0].tolist() == list(range(6))
    # Schema (0, 1, 2) from vertex 1: hop 0 takes a label-0 edge to 0 or 2,
    # hop 1 a label-1 edge; from 0 that edge leads to 2, and no edge at 2
    # carries label 2, so those walks end at hop 2 and are padded.
    rows = oracle.walk(g, "metapath", oracle.params(schema=[0, 1, 2]),
                       np.full(2000, 1), 4, 3)
    assert set(rows[:, 1].tolist()) <= {0, 2}
    dead = (rows[:, 1] == 0) & (rows[:, 2] == 2)
    assert dead.any()
    assert (rows[dead, 3] == END).all() and (rows[dead, 4] == END).all()
    live = rows[:, 3] != END
    assert (rows[:, 3] != END).any()


def _stop_threshold(num, den):
    """PPR's coin stops exactly for the words u1 with u1 * den < num * 2^64,
    i.e. u1 < ceil(num * 2^64 / den) (Python integers)."""
    return -(-(num << 64) // den)


def pin_stop_coin_closed_form():
    rng = np.random.default_rng(5)
    for num, den in [(1, 5), (0, 1), (1, 1), (3, 7), (M64 >> 32, M64 >> 32), (1, M64 >> 32),
                     (4, 5), (123456, 999999)]:
        c = _stop_threshold(num, den)
        for u in {0, 1, c - 1, c, c + 1, M64, M64 - 1}:
            if 0 <= u <= M64:
                assert oracle.stop_coin(u, num, den) == (u < c), (num, den, u, c)
        for u in rng.integers(0, 1 << 63, 50, dtype=np.uint64):
            u = int(u) * 2 + 1
            assert oracle.stop_coin(u, num, den) == (u < c), (num, den, u)


def pin_stop_keying(cases=100):
    """PPR's coin is word 1 of the block at counter (qid, t, 0, 0), key
    (seed, 0) (numpy's Philox), the step draw word 0 of the same block."""
    rng = np.random.default_rng(13)
    for _ in range(cases):
        seed, qid, t = (int(x) for x in rng.integers(0, 1 << 40, 3))
        t %= 1000
        num, den = (1, 5) if qid % 2 else (2, 3)
        block = _numpy_philox_block([qid, t, 0, 0], [seed, 0])
        assert oracle.stop(seed, qid, t, num, den) == (block[1] < _stop_threshold(num, den))
        assert oracle.draw(seed, qid, t) == block[0]


def _python_ppr_walk(g, dist, start, qid, length, seed, stop):
    """A PPR walk rebuilt from independent parts: numpy's Philox (word 1 for
    the coin, word 0 for the draw), Python integers, DeepWalk chances."""
    from helpers import chances
    c = _stop_threshold(*stop)
    row = [start]
    for t in range(length):
        block = _numpy_philox_block([qid, t, 0, 0], [seed, 0])
        if block[1] < c:
            return row + [END] * (length - t)
        ch = chances(g, dist, "deepwalk", row[-1], None, t)
        tot = sum(ch)
        if tot == 0:
            return row + [END] * (length - t)
        r = (block[0] * tot) >> 64
        acc = 0
        for i, ci in enumerate(ch):
            acc += ci
            if acc > r:
                break
        row.append(int(g.adj[int(g.offsets[row[-1]]) + i]))
    return row


def pin_ppr_rebuilt():
    from helpers import hop_distances
    g, _ = tiny6()
    dist = hop_distances(g)
    seed, L, base = 987654321, 9, 77
    starts = np.arange(60, dtype=np.uint32) % 6
    for stop in [(1, 5), (1, 2), (2, 7)]:
        rows = oracle.walk(g, "ppr", oracle.params(stop=stop), starts, L, seed, qid_base=base)
        for i, s in enumerate(starts):
            exp = _python_ppr_walk(g, dist, int(s), base + i, L, seed, stop)
            assert rows[i].tolist() == exp, (stop, i, rows[i], exp)


def pin_ppr_length_distribution(n=200_000):
    """On a graph with no dead end the number of hops is geometric: k hops
    with chance (1 - a)^k a below the cap L, and (1 - a)^L at the cap."""
    from fractions import Fraction
    from scipy.stats import chisquare
    nv = 12
    edges = {tuple(sorted((i, (i + s) % nv))) for i in range(nv) for s in (1, 2, 5)}
    g = csr_from_edges(nv, [(u, v, 1 + (u * v) % 4, 0) for (u, v) in sorted(edges)])
    L, a = 12, Fraction(1, 5)
    rows = oracle.walk(g, "ppr", oracle.params(stop=(1, 5)), np.zeros(n, np.uint32), L, 4242)
    hops = (rows[:, 1:] != END).sum(axis=1)
    # the hops present form a prefix
    assert all((rows[i, 1:hops[i] + 1] != END).all() for i in range(0, n, 997))
    counts = np.bincount(hops, minlength=L + 1)
    exp = [float((1 - a) ** k * a) * n for k in range(L)] + [float((1 - a) ** L) * n]
    assert chisquare(counts, exp).pvalue > 1e-4, counts


def pin_ppr_limits():
    """Stop chance 0 is weighted DeepWalk bit for bit; stop chance 1 ends
    every query before its first hop; bad stop fractions are rejected."""
    g, _ = tiny6()
    starts = np.arange(6, dtype=np.uint32).repeat(40)
    a = oracle.walk(g, "deepwalk", oracle.params(), starts, 10, 31)
    b = oracle.walk(g, "ppr", oracle.params(stop=(0, 3)), starts, 10, 31)
    assert np.array_equal(a, b)
    c = oracle.walk(g, "ppr", oracle.params(stop=(3, 3)), starts, 10, 31)
    assert (c[:, 0] == starts).all() and (c[:, 1:] == END).all()
    for stop in [(1, 0), (4, 3)]:
        rc, _ = oracle.walk_status(g, "ppr", oracle.params(stop=stop), starts, 3, 1)
        assert rc == oracle.EINVAL, stop


def pin_entry_draw_keying(cases=100):
    """A reservoir sampler's word for entry i at hop t is word i mod 4 of the
    block at counter (qid, t, i div 4, 1), key (seed, 0) (numpy's Philox)."""
    rng = np.random.default_rng(17)
    for _ in range(cases):
        seed, qid, t, i = (int(x) for x in rng.integers(0, 1 << 40, 4))
        t %= 1000
        i %= 100_000
        block = _numpy_philox_block([qid, t, i // 4, 1], [seed, 0])
        assert oracle.entry_draw(seed, qid, t, i) == block[i % 4], (seed, qid, t, i)


def pin_zigzag_golden():
    import json
    from pathlib import Path
    cases = json.loads((Path(__file__).parent / "golden" / "zigzag_order.json").read_text())
    for c in cases["cases"]:
        assert oracle.zigzag_order(c["d"], c["k"]).tolist() == c["order"], c


def pin_reservoir_extremes():
    """Words 0 select every entry, so the last positive weight wins; words
    2^64 - 1 select only the first positive weight (floor((2^64-1) W / 2^64)
    = W - 1 < w only while W = w); no positive weight selects nothing."""
    rng = np.random.default_rng(19)
    for _ in range(200):
        d = int(rng.integers(1, 40))
        w = rng.integers(0, 4, d).astype(np.uint64)
        order = rng.permutation(d).astype(np.uint64)
        pos = [int(i) for i in order if w[int(i)] > 0]
        got0 = oracle.reservoir(w, np.zeros(d, np.uint64), order)
        gotm = oracle.reservoir(w, np.full(d, M64, np.uint64), order)
        assert got0 == (pos[-1] if pos else -1)
        assert gotm == (pos[0] if pos else -1)


def pin_reservoir_distribution(n=100_000):
    """Algorithm 2 picks entry i with chance w_i / T in any visiting order
    (Proposition 1), here with words from numpy's default generator."""
    from scipy.stats import chisquare
    w = np.array([3, 0, 5, 1, 7, 2, 0, 4], dtype=np.uint64)
    rng = np.random.default_rng(23)
    for order in [np.arange(8), np.array([5, 2, 7, 0, 4, 1, 6, 3])]:
        counts = np.zeros(8, dtype=np.int64)
        for _ in range(n):
            u = rng.integers(0, 1 << 63, 8, dtype=np.uint64) * np.uint64(2) + \
                rng.integers(0, 2, 8, dtype=np.uint64)
            counts[oracle.reservoir(w, u, order.astype(np.uint64))] += 1
        nz = w > 0
        assert counts[~nz].sum() == 0
        exp = w[nz].astype(np.float64) / float(w.sum()) * n
        assert chisquare(counts[nz], exp).pvalue > 1e-4, (order, counts)


def _hub_graph(d=700):
    """Vertex 0 joined to 1..d (varied weights), plus a ring over the leaves
    so that walks continue."""
    edges = [(0, i, 1 + (i * 37) % 50, 0) for i in range(1, d + 1)]
    edges += [(i, i % d + 1, 1 + i % 3, 0) for i in range(1, d + 1)]
    return csr_from_edges(d + 1, edges)


def _python_reservoir_walk(g, start, qid, length, seed, sampler, k=64):
    """Rebuilt from independent parts: numpy's Philox words, Python integers,
    the visiting order as a sort by (lane, quad, position)."""
    row = [start]
    for t in range(length):
        cur = row[-1]
        b, e = int(g.offsets[cur]), int(g.offsets[cur + 1])
        d = e - b
        w = [int(g.weights[b + i]) for i in range(d)]
        if sum(w) == 0:
            return row + [END] * (length - t)
        if sampler == "dprs":
            order = list(range(d))
        else:
            order = sorted(range(d), key=lambda i: ((i // 4) % k, i // 4, i % 4))
        sel, tot = -1, 0
        for i in order:
            if w[i] == 0:
                continue
            tot += w[i]
            u = _numpy_philox_block([qid, t, i // 4, 1], [seed, 0])[i % 4]
            if (u * tot) >> 64 < w[i]:
                sel = i
        row.append(int(g.adj[b + sel]))
    return row


def pin_reservoir_walks_rebuilt():
    g = _hub_graph()
    starts = np.array([0, 0, 0, 5, 0, 17, 0, 0], dtype=np.uint32)
    for sampler in ["dprs", "zprs"]:
        rows = oracle.walk(g, "deepwalk", oracle.params(), starts, 3, 55, qid_base=9,
                           sampler=sampler)
        for i, s in enumerate(starts):
            exp = _python_reservoir_walk(g, int(s), 9 + i, 3, 55, sampler)
            assert rows[i].tolist() == exp, (sampler, i, rows[i], exp)


def pin_reservoir_hop_distribution(n=150_000):
    """One hop from a 700-neighbour hub: both samplers pick neighbour i with
    chance w_i / T (chi-square), while ZPRS's picks differ from DPRS's."""
    from scipy.stats import chisquare
    g = _hub_graph()
    b, e = int(g.offsets[0]), int(g.offsets[1])
    w = g.weights[b:e].astype(np.float64)
    starts = np.zeros(n, dtype=np.uint32)
    got = {}
    for sampler in ["dprs", "zprs"]:
        rows = oracle.walk(g, "deepwalk", oracle.params(), starts, 1, 8, sampler=sampler)
        counts = np.bincount(rows[:, 1].astype(np.int64) - 1, minlength=e - b)
        assert chisquare(counts, w / w.sum() * n).pvalue > 1e-4, sampler
        got[sampler] = rows[:, 1]
    assert (got["dprs"] != got["zprs"]).mean() > 0.5


def pin_alias_golden():
    import json
    from pathlib import Path
    cases = json.loads((Path(__file__).parent / "golden" / "alias_table.json").read_text())
    for c in cases["cases"]:
        T, prob, alias = oracle.alias_table(c["w"])
        assert T == c["T"], c
        if T:
            assert prob.tolist() == c["prob"] and alias.tolist() == c["alias"], (c, prob, alias)


def pin_alias_mass_identity():
    """What makes an alias table exact: column c keeps prob[c] <= T of its
    own item and gives T - prob[c] to alias[c], so item i owns
    prob[i] + sum over {c != i : alias[c] = i} of (T - prob[c]) = w_i * n."""
    rng = np.random.default_rng(29)
    for trial in range(300):
        n = int(rng.integers(1, 300))
        kind = trial % 3
        if kind == 0:
            w = rng.integers(0, 10, n)
        elif kind == 1:
            w = np.floor(rng.lognormal(0, 2.5, n)).astype(np.int64)
        else:
            w = rng.integers(0, 1 << 32, n, dtype=np.uint64) * (rng.random(n) < 0.3)
        w = w.astype(np.uint32)
        T, prob, alias = oracle.alias_table(w)
        assert T == int(w.astype(np.uint64).sum())
        if T == 0:
            continue
        own = [int(p) for p in prob]
        assert max(own) <= T and min(own) >= 0
        mass = own[:]
        for c in range(n):
            if int(alias[c]) != c:
                mass[int(alias[c])] += T - own[c]
            else:
                assert own[c] == T, (c, own[c], T)
        assert mass == [int(x) * n for x in w], trial


def _task_weights(size, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(1, 256, size).astype(np.uint32)
    w = np.floor(rng.lognormal(0, 1.5, size) * 8).astype(np.uint32)
    w[size // 3] = 0
    return w


def pin_task_samplers_law(n=60_000):
    """Every microbenchmark sampler picks index i with chance w_i / T
    (chi-square over n tasks with the same weights and different ids)."""
    from scipy.stats import chisquare
    w = _task_weights(24, "lognormal", 3)
    T = float(w.astype(np.float64).sum())
    for sampler in ["its", "dprs", "zprs", "its_buffered", "alias", "rejection"]:
        picks = [oracle.sample_task(sampler, w, 31, j) for j in range(n)]
        counts = np.bincount(picks, minlength=w.shape[0])
        nz = w > 0
        assert counts[~nz].sum() == 0, sampler
        assert chisquare(counts[nz], w[nz] / T * n).pvalue > 1e-4, (sampler, counts)


def _py_task(sampler, w, seed, task):
    """Tasks rebuilt from numpy's Philox and Python integers; the alias
    table comes from the oracle (pinned above), the reservoir samplers reuse
    the rebuilt walk step."""
    w = [int(x) for x in w]
    n, T, wmax = len(w), sum(w), max(w)
    if T == 0:
        return -1
    if sampler in ("its", "its_buffered"):
        r = (_numpy_philox_block([task, 0, 0, 0], [seed, 0])[0] * T) >> 64
        acc = 0
        for i, x in enumerate(w):
            acc += x
            if acc > r:
                return i
    if sampler == "alias":
        _, prob, alias = oracle.alias_table(w)
        u = _numpy_philox_block([task, 0, 0, 2], [seed, 0])
        c = (u[0] * n) >> 64
        return c if (u[1] * T) >> 64 < int(prob[c]) else int(alias[c])
    if sampler == "rejection":
        for k in range(1 << 24):
            u = _numpy_philox_block([task, k, 0, 3], [seed, 0])
            c = (u[0] * n) >> 64
            if (u[1] * wmax) >> 64 < w[c]:
                return c
        return -1
    raise ValueError(sampler)


def pin_task_samplers_rebuilt():
    for size, kind in [(1, "uniform"), (5, "lognormal"), (40, "lognormal"), (300, "uniform")]:
        w = _task_weights(size, kind, size)
        for sampler in ["its", "its_buffered", "alias", "rejection"]:
            for task in [0, 1, 77, 123456]:
                assert oracle.sample_task(sampler, w, 5, task) == _py_task(sampler, w, 5, task), \
                    (sampler, size, task)
    # uniform weights: the first rejection trial is always accepted
    w = np.full(50, 7, np.uint32)
    for task in range(20):
        u = _numpy_philox_block([task, 0, 0, 3], [9, 0])
        assert oracle.sample_task("rejection", w, 9, task) == (u[0] * 50) >> 64
    for sampler in oracle.TASK_SAMPLERS:
        assert oracle.sample_task(sampler, np.zeros(9, np.uint32), 1, 1) == -1
        one = np.zeros(9, np.uint32)
        one[6] = 3
        assert all(oracle.sample_task(sampler, one, 1, t) == 6 for t in range(10)), sampler


ALL_PINS = [pin_philox_kat, pin_philox_numpy, pin_draw_keying, pin_scale_closed_form,
            pin_pick_bruteforce, pin_hand_weights, pin_walk_rebuilt, pin_walk_ids_rebuilt,
            pin_walk_ids_rmat12, pin_chi2_paths, pin_identities,
            pin_regular_uniform, pin_path_graph_edges, pin_errors,
            pin_zero_length_and_dead_ends, pin_stop_coin_closed_form, pin_stop_keying,
            pin_ppr_rebuilt, pin_ppr_length_distribution, pin_ppr_limits,
            pin_entry_draw_keying, pin_zigzag_golden, pin_reservoir_extremes,
            pin_reservoir_distribution, pin_reservoir_walks_rebuilt,
            pin_reservoir_hop_distribution, pin_alias_golden, pin_alias_mass_identity,
            pin_task_samplers_law, pin_task_samplers_rebuilt]

# The statistical pins take seconds each; a planted mistake is looked for
# with the exact pins first.
SLOW_PINS = [pin_chi2_paths, pin_reservoir_distribution, pin_reservoir_hop_distribution,
             pin_task_samplers_law]
