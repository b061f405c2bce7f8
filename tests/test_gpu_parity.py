"""GPU parity (HIP path through the C ABI) against the oracle, bit-exact.

Sizes are small enough for the oracle to finish in seconds and still cover
several 64-wide chunks, multi-level locates (degrees past 64 and 4096), rows
longer than one 64-entry store, ragged tails, early ends and every algorithm,
in both the plain and the persistent kernels."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import END, assert_rows_equal, gpu_walk, torch_or_skip
from helpers import csr_from_edges, tiny6

pytestmark = pytest.mark.gpu

MODES = ["plain", "persistent", "staged"]


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    return torch, fw


def _check(env, g, algo, factors, schema, starts, length, seed, mode, qid_base=0, stop=(0, 1),
           **kw):
    torch, fw = env
    G = fw.Graph.of(g)
    prm = fw.make_params(factors, schema, stop)
    got = gpu_walk(torch, fw, G, algo, prm, starts, length, seed, mode, qid_base=qid_base, **kw)
    exp = oracle.walk(g, algo, oracle.params(*factors, schema=schema, stop=stop), starts, length,
                      seed, qid_base=qid_base)
    assert_rows_equal(got, exp, f"{algo} {mode} L={length}")
    return got


ALGOS = [("deepwalk", (1, 1, 1), ()), ("node2vec", (1, 2, 4), ()), ("node2vec", (4, 2, 1), ()),
         ("metapath", (1, 1, 1), (0, 1, 2)), ("metapath", (1, 1, 1), (1,))]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("weighted", [True, False])
@pytest.mark.parametrize("algo,factors,schema", ALGOS)
@pytest.mark.parametrize("length", [0, 1, 5, 70, 130])
def test_tiny6(env, mode, weighted, algo, factors, schema, length):
    g, _ = tiny6(weighted=weighted)
    starts = np.tile(np.arange(6, dtype=np.uint32), 40)
    _check(env, g, algo, factors, schema, starts, length, 99, mode, qid_base=7)


def _star(d, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 1000, d)
    lab = rng.integers(0, 3, d)
    return csr_from_edges(d + 1, [(0, i + 1, int(w[i]), int(lab[i])) for i in range(d)])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [1, 63, 64, 65, 127, 4095, 4096, 4097, 70_000, 300_001])
def test_star_hub_degrees(env, mode, d):
    g = _star(d, d)
    starts = np.concatenate([np.zeros(64, np.uint32),
                             np.arange(1, min(d, 200) + 1, dtype=np.uint32)])
    for algo, f, sch in [("deepwalk", (1, 1, 1), ()), ("node2vec", (2, 3, 5), ()),
                         ("metapath", (1, 1, 1), (1, 2))]:
        _check(env, g, algo, f, sch, starts, 9, 1234, mode)


def _big_star(d, seed):
    """Star of d leaves built with numpy (vertex 0 is the hub).  The last
    fiftieth of the hub's row carries about half of its weight, so draws land
    in the tail groups of the multi-level locate as often as elsewhere."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 1000, d).astype(np.uint32)
    tail = d - d // 50
    w[tail:] = rng.integers(20_000, 29_000, d - tail)
    lab = rng.integers(0, 3, d).astype(np.uint8)
    from types import SimpleNamespace
    off = np.concatenate([[0], d + np.arange(0, d + 1)]).astype(np.uint64)
    adj = np.concatenate([np.arange(1, d + 1), np.zeros(d)]).astype(np.uint32)
    return SimpleNamespace(offsets=off, adj=adj, weights=np.concatenate([w, w]),
                           labels=np.concatenate([lab, lab]), n_vertices=d + 1,
                           n_edges=2 * d)


_BIG_STAR_ALGOS = [("deepwalk", (1, 1, 1), (), (0, 1)), ("node2vec", (2, 3, 5), (), (0, 1)),
                   ("metapath", (1, 1, 1), (1, 2), (0, 1)), ("ppr", (1, 1, 1), (), (1, 5))]


@pytest.mark.parametrize("d", [1_048_577, 2_840_149])
def test_star_hub_three_level_locate(env, d):
    """Hubs of more than 2^20 entries: the locate descends three levels of
    64 groups before the last 64 quads (rows of the largest synthetic
    graph reach 2,840,149 entries).  Every algorithm, every mode."""
    torch, fw = env
    g = _big_star(d, d)
    G = fw.Graph.of(g)
    starts = np.concatenate([np.zeros(24, np.uint32), np.arange(1, 25, dtype=np.uint32),
                             np.array([d, d - 1, d // 2], np.uint32)])
    for algo, f, sch, stop in _BIG_STAR_ALGOS:
        exp = oracle.walk(g, algo, oracle.params(*f, schema=sch, stop=stop), starts, 6, 4321)
        prm = fw.make_params(f, sch, stop)
        for mode in MODES:
            got = gpu_walk(torch, fw, G, algo, prm, starts, 6, 4321, mode)
            assert_rows_equal(got, exp, f"{algo} {mode} d={d}")
    G.free()


@pytest.fixture(scope="module")
def powerlaw():
    g = synth.chung_lu(20_000, 300_000, 2.1, 1.5, seed=5)
    g.weights = synth.weights_zipf(g, 1.2, 65535, 6)
    g.labels = synth.labels_uniform(g, 5, 7)
    return g


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("algo,factors,schema", ALGOS)
def test_powerlaw_graph(env, powerlaw, mode, algo, factors, schema):
    g = powerlaw
    assert g.degrees().max() > 4096
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::5]
    _check(env, g, algo, factors, schema, starts, 12, 31337, mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("schema", [(0x80, 0xFF, 0x7F), (0x00, 0x01, 0xFE, 0x81), (0x55,)])
def test_metapath_label_bytes(env, mode, schema):
    """Unweighted MetaPath with labels over the whole byte range (the walkers
    count matching label bytes of a quad with bit operations): bytes whose
    high bit or low seven bits equal the wanted label's must not count."""
    g = synth.chung_lu(20_000, 300_000, 2.1, 1.5, seed=9)
    rng = np.random.default_rng(10)
    pool = np.array(sorted({*schema, *(b ^ 0x80 for b in schema), *(b ^ 0x01 for b in schema),
                            0x00, 0x7F, 0x80, 0xFF}), dtype=np.uint8)
    g.labels = pool[rng.integers(0, len(pool), g.n_edges)]
    g.weights = None
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::4]
    _check(env, g, "metapath", (1, 1, 1), schema, starts, 10, 2718, mode)


_HUB_ROWS = {}


def _labelled_hub(d, lead):
    """Vertex 1 is a hub of degree d with random labels in {0, 1, 2} and no
    weights; vertex 0 has `lead` neighbours of its own, so the hub's row
    starts `lead` entries into a 4-entry quad."""
    key = (d, lead)
    if key not in _HUB_ROWS:
        rng = np.random.default_rng(d * 4 + lead)
        lab = rng.integers(0, 3, d + lead)
        edges = [(0, 2 + d + i, 1, int(lab[d + i])) for i in range(lead)]
        edges += [(1, 2 + i, 1, int(lab[i])) for i in range(d)]
        _HUB_ROWS[key] = csr_from_edges(2 + d + lead, edges, weights=False)
    return _HUB_ROWS[key]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d,lead", [(65, 1), (255, 2), (257, 3), (2049, 0), (2049, 1),
                                    (16385, 2), (114691, 3), (131073, 1), (300001, 2)])
def test_metapath_unweighted_hub_rows(env, mode, d, lead):
    """Unweighted MetaPath counts matching labels per quad in its streaming
    pass, several quads per lane at once, with the slice's first and last
    quads masked: hub rows of every length class (one chunk, fewer than eight
    chunks per group, eight or more) at every alignment of the row's start."""
    g = _labelled_hub(d, lead)
    assert int(g.offsets[1]) % 4 == lead
    starts = np.concatenate([np.ones(96, np.uint32), np.arange(2, 34, dtype=np.uint32)])
    for schema in [(1,), (2, 0)]:
        _check(env, g, "metapath", (1, 1, 1), schema, starts, 6, 4242 + d, mode)


def _colliding_graph(npd, nother=150, V=40_000, seed=1):
    """Vertex 0 (prev) whose npd neighbours all fall into one bucket of the
    persistent walker's LDS hash set (Fibonacci hashing: the top bits of
    (u mod 2^24) * 0x9E3779 mod 2^32; a table fills its wavefront's region, so
    keys sharing the top 8 bits share a bucket in every table of up to 256
    buckets), so membership tests of vertex 1's neighbours must probe long
    bucket chains; every walk goes 0 -> 1 -> ..."""
    h = lambda u: (((u & 0xFFFFFF) * 0x9E3779) & 0xFFFFFFFF) >> 24  # noqa: E731
    keys = [u for u in range(2, V) if h(u) == h(2)][:npd]
    assert len(keys) == npd
    rng = np.random.default_rng(seed)
    ks = set(keys)
    others = [u for u in rng.permutation(np.arange(2, V)).tolist() if u not in ks][:nother]
    edges = [(0, 1, 1_000_000, 0)] + [(0, k, 1, 0) for k in keys]
    edges += [(1, k, 1 + k % 7, 0) for k in keys] + [(1, o, 1 + o % 5, 0) for o in others]
    edges += [(i, i + 1, 1, 0) for i in range(2, V - 1)]
    return csr_from_edges(V, sorted(set(edges)))


@pytest.mark.parametrize("npd,V", [(30, 12_000), (60, 24_000), (120, 40_000), (300, 120_000)])
def test_hash_bucket_collisions(env, npd, V):
    """Every key of N(prev) in one bucket chain, in tables of 64 and 256
    buckets (regions of 256 and 1024 cells)."""
    torch, fw = env
    g = _colliding_graph(npd, V=V)
    starts = np.zeros(5000, dtype=np.uint32)
    for tune in [dict(hash_cells=1024, wgs_per_cu=8, tiny_max=0),
                 dict(hash_cells=256, wgs_per_cu=4, tiny_max=16)]:
        _check(env, g, "node2vec", (1, 2, 4), (), starts, 3, 777, "persistent",
               tune=fw.make_tune(**tune))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("factors", [(1, 2, 4), (7, 3, 5), (1, 1, 16)])
@pytest.mark.parametrize("wmax", [(1 << 24) // 16 - 1, (1 << 24) // 16, (1 << 31) + 12345])
def test_node2vec_weight_widths(env, mode, factors, wmax):
    """Weight times factor just below, at and far above 2^24: the walkers
    switch between 24-bit and full products at that bound, and both must
    give the oracle's walks."""
    g = synth.chung_lu(6_000, 90_000, 2.1, 1.5, seed=17)
    rng = np.random.default_rng(wmax % 1000)
    w = rng.integers(1, wmax + 1, g.n_edges, dtype=np.uint64)
    w[rng.integers(0, g.n_edges, 50)] = wmax
    g.weights = w.astype(np.uint32)
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::3]
    _check(env, g, "node2vec", factors, (), starts, 9, 5151, mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("weighted", [True, False])
@pytest.mark.parametrize("stop", [(1, 5), (0, 1), (1, 1), (2, 3)])
@pytest.mark.parametrize("length", [0, 1, 7, 70])
def test_ppr_tiny6(env, mode, weighted, stop, length):
    """PPR (stop coin before each hop, DeepWalk weights), including the
    never-stop and always-stop limits."""
    g, _ = tiny6(weighted=weighted)
    starts = np.tile(np.arange(6, dtype=np.uint32), 40)
    _check(env, g, "ppr", (1, 1, 1), (), starts, length, 2024, mode, qid_base=3, stop=stop)


@pytest.mark.parametrize("mode", MODES)
def test_ppr_from_the_hub(env, powerlaw, mode):
    """The experiments' PPR set-up: every query starts at the vertex of
    largest degree (here about 2,000 neighbours), stop chance 1/5."""
    g = powerlaw
    hub = int(np.argmax(g.degrees()))
    starts = np.full(3000, hub, dtype=np.uint32)
    got = _check(env, g, "ppr", (1, 1, 1), (), starts, 40, 77, mode, stop=(1, 5))
    hops = (got[:, 1:] != END).sum(axis=1)
    assert (hops == 0).any() and hops.max() >= 10


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [65, 4097, 70_000])
def test_ppr_star_hub(env, mode, d):
    g = _star(d, d + 1)
    starts = np.zeros(200, np.uint32)
    _check(env, g, "ppr", (1, 1, 1), (), starts, 5, 4321, mode, stop=(1, 3))


@pytest.mark.parametrize("algo,factors,schema", [ALGOS[1], ALGOS[3]])
def test_count_steps_matches_oracle(env, powerlaw, algo, factors, schema):
    """fw_count_steps counts exactly the oracle's realised hops (MetaPath
    walks end early, so the count is below n * length)."""
    torch, fw = env
    g = powerlaw
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::3]
    G = fw.Graph.of(g)
    st = torch.from_numpy(starts.view(np.int32)).cuda()
    out = fw.walk(G, algo, fw.make_params(factors, schema), st, 17, 99, mode="persistent")
    exp = oracle.walk(g, algo, oracle.params(*factors, schema=schema), starts, 17, 99)
    want = int((exp[:, 1:] != END).sum())
    assert fw.count_steps(out) == want
    assert fw.count_steps(out[:1]) == int((exp[:1, 1:] != END).sum())
    if algo == "metapath":
        assert want < starts.shape[0] * 17


@pytest.mark.parametrize("mode", MODES)
def test_rmat12_node2vec_full(env, mode):
    """R-MAT scale 12, node2vec p=2 q=1/2 (factors 1, 2, 4), one query per
    vertex, 20 hops, seed 42: the whole query set."""
    g = synth.load_recipe_graph("rmat12_n2v", use_cache=False)
    starts = np.arange(g.n_vertices, dtype=np.uint32)
    got = _check(env, g, "node2vec", (1, 2, 4), (), starts, 20, 42, mode)
    assert (got[:, 1] != END).sum() > 2000


def test_modes_agree_unweighted_deepwalk(env):
    torch, fw = env
    g = synth.rmat(12, 8, seed=3)
    starts = np.arange(g.n_vertices, dtype=np.uint32)
    G = fw.Graph.of(g)
    a = gpu_walk(torch, fw, G, "deepwalk", None, starts, 40, 5, "plain")
    b = gpu_walk(torch, fw, G, "deepwalk", None, starts, 40, 5, "persistent")
    assert_rows_equal(a, b, "plain vs persistent")
    exp = oracle.walk(g, "deepwalk", oracle.params(), starts, 40, 5)
    assert_rows_equal(a, exp, "unweighted deepwalk")


def test_errors(env):
    torch, fw = env
    g, _ = tiny6(labelled=False)
    G = fw.Graph.of(g)
    st = torch.tensor([0, 6], dtype=torch.int32, device="cuda")
    for mode in MODES:
        with pytest.raises(fw.FWError) as e:
            fw.walk(G, "deepwalk", None, st, 3, 1, mode=mode)
        assert e.value.status == fw.EINVAL
    ok = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    fw.walk(G, "deepwalk", None, ok, 3, 1)  # the status was cleared
    with pytest.raises(fw.FWError) as e:
        fw.walk(G, "metapath", fw.make_params(schema=[0]), ok, 3, 1)
    assert e.value.status == fw.EINVAL
    with pytest.raises(fw.FWError) as e:
        fw.walk(G, "node2vec", fw.make_params((0, 0, 0)), ok, 3, 1)
    assert e.value.status == fw.EINVAL
    big = csr_from_edges(3, [(0, 1, 0xFFFFFFFF, 0), (0, 2, 1, 0)])
    B = fw.Graph.of(big)
    with pytest.raises(fw.FWError) as e:
        fw.walk(B, "node2vec", fw.make_params((0xFFFFFFFF, 1, 1)), ok, 3, 1)
    assert e.value.status == fw.EOVERFLOW
    for stop in [(1, 0), (5, 4)]:
        with pytest.raises(fw.FWError) as e:
            fw.walk(G, "ppr", fw.make_params(stop=stop), ok, 3, 1)
        assert e.value.status == fw.EINVAL
    with pytest.raises(fw.FWError) as e:
        fw.walk(G, "ppr", None, ok, 3, 1)
    assert e.value.status == fw.EINVAL
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    out = fw.walk(G, "deepwalk", None, empty, 3, 1)
    assert out.shape == (0, 4)


STAGED_TUNES = [
    dict(wg_size=256, slots=1, tiny_max=1, hub_min=2, wgs_per_cu=1, hash_cells=256),
    dict(wg_size=256, slots=7, tiny_max=4, hub_min=65, wgs_per_cu=3, hash_cells=256),
    dict(wg_size=512, slots=64, tiny_max=16, hub_min=2048, wgs_per_cu=2, hash_cells=8192),
    dict(wg_size=1024, slots=128, tiny_max=16, hub_min=300, wgs_per_cu=1, hash_cells=16384),
    dict(wg_size=512, slots=33, tiny_max=8, hub_min=100000, wgs_per_cu=4, hash_cells=512),
]

PERSISTENT_TUNES = [
    dict(tiny_max=1, wgs_per_cu=1, hash_cells=64),
    dict(tiny_max=2, wgs_per_cu=2, hash_cells=512),
    dict(tiny_max=4, wgs_per_cu=3, hash_cells=256),
    dict(tiny_max=16, wgs_per_cu=4, hash_cells=1024),
    dict(tiny_max=16, wgs_per_cu=8, hash_cells=4096),
    dict(tiny_max=8, wgs_per_cu=2, hash_cells=128),
]

TUNED = [("staged", t) for t in STAGED_TUNES] + [("persistent", t) for t in PERSISTENT_TUNES]


def _tid(mt):
    mode, t = mt
    return mode + "-" + "-".join(f"{k}{v}" for k, v in t.items())


@pytest.mark.parametrize("mode_tune", TUNED, ids=_tid)
@pytest.mark.parametrize("algo,factors,schema", ALGOS[:3] + ALGOS[3:4])
def test_tunes(env, powerlaw, mode_tune, algo, factors, schema):
    """Every launch configuration gives the oracle's walks (degree classes,
    pool sizes, membership structures: hash set, filter, global search)."""
    torch, fw = env
    mode, tune = mode_tune
    g = powerlaw
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::7]
    _check(env, g, algo, factors, schema, starts, 10, 4242, mode, tune=fw.make_tune(**tune))


@pytest.mark.parametrize("mode_tune", TUNED, ids=_tid)
def test_star_hubs_with_tunes(env, mode_tune):
    torch, fw = env
    mode, tune = mode_tune
    g = _star(70_000, 3)
    starts = np.concatenate([np.zeros(40, np.uint32), np.arange(1, 300, dtype=np.uint32)])
    _check(env, g, "node2vec", (2, 3, 5), (), starts, 7, 99, mode, tune=fw.make_tune(**tune))


def _two_hubs(d):
    """Two adjacent hubs sharing most neighbours: node2vec hops between them
    test membership against a large N(prev) (hash set overflow -> filter)."""
    rng = np.random.default_rng(d)
    edges = [(0, 1, 7, 0)]
    for i in range(2, d + 2):
        w = int(rng.integers(1, 100))
        edges.append((0, i, w, i % 3))
        if i % 3:
            edges.append((1, i, w + 1, (i + 1) % 3))
    return csr_from_edges(d + 2, edges)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [100, 5000, 40000])
def test_hub_to_hub_membership(env, mode, d):
    g = _two_hubs(d)
    starts = np.array([0, 1] * 64 + list(range(2, min(200, d + 2))), dtype=np.uint32)
    _check(env, g, "node2vec", (4, 2, 1), (), starts, 12, 5, mode)
    _check(env, g, "node2vec", (1, 2, 4), (), starts, 12, 6, mode)


@pytest.mark.parametrize("cells", [256, 512, 1024, 4096])
@pytest.mark.parametrize("d", [700, 3000, 40000])
def test_merge_membership_windows(env, cells, d):
    """Hub-to-hub hops whose N(prev) exceeds the hash set: the merge of the
    sorted rows, with windows that fit, that need several staging rounds, and
    that overflow the region (falling back to global search)."""
    torch, fw = env
    g = _two_hubs(d)
    starts = np.array([0, 1] * 128, dtype=np.uint32)
    _check(env, g, "node2vec", (4, 2, 1), (), starts, 9, 11, "persistent",
           tune=fw.make_tune(hash_cells=cells, tiny_max=1))


def _ratio_boundary(dc, pd):
    """Hub 0 with pd neighbours, 64 of them the vertices 1..64 of degree dc:
    the hub plus dc - 1 others, half of those also neighbours of the hub.
    Heavy edges send walks hub -> vertex k -> hub -> vertex j, so the hops
    from vertex j test N(cur), dc entries, against the hub's pd."""
    rng = np.random.default_rng(pd * 131 + dc)
    hub_others = 65 + np.arange(pd - 64)
    nonshared = 65 + (pd - 64) + np.arange(4 * dc)
    edges = [(0, k, 50_000, 0) for k in range(1, 65)]
    edges += [(0, int(v), 1, 0) for v in hub_others]
    for k in range(1, 65):
        sh = rng.choice(hub_others, (dc - 1) // 2, replace=False)
        ns = rng.choice(nonshared, dc - 1 - len(sh), replace=False)
        edges += [(k, int(v), int(rng.integers(1, 1000)), 0) for v in np.concatenate([sh, ns])]
    return csr_from_edges(65 + (pd - 64) + 4 * dc, edges, labels=False)


@pytest.mark.parametrize("cells", [1024, 4096])
@pytest.mark.parametrize("pd", [1280, 1281])
def test_node2vec_search_ratio_boundary(env, cells, pd):
    """N(prev) at 64x N(cur) (merge with 1,024 cells, hash set with 4,096)
    and one entry past it (binary search in global memory): the same walks
    as the oracle on both sides of the switch."""
    torch, fw = env
    g = _ratio_boundary(20, pd)
    assert int(g.offsets[1] - g.offsets[0]) == pd and int(g.offsets[2] - g.offsets[1]) == 20
    starts = np.tile(np.arange(1, 65, dtype=np.uint32), 4)
    for f in [(4, 2, 1), (1, 2, 4)]:
        _check(env, g, "node2vec", f, (), starts, 12, 2024, "persistent",
               tune=fw.make_tune(hash_cells=cells, sparse_ratio=0xFFFFFFFF))


def _hub_with_parallel_edges(weighted):
    """Hub 0 with 3,000 leaves, parallel edges to 5 (three) and 7 (two), and a
    self-loop; vertex 5 has parallel edges to 8, a self-loop, and edges to 6
    and 7; vertex 10 has 100 neighbours.  Node2vec hops from the hub after 5
    or 10 take the sparse-N(prev) pass."""
    rng = np.random.default_rng(77)
    edges = [(0, i, int(rng.integers(1, 60_000)), 0) for i in range(1, 3001)]
    edges += [(0, 5, 7, 0), (0, 5, 9, 0), (0, 7, 11, 0), (0, 0, 5, 0)]
    edges += [(5, 8, 3, 0), (5, 8, 4, 0), (5, 5, 2, 0), (5, 6, 1, 0), (5, 7, 13, 0)]
    edges += [(10, j, int(rng.integers(1, 100)), 0) for j in range(11, 111)]
    return csr_from_edges(3001, edges, weights=weighted, labels=False)


@pytest.mark.parametrize("weighted", [True, False])
@pytest.mark.parametrize("ratio", [1, 16, 0xFFFFFFFF])
def test_node2vec_sparse_prev_edge_cases(env, weighted, ratio):
    """Parallel edges in both rows, self-loops, prev repeated in N(cur):
    the same walks whether N(prev)'s keys are looked up in N(cur) or every
    entry of N(cur) is tested against N(prev)."""
    torch, fw = env
    g = _hub_with_parallel_edges(weighted)
    starts = np.array([5] * 96 + [10] * 96 + [0] * 32 + list(range(11, 43)), dtype=np.uint32)
    for f in [(1, 2, 4), (4, 2, 1), (3, 0, 5), (0, 7, 2)]:
        _check(env, g, "node2vec", f, (), starts, 6, 1357, "persistent",
               tune=fw.make_tune(sparse_ratio=ratio, tiny_max=1))


def test_graph_replay_matches_eager(env, powerlaw):
    """The captured hipGraph of the persistent launch replays to the same
    walks every time, with eager work and synchronisation in between."""
    torch, fw = env
    g = powerlaw
    G = fw.Graph.of(g)
    prm = fw.make_params((1, 2, 4))
    starts = torch.arange(0, g.n_vertices, 3, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    eager = fw.walk(G, "node2vec", prm, starts, 15, 77, mode="plain")
    torch.cuda.synchronize()
    out = torch.empty_like(eager)
    for i in range(4):
        out.fill_(-7)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            fw.walk(G, "node2vec", prm, starts, 15, 77, out=out,
                    mode=("persistent", "staged")[i % 2], stream=stream, use_graph=True)
        stream.synchronize()
        assert torch.equal(out, eager), f"replay {i}"
        junk = fw.walk(G, "deepwalk", None, starts[:100], 3, i, mode="plain")
        torch.cuda.synchronize()
        del junk
    exp = oracle.walk(g, "node2vec", oracle.params(1, 2, 4), starts.cpu().numpy(), 15, 77)
    assert_rows_equal(out.cpu().numpy().view(np.uint32), exp, "graph replay")


def test_graph_replay_beside_eager_walks(env, powerlaw):
    """A captured walk replayed on one stream while more eager persistent
    walks than there are rotating head slots (64) run on another stream: the
    captured launch claims queries from a counter of its own, so no query of
    either side is skipped or walked twice."""
    torch, fw = env
    g = powerlaw
    G = fw.Graph.of(g)
    prm = fw.make_params((1, 2, 4))
    starts = torch.arange(0, g.n_vertices, 2, dtype=torch.int32, device="cuda")
    small = starts[:777].contiguous()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    out_a = torch.empty((starts.numel(), 13), dtype=torch.int32, device="cuda")
    outs_b = [torch.empty((small.numel(), 6), dtype=torch.int32, device="cuda")
              for _ in range(70)]
    exp_a = oracle.walk(g, "node2vec", oracle.params(1, 2, 4), starts.cpu().numpy(), 12, 5)
    small_np = small.cpu().numpy()
    exp_b = [oracle.walk(g, "deepwalk", oracle.params(), small_np, 5, 1000 + i)
             for i in range(len(outs_b))]
    for rep in range(3):
        out_a.fill_(-7)
        for ob in outs_b:
            ob.fill_(-7)
        torch.cuda.synchronize()
        with torch.cuda.stream(sa):
            fw.walk(G, "node2vec", prm, starts, 12, 5, out=out_a, mode="persistent",
                    stream=sa, async_=True, use_graph=True)
        with torch.cuda.stream(sb):
            for i, ob in enumerate(outs_b):
                fw.walk(G, "deepwalk", None, small, 5, 1000 + i, out=ob, mode="persistent",
                        stream=sb, async_=True)
        fw.sync(G, sa)
        fw.sync(G, sb)
        assert_rows_equal(out_a.cpu().numpy().view(np.uint32), exp_a, f"replay {rep}")
        for i, ob in enumerate(outs_b):
            assert_rows_equal(ob.cpu().numpy().view(np.uint32), exp_b[i], f"eager {i} rep {rep}")


def test_graph_cache_is_bounded(env, powerlaw):
    """Replays keyed by many seeds (more than the cache holds) stay correct:
    old captured launches are dropped, the latest ones replay."""
    torch, fw = env
    g = powerlaw
    G = fw.Graph.of(g)
    starts = torch.arange(0, g.n_vertices, 37, dtype=torch.int32, device="cuda")
    st_np = starts.cpu().numpy()
    s = torch.cuda.Stream()
    out = torch.empty((starts.numel(), 8), dtype=torch.int32, device="cuda")
    for seed in list(range(40)) + [39, 38, 0]:
        out.fill_(-7)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            fw.walk(G, "deepwalk", None, starts, 7, seed, out=out, mode="persistent",
                    stream=s, use_graph=True)
        exp = oracle.walk(g, "deepwalk", oracle.params(), st_np, 7, seed)
        assert_rows_equal(out.cpu().numpy().view(np.uint32), exp, f"seed {seed}")


def test_async_on_stream_and_qid_base(env, powerlaw):
    torch, fw = env
    g = powerlaw
    G = fw.Graph.of(g)
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::11]
    st = torch.from_numpy(starts.astype(np.int32)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = fw.walk(G, "metapath", fw.make_params(schema=[2, 0]), st, 9, 5, mode="persistent",
                      stream=s, async_=True, qid_base=123456789)
    fw.sync(G, s)
    exp = oracle.walk(g, "metapath", oracle.params(schema=[2, 0]), starts, 9, 5,
                      qid_base=123456789)
    assert_rows_equal(out.cpu().numpy().view(np.uint32), exp, "async qid_base")


def test_autotune_then_walks_match(env, powerlaw):
    torch, fw = env
    g = powerlaw
    G = fw.Graph.of(g)
    prm = fw.make_params((1, 2, 4))
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::3]
    st = torch.from_numpy(starts.astype(np.int32)).cuda()
    best = fw.autotune(G, "node2vec", prm, st[::4].contiguous(), 10, 1)
    assert best["wgs_per_cu"] >= 1 and best["hash_cells"] >= 64 and best["tiny_max"] <= 16
    assert best["mode"] in (2, 3)
    exp = oracle.walk(g, "node2vec", oracle.params(1, 2, 4), starts, 10, 4)
    for mode in ("auto", "persistent", "staged"):
        got = fw.walk(G, "node2vec", prm, st, 10, 4, mode=mode)
        torch.cuda.synchronize()
        assert_rows_equal(got.cpu().numpy().view(np.uint32), exp, f"after autotune {mode}")
    # A second upload of the same graph has the same fingerprint and finds
    # the tuned configurations.
    G2 = fw.Graph.of(g)
    got = fw.walk(G2, "node2vec", prm, st, 10, 4, mode="auto")
    torch.cuda.synchronize()
    assert_rows_equal(got.cpu().numpy().view(np.uint32), exp, "re-uploaded graph, auto")
    G2.free()
