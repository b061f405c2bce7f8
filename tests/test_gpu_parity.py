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

MODES = ["plain", "persistent"]


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    return torch, fw


def _check(env, g, algo, factors, schema, starts, length, seed, mode, qid_base=0, **kw):
    torch, fw = env
    G = fw.Graph.of(g)
    prm = fw.make_params(factors, schema)
    got = gpu_walk(torch, fw, G, algo, prm, starts, length, seed, mode, qid_base=qid_base, **kw)
    exp = oracle.walk(g, algo, oracle.params(*factors, schema=schema), starts, length, seed,
                      qid_base=qid_base)
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
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    out = fw.walk(G, "deepwalk", None, empty, 3, 1)
    assert out.shape == (0, 4)
