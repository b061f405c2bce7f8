"""Reservoir-sampler walkers (GPU) against the oracle, bit-exact: DPRS
(Algorithm 3) and ZPRS (Algorithm 4) with one Philox word per entry, for
every algorithm, on hand-sized graphs, hubs whose degree spans several
256-entry chunks and 64-lane zig-zag rounds with ragged tails, and a
power-law graph."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_rows_equal, gpu_walk, torch_or_skip
from helpers import csr_from_edges, tiny6

pytestmark = pytest.mark.gpu

SAMPLERS = ["dprs", "zprs"]
ALGOS = [("deepwalk", (1, 1, 1), (), (0, 1)), ("node2vec", (1, 2, 4), (), (0, 1)),
         ("metapath", (1, 1, 1), (0, 1, 2), (0, 1)), ("ppr", (1, 1, 1), (), (1, 5))]


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    return torch, fw


def _check(env, g, sampler, algo, f, sch, stop, starts, length, seed, qid_base=0):
    torch, fw = env
    G = fw.Graph.of(g)
    got = gpu_walk(torch, fw, G, algo, fw.make_params(f, sch, stop), starts, length, seed,
                   "plain", qid_base=qid_base, sampler=sampler)
    exp = oracle.walk(g, algo, oracle.params(*f, schema=sch, stop=stop), starts, length, seed,
                      qid_base=qid_base, sampler=sampler)
    assert_rows_equal(got, exp, f"{sampler} {algo} L={length}")
    return got


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("weighted", [True, False])
@pytest.mark.parametrize("algo,f,sch,stop", ALGOS)
@pytest.mark.parametrize("length", [0, 1, 5, 70])
def test_tiny6(env, sampler, weighted, algo, f, sch, stop, length):
    g, _ = tiny6(weighted=weighted)
    starts = np.tile(np.arange(6, dtype=np.uint32), 30)
    _check(env, g, sampler, algo, f, sch, stop, starts, length, 31, qid_base=5)


def _hub(d, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 50, d)  # some zero weights
    lab = rng.integers(0, 3, d)
    edges = [(0, i + 1, int(w[i]), int(lab[i])) for i in range(d)]
    edges += [(i, i % d + 1, 1 + i % 5, int(i % 3)) for i in range(1, d + 1)]
    return csr_from_edges(d + 1, edges)


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("d", [3, 65, 255, 257, 700, 4097, 70_001])
def test_hub_degrees(env, sampler, d):
    g = _hub(d, d)
    starts = np.concatenate([np.zeros(48, np.uint32), np.arange(1, min(d, 40) + 1,
                                                                  dtype=np.uint32)])
    for algo, f, sch, stop in ALGOS:
        _check(env, g, sampler, algo, f, sch, stop, starts, 4, 777)


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("algo,f,sch,stop", ALGOS)
def test_powerlaw(env, sampler, algo, f, sch, stop):
    g = synth.chung_lu(20_000, 300_000, 2.1, 1.5, seed=5)
    g.weights = synth.weights_zipf(g, 1.2, 65535, 6)
    g.labels = synth.labels_uniform(g, 5, 7)
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::9]
    _check(env, g, sampler, algo, f, sch, stop, starts, 12, 99)


def test_samplers_differ_but_agree_in_law(env):
    """On a 700-neighbour hub the three samplers pick differently query by
    query, with the same chances (chi-square against w_i / T)."""
    from scipy.stats import chisquare
    torch, fw = env
    d = 700
    g = _hub(d, 1)
    G = fw.Graph.of(g)
    n = 400_000
    starts = np.zeros(n, dtype=np.uint32)
    w = g.weights[int(g.offsets[0]):int(g.offsets[1])].astype(np.float64)
    picks = {}
    for sampler in ["its", "dprs", "zprs"]:
        rows = gpu_walk(torch, fw, G, "deepwalk", None, starts, 1, 3, "plain", sampler=sampler)
        counts = np.bincount(rows[:, 1].astype(np.int64) - 1, minlength=d)
        assert counts[w == 0].sum() == 0
        nz = w > 0
        assert chisquare(counts[nz], w[nz] / w.sum() * n).pvalue > 1e-4, sampler
        picks[sampler] = rows[:, 1]
    assert (picks["its"] != picks["dprs"]).mean() > 0.5
    assert (picks["dprs"] != picks["zprs"]).mean() > 0.5


def test_sampler_errors(env):
    torch, fw = env
    g, _ = tiny6()
    G = fw.Graph.of(g)
    st = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    for mode in ["persistent", "auto", "staged"]:
        with pytest.raises(fw.FWError) as e:
            fw.walk(G, "deepwalk", None, st, 3, 1, mode=mode, sampler="zprs")
        assert e.value.status == fw.EINVAL
    with pytest.raises(fw.FWError) as e:
        fw.walk(G, "deepwalk", None, st, 3, 1, mode="plain", sampler=7)
    assert e.value.status == fw.EINVAL
