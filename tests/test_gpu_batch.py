"""Out-of-HBM result batching (GPU): fw_walk_host with device budgets that
force many ping-pong batches, a ragged last batch and a single batch gives
the oracle's rows (query i keeps id i across batches), in every mode."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_rows_equal, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    g = synth.chung_lu(20_000, 300_000, 2.1, 1.5, seed=5)
    g.weights = synth.weights_zipf(g, 1.2, 65535, 6)
    g.labels = synth.labels_uniform(g, 5, 7)
    return fw, g, fw.Graph.of(g)


CASES = [("node2vec", (1, 2, 4), (), (0, 1)), ("ppr", (1, 1, 1), (), (1, 5)),
         ("metapath", (1, 1, 1), (0, 1, 2), (0, 1))]


@pytest.mark.parametrize("mode", ["plain", "persistent", "auto"])
@pytest.mark.parametrize("algo,f,sch,stop", CASES)
@pytest.mark.parametrize("budget_queries", [1, 777, 5000, 100_000])
def test_batches_equal_oracle(env, mode, algo, f, sch, stop, budget_queries):
    fw, g, G = env
    L = 17
    starts = np.arange(g.n_vertices, dtype=np.uint32)[::4]
    n = starts.shape[0]
    budget = budget_queries * 2 * (L + 2) * 4
    rows, B, nb = fw.walk_host(G, algo, fw.make_params(f, sch, stop), starts, L, 4242,
                               device_budget_bytes=budget, mode=mode)
    assert B == min(budget_queries, n) and nb == -(-n // B)
    exp = oracle.walk(g, algo, oracle.params(*f, schema=sch, stop=stop), starts, L, 4242)
    assert_rows_equal(rows, exp, f"host batches B={B}")


def test_cap_and_defaults(env):
    fw, g, G = env
    starts = np.arange(g.n_vertices, dtype=np.uint32)
    rows, B, nb = fw.walk_host(G, "deepwalk", None, starts, 9, 3, max_batch_queries=3001)
    assert B == 3001 and nb == -(-g.n_vertices // 3001)
    exp = oracle.walk(g, "deepwalk", oracle.params(), starts, 9, 3)
    assert_rows_equal(rows, exp, "capped batches")
    rows, B, nb = fw.walk_host(G, "deepwalk", None, starts, 9, 3)
    assert nb == 1
    assert_rows_equal(rows, exp, "one batch")


def test_errors_and_edges(env):
    fw, g, G = env
    with pytest.raises(fw.FWError) as e:
        fw.walk_host(G, "deepwalk", None, np.array([0, g.n_vertices], np.uint32), 3, 1)
    assert e.value.status == fw.EINVAL
    with pytest.raises(fw.FWError) as e:
        fw.walk_host(G, "deepwalk", None, np.array([0, 1], np.uint32), 3, 1,
                     device_budget_bytes=10)
    assert e.value.status == fw.EINVAL
    rows, B, nb = fw.walk_host(G, "deepwalk", None, np.zeros(0, np.uint32), 3, 1)
    assert rows.shape == (0, 4) and nb == 0
    rows, _, _ = fw.walk_host(G, "deepwalk", None, np.array([5, 6], np.uint32), 0, 1)
    assert rows.tolist() == [[5], [6]]
