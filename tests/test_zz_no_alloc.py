"""fw_walk_noalloc (the persistent walk whose task-pool counter lives in the
library's static device array) against fw_walk_ex in FW_MODE_PERSISTENT and
the oracle, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_rows_equal, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    return torch, fw


@pytest.mark.parametrize("algo,factors,schema", [("node2vec", (1, 2, 4), ()),
                                                 ("deepwalk", (1, 1, 1), ()),
                                                 ("metapath", (1, 1, 1), (0, 1, 2))])
def test_noalloc_matches_persistent(env, algo, factors, schema):
    torch, fw = env
    g = synth.chung_lu(20_000, 300_000, 2.1, 1.5, seed=5)
    g.weights = synth.weights_zipf(g, 1.2, 65535, 6)
    g.labels = synth.labels_uniform(g, 5, 7)
    G = fw.Graph.of(g)
    prm = fw.make_params(factors, schema)
    oprm = oracle.params(*factors, schema=schema)
    s = torch.cuda.Stream()
    for call, (n, length, seed) in enumerate([(20_000, 17, 3), (1_234, 9, 4)]):
        starts_np = np.arange(n, dtype=np.uint32) * 7 % g.n_vertices
        st = torch.from_numpy(starts_np.view(np.int32)).cuda()
        out = torch.full((n, length + 1), -7, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            fw.walk_noalloc(G, algo, prm, st, out, length, seed, stream=s)
        fw.sync(G, s)
        ref = fw.walk(G, algo, prm, st, length, seed, mode="persistent")
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert_rows_equal(got, ref.cpu().numpy().view(np.uint32), f"{algo} call {call} vs persistent")
        exp = oracle.walk(g, algo, oprm, starts_np, length, seed)
        assert_rows_equal(got, exp, f"{algo} call {call} vs oracle")
    G.free()


def test_noalloc_errors(env):
    torch, fw = env
    g = synth.chung_lu(2_000, 20_000, 2.1, 1.5, seed=9)
    G = fw.Graph.of(g)
    st = torch.tensor([0, 1, g.n_vertices + 5], dtype=torch.int32, device="cuda")
    out = torch.empty((3, 5), dtype=torch.int32, device="cuda")
    fw.walk_noalloc(G, "deepwalk", None, st, out, 4, 1)
    with pytest.raises(fw.FWError):
        fw.sync(G)  # the kernel flags the start vertex >= V
    with pytest.raises(fw.FWError):
        fw.walk_noalloc(G, "metapath", fw.make_params(schema=[]), st[:2], out[:2], 4, 1)
    fw.walk_noalloc(G, "deepwalk", None, st[:0], out[:0], 4, 1)  # n = 0: no-op
    fw.sync(G)
    G.free()
