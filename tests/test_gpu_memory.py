"""Device memory of a walk (the memory table of the experiments): the graph's
arrays are resident once, and a walk adds nothing but the caller's result
rows, n*(L+1)*4 bytes.  The walkers keep no per-query or per-vertex state in
device memory."""
import numpy as np
import pytest

import synth
from gpu_common import torch_or_skip

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def _graph():
    g = synth.rmat(18, 16, seed=31)
    g.weights = synth.weights_uniform(g, 1, 255, 32)
    g.labels = synth.labels_uniform(g, 5, 33)
    return g


def _free(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_graph_bytes_match_the_layout():
    """offsets u64[V+1], adj u32[E], weights u32[E], labels u8[E], plus a few
    KB of padding and per-graph walk state."""
    torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    g = _graph()
    G = fw.Graph.of(g)
    arrays = 8 * (g.n_vertices + 1) + (4 + 4 + 1) * g.n_edges
    assert arrays <= G.info()["device_bytes"] <= arrays + 64 * 1024
    G.free()


@pytest.mark.parametrize("mode", ["plain", "persistent", "staged"])
def test_walk_keeps_no_device_memory(mode):
    """Repeated walks into a caller-owned row buffer leave the device's free
    memory unchanged, apart from what torch's own allocator reserves."""
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    g = _graph()
    G = fw.Graph.of(g)
    n, L = 100_000, 40
    starts = torch.from_numpy(np.arange(n, dtype=np.int32) % g.n_vertices).cuda()
    out = torch.empty((n, L + 1), dtype=torch.int32, device="cuda")
    assert out.numel() * 4 == n * (L + 1) * 4
    prm = fw.make_params(fw.node2vec_factors(2, 1, 1, 2))
    fw.walk(G, "node2vec", prm, starts, L, 7, out=out, mode=mode)  # first launch loads code
    free0, res0 = _free(torch), torch.cuda.memory_reserved()
    for seed in range(3):
        fw.walk(G, "node2vec", prm, starts, L, seed, out=out, mode=mode)
    free1, res1 = _free(torch), torch.cuda.memory_reserved()
    assert (free0 - free1) - (res1 - res0) <= 2 * MiB
    G.free()
