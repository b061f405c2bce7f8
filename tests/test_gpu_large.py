"""Parity on the two largest workloads (GPU through the C ABI, bit-exact
against the oracle on samples the oracle computes one query at a time):

* the 227M-vertex Chung-Lu graph (gamma 2.0, ~2.7 G stored edges, hubs of up
  to 2.84 M entries) with node2vec p=1/2 q=2 from all 10,000,000 uniform
  starts, 80 hops, in the persistent form: a strided sample of query ids
  plus queries whose walks pass through the highest-degree vertices;
* the served request mix on R-MAT scale 24 (DeepWalk, node2vec p=2 q=1/2,
  MetaPath [0,1,2]; sizes floor(log-uniform[1, 65536]); lengths U{10..80}):
  sampled rows of every request, submitted from a client thread with
  Poisson gaps while earlier requests run.

The phases of each workload are separate tests sharing a module fixture, so
that the runner reports progress between them."""
import os
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_rows_equal, torch_or_skip

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def c5():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    recipe = "chunglu227m_n2v"
    g = synth.load_recipe_graph(recipe, use_cache=False)
    walk = synth.RECIPES[recipe]["walk"]
    (pn, pd), (qn, qd) = walk["p"], walk["q"]
    f = fw.node2vec_factors(pn, pd, qn, qd)
    starts = synth.recipe_starts(recipe, g)
    G = fw.Graph.of(g)
    state = dict(torch=torch, fw=fw, g=g, G=G, f=f, L=walk["length"], seed=walk["seed"],
                 starts=starts)
    yield state
    G.free()


@pytest.mark.timeout(900)
def test_c5_graph_shape(c5):
    g = c5["g"]
    assert g.n_vertices == 227_000_000
    assert 2.6e9 < g.n_edges < 2.8e9
    assert c5["G"].info()["max_degree"] > (1 << 21)  # three-level locates happen
    assert c5["starts"].shape[0] == 10_000_000


@pytest.mark.timeout(900)
def test_c5_persistent_all_starts(c5):
    """One persistent launch over all 10,000,000 queries (about two minutes)."""
    torch, fw = c5["torch"], c5["fw"]
    st = torch.from_numpy(c5["starts"].view(np.int32)).cuda()
    out = fw.walk(c5["G"], "node2vec", fw.make_params(c5["f"]), st, c5["L"], c5["seed"],
                  mode="persistent")
    torch.cuda.synchronize()
    c5["out"] = out
    hops = int(fw.count_steps(out))
    # Starts are uniform over all vertices, and many of them have no
    # neighbour (their walks end at once): about 83% of the 800M hops happen.
    assert hops == int((out[:, 1:] != -1).sum())
    assert hops > 0.5 * 10_000_000 * c5["L"]


@pytest.mark.timeout(900)
def test_c5_parity_sample(c5):
    """8,192 strided query ids plus 256 queries whose walks visit the 64
    vertices of largest degree, recomputed by the oracle (about 35 s on 16
    host threads: these walks scan 144 K neighbours per hop on average)."""
    torch = c5["torch"]
    g, out = c5["g"], c5["out"]
    n = c5["starts"].shape[0]
    deg = g.degrees()
    top = np.argsort(deg)[::-1][:64].astype(np.uint32)
    strided = np.arange(0, n, n // 8192, dtype=np.uint64)[:8192]
    # Rows (on the device) that contain a top vertex after the start.
    hit = torch.isin(out[:, 1:], torch.from_numpy(top.view(np.int32)).cuda()).any(dim=1)
    hub_q = torch.nonzero(hit).flatten()[:256].cpu().numpy().astype(np.uint64)
    assert hub_q.size == 256
    qids = np.unique(np.concatenate([strided, hub_q]))
    got = out[torch.from_numpy(qids.astype(np.int64)).cuda()].cpu().numpy().view(np.uint32)
    exp = oracle.walk_ids_threaded(g, "node2vec", oracle.params(*c5["f"]), c5["starts"], qids,
                                   c5["L"], c5["seed"], THREADS)
    assert_rows_equal(got, exp, "chunglu227m_n2v persistent")
    del c5["out"]


@pytest.fixture(scope="module")
def c4():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    g = synth.load_recipe_graph("rmat24_serve", use_cache=False)
    G = fw.Graph.of(g)
    yield dict(torch=torch, fw=fw, g=g, G=G)
    G.free()


C4_ALGOS = [("deepwalk", (1, 1, 1), ()), ("node2vec", (1, 2, 4), ()),
            ("metapath", (1, 1, 1), (0, 1, 2))]


@pytest.mark.timeout(900)
def test_c4_served_mix_matches_oracle(c4):
    """96 requests of the R-MAT-24 mix at 2000 requests/s (Poisson gaps)
    through the server: up to 64 strided rows of every request (all rows of
    the small ones) equal the oracle's walks of the same request (query i
    of a request has id i and the request's seed)."""
    fw, g, G = c4["fw"], c4["g"], c4["G"]
    rng = np.random.default_rng(424242)
    n_req = 96
    gaps = rng.exponential(1 / 2000, n_req)
    sizes = np.floor(np.exp(rng.uniform(0, np.log(65536), n_req))).astype(np.int64)
    kinds = rng.integers(0, 3, n_req)
    lengths = rng.integers(10, 81, n_req)
    seeds = rng.integers(0, 1 << 62, n_req)
    starts = [synth.uniform_ids(int(sizes[i]), g.n_vertices, 500 + i) for i in range(n_req)]
    srv = fw.Server(G, mem_budget_bytes=1 << 30, max_inflight=4, max_batch_requests=512)
    tickets = [None] * n_req

    def client():
        for i in range(n_req):
            time.sleep(float(gaps[i]))
            algo, f, sch = C4_ALGOS[kinds[i]]
            tickets[i] = srv.submit(algo, fw.make_params(f, sch), starts[i], int(lengths[i]),
                                    int(seeds[i]))

    th = threading.Thread(target=client)
    th.start()
    th.join()
    rows = [srv.wait(t)[0] for t in tickets]
    srv.close()
    for i in range(n_req):
        algo, f, sch = C4_ALGOS[kinds[i]]
        n = int(sizes[i])
        qids = np.unique(np.arange(0, n, max(1, n // 64), dtype=np.uint64)[:64])
        exp = oracle.walk_ids(g, algo, oracle.params(*f, schema=sch), starts[i], qids,
                              int(lengths[i]), int(seeds[i]))
        assert rows[i].shape == (n, int(lengths[i]) + 1)
        assert_rows_equal(rows[i][qids.astype(np.int64)], exp,
                          f"request {i} ({algo}, n={n}, L={lengths[i]})")
