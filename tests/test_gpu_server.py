"""Served form (GPU): every request's walks equal the oracle's and fw_walk's
on the same starts and seed, alone and in a concurrent mix of algorithms,
lengths and sizes; admission by memory; cancellation on shutdown."""
import threading

import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_rows_equal, gpu_walk, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    g = synth.chung_lu(30_000, 400_000, 2.1, 1.5, seed=11)
    g.weights = synth.weights_uniform(g, 1, 255, 12)
    g.labels = synth.labels_uniform(g, 5, 13)
    return torch, fw, g, fw.Graph.of(g)


KINDS = [("deepwalk", (1, 1, 1), ()), ("node2vec", (1, 2, 4), ()), ("metapath", (1, 1, 1), (0, 1, 2)),
         ("ppr", (1, 1, 1), ())]
STOP = {"ppr": (1, 5)}


def _fw_params(fw, algo, f, sch):
    return fw.make_params(f, sch, STOP.get(algo, (0, 1)))


def _oracle_params(algo, f, sch):
    return oracle.params(*f, schema=sch, stop=STOP.get(algo, (0, 1)))


def _requests(g, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        algo, f, sch = KINDS[i % len(KINDS)]
        n = int(np.exp(rng.uniform(0, np.log(3000))))
        L = int(rng.integers(10, 81))
        starts = rng.integers(0, g.n_vertices, n).astype(np.uint32)
        reqs.append((algo, f, sch, starts, L, int(rng.integers(0, 1 << 40))))
    return reqs


@pytest.mark.parametrize("small_max,express", [(0, 0), (2048, 0), (1 << 30, 0), (0, 500),
                                               (0, 1 << 30)])
def test_mix_equals_alone_and_oracle(env, small_max, express):
    """small_max: one phase per batch, batches split into small and large
    requests, every request small; express: no express lane, one for the
    requests of at most 500 queries, one every request may take."""
    torch, fw, g, G = env
    reqs = _requests(g, 24, 1)
    srv = fw.Server(G, mem_budget_bytes=64 << 20, max_inflight=4, max_batch_requests=8,
                    small_max_queries=small_max, express_max_queries=express)
    try:
        # Submitted from several threads at once, so they mix on the GPU.
        tickets = [None] * len(reqs)

        def sub(idx):
            for i in idx:
                algo, f, sch, st, L, seed = reqs[i]
                tickets[i] = srv.submit(algo, _fw_params(fw, algo, f, sch), st, L, seed)

        th = [threading.Thread(target=sub, args=(range(k, len(reqs), 3),)) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (algo, f, sch, st, L, seed), (paths, stats) in zip(reqs, results):
        exp = oracle.walk(g, algo, _oracle_params(algo, f, sch), st, L, seed)
        assert_rows_equal(paths, exp, f"served {algo} n={len(st)} L={L}")
        assert stats["status"] == 0 and stats["done_ns"] >= stats["admit_ns"] >= stats["submit_ns"]
        assert stats["steps"] == int((paths[:, 1:] != 0xFFFFFFFF).sum())
        alone = gpu_walk(torch, fw, G, algo, _fw_params(fw, algo, f, sch), st, L, seed, "persistent")
        assert_rows_equal(paths, alone, "served vs alone")


def test_admission_by_memory(env):
    """A budget that holds only a few requests at a time still serves a long
    queue; a request larger than the whole budget is refused at submit."""
    torch, fw, g, G = env
    reqs = _requests(g, 12, 2)
    need = max(len(st) * 4 + len(st) * (L + 1) * 4 for (_, _, _, st, L, _) in reqs)
    srv = fw.Server(G, mem_budget_bytes=2 * need + 4096, max_inflight=2)
    try:
        tickets = [srv.submit(a, _fw_params(fw, a, f, s), st, L, sd) for (a, f, s, st, L, sd) in reqs]
        for (a, f, s, st, L, sd), t in zip(reqs, tickets):
            paths, _ = srv.wait(t)
            assert_rows_equal(paths, oracle.walk(g, a, _oracle_params(a, f, s), st, L, sd),
                              "admission")
        big = np.zeros(1_000_000, dtype=np.uint32)
        with pytest.raises(fw.FWError) as e:
            srv.submit("deepwalk", None, big, 80, 1)
        assert e.value.status == fw.ENOMEM
        with pytest.raises(fw.FWError) as e:
            srv.submit("deepwalk", None, np.array([g.n_vertices], np.uint32), 5, 1)
        assert e.value.status == fw.EINVAL
    finally:
        srv.close()


def test_waits_in_reverse_order_under_a_tight_budget(env):
    """The budget holds two requests at a time; the client waits for the
    last request first.  Finished requests that are not collected yet give
    their memory back, so every request is admitted and served."""
    torch, fw, g, G = env
    reqs = _requests(g, 8, 3)
    need = max(256 + len(st) * 4 + 256 + len(st) * (L + 1) * 4 for (_, _, _, st, L, _) in reqs)
    srv = fw.Server(G, mem_budget_bytes=2 * need, max_inflight=2, max_batch_requests=1)
    try:
        tickets = [srv.submit(a, _fw_params(fw, a, f, s), st, L, sd) for (a, f, s, st, L, sd) in reqs]
        for (a, f, s, st, L, sd), t in reversed(list(zip(reqs, tickets))):
            paths, stats = srv.wait(t)
            assert_rows_equal(paths, oracle.walk(g, a, _oracle_params(a, f, s), st, L, sd),
                              "reverse-order wait")
            assert stats["steps"] == int((paths[:, 1:] != 0xFFFFFFFF).sum())
    finally:
        srv.close()


def test_shutdown_cancels_queued(env):
    torch, fw, g, G = env
    srv = fw.Server(G, mem_budget_bytes=1 << 20, max_inflight=1, max_batch_requests=1)
    st = np.arange(2000, dtype=np.uint32)
    tickets = [srv.submit("node2vec", fw.make_params((1, 2, 4)), st, 60, i) for i in range(20)]
    srv.close()  # queued ones are cancelled, launched ones finish
    # The handle is gone: nothing more to wait on; the call must not hang.
    assert len(tickets) == 20


def test_one_wait_per_ticket(env):
    """Two threads wait for the same ticket through the C ABI: one gets the
    rows (equal to the oracle's), the other FW_EINVAL (the ticket is taken,
    or already released), and neither reads memory the other gave back."""
    import ctypes
    torch, fw, g, G = env
    srv = fw.Server(G, mem_budget_bytes=1 << 26)
    try:
        st = np.arange(3000, dtype=np.uint32)
        prm = fw.make_params((1, 2, 4))
        t = srv.submit("node2vec", prm, st, 80, 77)
        outs = [np.zeros((3000, 81), dtype=np.uint32) for _ in range(2)]
        rcs = [None, None]

        def wait(i):
            stats = fw.ReqStats()
            rcs[i] = fw._lib.fw_server_wait(srv._h, t, outs[i].ctypes.data, ctypes.byref(stats))

        th = [threading.Thread(target=wait, args=(i,)) for i in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=60)
        assert sorted(rcs) == sorted([fw.OK, fw.EINVAL]), rcs
        got = outs[rcs.index(fw.OK)]
        assert_rows_equal(got, oracle.walk(g, "node2vec", oracle.params(1, 2, 4), st, 80, 77),
                          "the one wait")
    finally:
        srv.close()
