"""Sampler microbenchmark tasks (GPU) against the oracle, bit-exact, for
every sampler: task sizes below, at and past one wavefront, one 256-entry
chunk and several group levels, ragged ends at the array end, zero-weight
entries and all-zero tasks; uniform and log-normal (sigma 1..3) weights."""
import numpy as np
import pytest

import oracle
from gpu_common import torch_or_skip

pytestmark = pytest.mark.gpu

SAMPLERS = ["its", "dprs", "zprs", "its_buffered", "alias", "rejection"]


@pytest.fixture(scope="module")
def env():
    torch = torch_or_skip()
    from paper_2404_08364_amd import flowwalk as fw
    return torch, fw


def _weights(n_tasks, size, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        w = rng.integers(1, 256, n_tasks * size)
    else:
        sigma = {"ln1": 1.0, "ln2": 2.0, "ln3": 3.0}[kind]
        w = np.minimum(np.floor(rng.lognormal(0, sigma, n_tasks * size) * 16), 2**32 - 1)
        w[rng.random(n_tasks * size) < 0.05] = 0
    w = w.astype(np.uint32)
    if n_tasks > 2:
        w[size:2 * size] = 0  # task 1 has no positive weight
    return w


def _check(env, sampler, size, n_tasks, kind, seed=12345):
    torch, fw = env
    w = _weights(n_tasks, size, kind, size * 7 + n_tasks)
    wt = torch.from_numpy(w.view(np.int32)).cuda()
    got = fw.sample_tasks(sampler, wt, size, seed).cpu().numpy().astype(np.int64)
    exp = oracle.sample_tasks(sampler, w, size, seed)
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, (sampler, size, kind, bad[:5], got[bad[:5]], exp[bad[:5]])
    return got


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("size,n_tasks", [(1, 500), (3, 500), (63, 300), (64, 300), (65, 300),
                                          (257, 200), (1000, 100), (4099, 40)])
@pytest.mark.parametrize("kind", ["uniform", "ln1", "ln3"])
def test_tasks_match_oracle(env, sampler, size, n_tasks, kind):
    got = _check(env, sampler, size, n_tasks, kind)
    assert got[1] == -1


@pytest.mark.parametrize("sampler", ["its", "dprs", "zprs", "its_buffered", "rejection"])
def test_large_tasks(env, sampler):
    _check(env, sampler, 70_001, 6, "ln2")
