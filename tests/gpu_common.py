"""Shared helpers for the GPU tests (they call the library through its C ABI
via the ctypes binding and compare with the oracle)."""
from __future__ import annotations

import numpy as np

import oracle

END = 0xFFFFFFFF


def torch_or_skip():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_walk(torch, fw, G, algo, prm, starts_np, length, seed, mode, **kw):
    st = torch.from_numpy(np.ascontiguousarray(starts_np, dtype=np.int32)).cuda()
    out = fw.walk(G, algo, prm, st, length, seed, mode=mode, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def oracle_params(algo, factors=(1, 1, 1), schema=()):
    return oracle.params(*factors, schema=schema)


def assert_rows_equal(got, exp, what=""):
    if not np.array_equal(got, exp):
        bad = np.nonzero((got != exp).any(axis=1))[0]
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} rows differ; first row {i}:\n"
                             f"gpu    {got[i].tolist()}\noracle {exp[i].tolist()}")
