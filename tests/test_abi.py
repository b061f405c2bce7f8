"""C ABI (CPU): the library loads, exports every symbol the header declares,
and rejects malformed input on the host before touching a device."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "flowwalk.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ["fw_graph_upload", "fw_graph_free", "fw_walk", "fw_walk_ex", "fw_sync",
                 "fw_node2vec_factors", "fw_last_error", "fw_graph_info_get", "fw_autotune",
                 "fw_count_steps", "fw_server_create", "fw_server_submit", "fw_server_poll",
                 "fw_server_wait", "fw_server_destroy", "fw_walk_noalloc", "fw_walk_host",
                 "fw_sample_tasks"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2404_08364_amd import flowwalk as fw
    lib = ctypes.CDLL(str(fw.LIB_PATH))
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_node2vec_factors_match_oracle_and_configs():
    import oracle
    from paper_2404_08364_amd import flowwalk as fw
    assert fw.node2vec_factors(2, 1, 1, 2) == (1, 2, 4)
    assert fw.node2vec_factors(1, 1, 2, 1) == (2, 2, 1)
    assert fw.node2vec_factors(1, 2, 2, 1) == (4, 2, 1)
    rng = np.random.default_rng(0)
    for _ in range(200):
        a = [int(x) for x in rng.integers(1, 1000, 4)]
        assert fw.node2vec_factors(*a) == oracle.node2vec_factors(*a)
    with pytest.raises(fw.FWError) as e:
        fw.node2vec_factors(0, 1, 1, 1)
    assert e.value.status == fw.EINVAL


def _upload_status(off, adj, weights=None, labels=None):
    from paper_2404_08364_amd import flowwalk as fw
    off = np.ascontiguousarray(off, dtype=np.uint64)
    adj = np.ascontiguousarray(adj, dtype=np.uint32)
    csr = fw.Csr(off.shape[0] - 1, adj.shape[0], off.ctypes.data, adj.ctypes.data)
    h = ctypes.c_void_p()
    return fw.lib().fw_graph_upload(ctypes.byref(csr), None, None, ctypes.byref(h))


@pytest.mark.parametrize("off,adj", [
    ([0, 2, 3], [1, 0, 0]),          # row 0 not ascending
    ([0, 1, 2], [1, 5]),             # id out of range
    ([1, 1, 2], [1, 0]),             # offsets[0] != 0
    ([0, 2, 1], [1, 0]),             # offsets decrease
    ([0, 1, 3], [1, 0]),             # offsets[V] != E
])
def test_upload_rejects_malformed_csr(off, adj):
    from paper_2404_08364_amd import flowwalk as fw
    assert _upload_status(off, adj) == fw.EINVAL


def test_null_arguments():
    from paper_2404_08364_amd import flowwalk as fw
    lib = fw.lib()
    assert lib.fw_graph_upload(None, None, None, None) == fw.EINVAL
    assert lib.fw_walk(None, 0, None, None, 0, 0, 0, None) == fw.EINVAL
    assert lib.fw_graph_free(None) == fw.OK
    assert isinstance(lib.fw_last_error(), bytes)


def test_count_steps_rejects_null_on_host():
    """fw_count_steps checks its pointers before any device work."""
    from paper_2404_08364_amd import flowwalk as fw
    lib = fw.lib()
    n = ctypes.c_uint64(7)
    assert lib.fw_count_steps(None, 4, 3, None, None) == fw.EINVAL
    assert lib.fw_count_steps(None, 4, 3, None, ctypes.byref(n)) == fw.EINVAL
    assert lib.fw_count_steps(None, 0, 3, None, ctypes.byref(n)) == fw.OK and n.value == 0
    assert lib.fw_count_steps(None, 5, 0, None, ctypes.byref(n)) == fw.OK and n.value == 0
    assert lib.fw_count_steps(None, 1 << 62, 7, None, ctypes.byref(n)) == fw.EINVAL


def test_walk_host_checks_arguments_on_host():
    from paper_2404_08364_amd import flowwalk as fw
    lib = fw.lib()
    assert lib.fw_walk_host(None, 0, None, None, 4, 3, 1, None, None) == fw.EINVAL


def test_sample_tasks_checks_arguments_on_host():
    from paper_2404_08364_amd import flowwalk as fw
    lib = fw.lib()
    assert lib.fw_sample_tasks(9, None, 4, 3, 1, None, None) == fw.EINVAL
    assert lib.fw_sample_tasks(0, None, 0, 3, 1, None, None) == fw.OK
    assert lib.fw_sample_tasks(0, None, 4, 0, 1, None, None) == fw.EINVAL
    assert lib.fw_sample_tasks(0, None, 4, 3, 1, None, None) == fw.EINVAL


def test_sample_tasks_size_limit():
    from paper_2404_08364_amd import flowwalk as fw
    assert fw.lib().fw_sample_tasks(0, None, 4, 1 << 28, 1, None, None) == fw.EINVAL
