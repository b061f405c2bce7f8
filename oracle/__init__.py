"""ctypes binding of the CPU oracle (``fw_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain single-threaded definition
of what a walk computes; the HIP library is checked against it bit for bit.
Only the test suite, the smoke check and the bench's CPU-baseline leg import
this module.  It shares no code with the library.
"""
from __future__ import annotations

import concurrent.futures as _cf
import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "fw_oracle.c"
_LIB = _HERE / "libfworacle.so"
_lib = None

OK, EINVAL, ENOMEM, EOVERFLOW = 0, -1, -2, -3
DEEPWALK, NODE2VEC, METAPATH, PPR = 0, 1, 2, 3
ALGOS = {"deepwalk": DEEPWALK, "node2vec": NODE2VEC, "metapath": METAPATH, "ppr": PPR}
END = 0xFFFFFFFF
SAMPLERS = {"its": 0, "dprs": 1, "zprs": 2}
ZPRS_LANES = 64


class Params(ctypes.Structure):
    _fields_ = [("f_ret", ctypes.c_uint32), ("f_in", ctypes.c_uint32),
                ("f_out", ctypes.c_uint32), ("schema_len", ctypes.c_uint32),
                ("schema", ctypes.c_uint8 * 16),
                ("stop_num", ctypes.c_uint32), ("stop_den", ctypes.c_uint32)]


class _Graph(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint64), ("n_edges", ctypes.c_uint64),
                ("offsets", ctypes.c_void_p), ("adj", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("labels", ctypes.c_void_p)]


def build(force: bool = True) -> Path:
    """Compile libfworacle.so with gcc (plain C, -O2)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Werror",
                        str(_SRC), "-o", str(tmp)], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB.exists():
        build(force=False)
    _lib = bind(ctypes.CDLL(str(_LIB)))
    return _lib


def bind(lib):
    """Declares the C signatures on a loaded oracle library."""
    u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    pg, pp = ctypes.POINTER(_Graph), ctypes.POINTER(Params)
    lib.fwo_philox4x64_10.argtypes = [vp, vp, vp]
    lib.fwo_philox4x64_10.restype = None
    lib.fwo_draw.argtypes = [u64, u64, u64]
    lib.fwo_draw.restype = u64
    lib.fwo_stop_coin.argtypes = [u64, u32, u32]
    lib.fwo_stop_coin.restype = i32
    lib.fwo_stop.argtypes = [u64, u64, u64, u32, u32]
    lib.fwo_stop.restype = i32
    lib.fwo_entry_draw.argtypes = [u64, u64, u64, u64]
    lib.fwo_entry_draw.restype = u64
    lib.fwo_zigzag_order.argtypes = [u64, u32, vp]
    lib.fwo_zigzag_order.restype = None
    lib.fwo_reservoir.argtypes = [vp, vp, vp, u64]
    lib.fwo_reservoir.restype = ctypes.c_int64
    lib.fwo_walk_sampler.argtypes = [pg, i32, pp, i32, vp, u64, u32, u64, u64, vp]
    lib.fwo_walk_sampler.restype = i32
    lib.fwo_alias_table.argtypes = [vp, u32, vp, vp]
    lib.fwo_alias_table.restype = u64
    lib.fwo_sample_task.argtypes = [i32, vp, u32, u64, u64]
    lib.fwo_sample_task.restype = ctypes.c_int64
    lib.fwo_scale.argtypes = [u64, u64]
    lib.fwo_scale.restype = u64
    lib.fwo_pick.argtypes = [vp, u64, u64]
    lib.fwo_pick.restype = ctypes.c_int64
    lib.fwo_node2vec_factors.argtypes = [u32, u32, u32, u32, pp]
    lib.fwo_validate.argtypes = [pg]
    lib.fwo_transition_weights.argtypes = [pg, i32, pp, u32, u32, u32, vp]
    lib.fwo_walk.argtypes = [pg, i32, pp, vp, u64, u32, u64, u64, vp]
    lib.fwo_walk_ids.argtypes = [pg, i32, pp, vp, vp, u64, u32, u64, vp]
    for f in ("fwo_node2vec_factors", "fwo_validate", "fwo_transition_weights", "fwo_walk",
              "fwo_walk_ids"):
        getattr(lib, f).restype = i32
    return lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what} failed with status {status}")
        self.status = status


def _c(a, dtype):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


class HostGraph:
    """Keeps contiguous host arrays alive and exposes the C view."""

    def __init__(self, offsets, adj, weights=None, labels=None):
        self.offsets = _c(offsets, np.uint64)
        self.adj = _c(adj, np.uint32)
        self.weights = _c(weights, np.uint32)
        self.labels = _c(labels, np.uint8)
        self.c = _Graph(self.offsets.shape[0] - 1, self.adj.shape[0],
                        self.offsets.ctypes.data, self.adj.ctypes.data,
                        None if self.weights is None else self.weights.ctypes.data,
                        None if self.labels is None else self.labels.ctypes.data)

    @classmethod
    def of(cls, g) -> "HostGraph":
        if isinstance(g, HostGraph):
            return g
        return cls(g.offsets, g.adj, g.weights, g.labels)

    @property
    def n_vertices(self) -> int:
        return int(self.c.n_vertices)


def params(f_ret=1, f_in=1, f_out=1, schema=(), stop=(0, 1)) -> Params:
    p = Params()
    p.f_ret, p.f_in, p.f_out = f_ret, f_in, f_out
    p.stop_num, p.stop_den = stop
    p.schema_len = len(schema)
    for i, s in enumerate(schema):
        p.schema[i] = s
    return p


def node2vec_factors(p_num: int, p_den: int, q_num: int, q_den: int) -> tuple[int, int, int]:
    out = Params()
    rc = _load().fwo_node2vec_factors(p_num, p_den, q_num, q_den, ctypes.byref(out))
    if rc:
        raise OracleError(rc, "fwo_node2vec_factors")
    return out.f_ret, out.f_in, out.f_out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().fwo_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def draw(seed: int, qid: int, t: int) -> int:
    return int(_load().fwo_draw(seed, qid, t))


def stop_coin(u1: int, stop_num: int, stop_den: int) -> bool:
    return bool(_load().fwo_stop_coin(u1, stop_num, stop_den))


def stop(seed: int, qid: int, t: int, stop_num: int, stop_den: int) -> bool:
    return bool(_load().fwo_stop(seed, qid, t, stop_num, stop_den))


def scale(u: int, total: int) -> int:
    return int(_load().fwo_scale(u, total))


def pick(w, r: int) -> int:
    a = np.ascontiguousarray(w, dtype=np.uint64)
    return int(_load().fwo_pick(a.ctypes.data, a.shape[0], r))


def validate(g) -> int:
    hg = HostGraph.of(g)
    return int(_load().fwo_validate(ctypes.byref(hg.c)))


def transition_weights(g, algo, prm: Params | None, prev: int, cur: int, t: int) -> np.ndarray:
    hg = HostGraph.of(g)
    d = int(hg.offsets[cur + 1] - hg.offsets[cur]) if 0 <= cur < hg.n_vertices else 0
    out = np.zeros(max(d, 1), dtype=np.uint64)
    a = ALGOS.get(algo, algo)
    rc = _load().fwo_transition_weights(ctypes.byref(hg.c), a,
                                        None if prm is None else ctypes.byref(prm),
                                        prev, cur, t, out.ctypes.data)
    if rc:
        raise OracleError(rc, "fwo_transition_weights")
    return out[:d]


def walk_status(g, algo, prm, starts, length: int, seed: int, qid_base: int = 0,
                sampler="its"):
    """Returns (status, paths); paths is uint32[n, length+1]."""
    hg = HostGraph.of(g)
    st = np.ascontiguousarray(starts, dtype=np.uint32)
    out = np.zeros((st.shape[0], length + 1), dtype=np.uint32)
    a = ALGOS.get(algo, algo)
    smp = SAMPLERS.get(sampler, sampler)
    rc = _load().fwo_walk_sampler(ctypes.byref(hg.c), a,
                                  None if prm is None else ctypes.byref(prm), smp,
                                  st.ctypes.data, st.shape[0], length, seed, qid_base,
                                  out.ctypes.data)
    return int(rc), out


def walk(g, algo, prm, starts, length: int, seed: int, qid_base: int = 0,
         sampler="its") -> np.ndarray:
    rc, out = walk_status(g, algo, prm, starts, length, seed, qid_base, sampler)
    if rc:
        raise OracleError(rc, "fwo_walk")
    return out


TASK_SAMPLERS = {"its": 0, "dprs": 1, "zprs": 2, "its_buffered": 3, "alias": 4, "rejection": 5}
RJS_MAX_TRIALS = 1 << 24


def alias_table(w):
    """(T, prob uint64[n], alias uint32[n]) of the sweep construction."""
    a = np.ascontiguousarray(w, dtype=np.uint32)
    n = a.shape[0]
    prob = np.zeros(max(n, 1), dtype=np.uint64)
    alias = np.zeros(max(n, 1), dtype=np.uint32)
    T = int(_load().fwo_alias_table(a.ctypes.data, n, prob.ctypes.data, alias.ctypes.data))
    return T, prob[:n], alias[:n]


def sample_task(sampler, w, seed: int, task: int) -> int:
    a = np.ascontiguousarray(w, dtype=np.uint32)
    return int(_load().fwo_sample_task(TASK_SAMPLERS.get(sampler, sampler), a.ctypes.data,
                                       a.shape[0], seed, task))


def sample_tasks(sampler, weights, size: int, seed: int) -> np.ndarray:
    """Picks of every task of the flat weight array (task j = weights[j*size:(j+1)*size])."""
    a = np.ascontiguousarray(weights, dtype=np.uint32)
    n = a.shape[0] // size
    out = np.empty(n, dtype=np.int64)
    for j in range(n):
        out[j] = sample_task(sampler, a[j * size:(j + 1) * size], seed, j)
    return out


def entry_draw(seed: int, qid: int, t: int, i: int) -> int:
    return int(_load().fwo_entry_draw(seed, qid, t, i))


def zigzag_order(d: int, k: int = ZPRS_LANES) -> np.ndarray:
    out = np.zeros(max(d, 1), dtype=np.uint64)
    _load().fwo_zigzag_order(d, k, out.ctypes.data)
    return out[:d]


def reservoir(w, u, order) -> int:
    w = np.ascontiguousarray(w, dtype=np.uint64)
    u = np.ascontiguousarray(u, dtype=np.uint64)
    o = np.ascontiguousarray(order, dtype=np.uint64)
    return int(_load().fwo_reservoir(w.ctypes.data, u.ctypes.data, o.ctypes.data, w.shape[0]))


def walk_ids(g, algo, prm, starts, qids, length: int, seed: int) -> np.ndarray:
    hg = HostGraph.of(g)
    st = np.ascontiguousarray(starts, dtype=np.uint32)
    q = np.ascontiguousarray(qids, dtype=np.uint64)
    out = np.zeros((q.shape[0], length + 1), dtype=np.uint32)
    a = ALGOS.get(algo, algo)
    rc = _load().fwo_walk_ids(ctypes.byref(hg.c), a, None if prm is None else ctypes.byref(prm),
                              st.ctypes.data, q.ctypes.data, q.shape[0], length, seed,
                              out.ctypes.data)
    if rc:
        raise OracleError(rc, "fwo_walk_ids")
    return out


def walk_ids_threaded(g, algo, prm, starts, qids, length: int, seed: int,
                      threads: int) -> np.ndarray:
    """Same result as walk_ids; query shards run on `threads` host threads
    (each shard is a plain single-threaded oracle call; ctypes drops the GIL)."""
    q = np.ascontiguousarray(qids, dtype=np.uint64)
    hg = HostGraph.of(g)
    if threads <= 1 or q.shape[0] < 2 * threads:
        return walk_ids(hg, algo, prm, starts, q, length, seed)
    shards = np.array_split(q, threads * 4)
    with _cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda s: walk_ids(hg, algo, prm, starts, s, length, seed), shards))
    return np.concatenate(parts, axis=0)
