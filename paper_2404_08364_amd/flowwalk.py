"""Python binding of libflowwalk.so (argument marshalling only).

Every hop of every walk runs in the library's HIP kernels; this module only
converts arguments.  PyTorch supplies device memory and streams: ``starts``
and ``out`` are CUDA (HIP) tensors.  There is no CPU fallback: if the native
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libflowwalk.so"

OK, EINVAL, ENOMEM, EOVERFLOW, EHIP, ECANCELED = 0, -1, -2, -3, -4, -5
DEEPWALK, NODE2VEC, METAPATH, PPR = 0, 1, 2, 3
ALGOS = {"deepwalk": DEEPWALK, "node2vec": NODE2VEC, "metapath": METAPATH, "ppr": PPR}
MODES = {"auto": 0, "plain": 1, "persistent": 2, "staged": 3}
END = 0xFFFFFFFF

if not LIB_PATH.exists():
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2404_08364_amd.build` "
        "(hipcc, gfx950); there is no fallback path")


class Csr(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint64), ("n_edges", ctypes.c_uint64),
                ("offsets", ctypes.c_void_p), ("adj", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("f_ret", ctypes.c_uint32), ("f_in", ctypes.c_uint32),
                ("f_out", ctypes.c_uint32), ("schema_len", ctypes.c_uint32),
                ("schema", ctypes.c_uint8 * 16),
                ("stop_num", ctypes.c_uint32), ("stop_den", ctypes.c_uint32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint64), ("n_edges", ctypes.c_uint64),
                ("max_degree", ctypes.c_uint64), ("max_weight", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("weighted", ctypes.c_int),
                ("labelled", ctypes.c_int), ("device", ctypes.c_int)]


class Tune(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("tiny_max", ctypes.c_uint32), ("hub_min", ctypes.c_uint32),
                ("wgs_per_cu", ctypes.c_uint32), ("fetch", ctypes.c_uint32),
                ("hash_cells", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("sparse_ratio", ctypes.c_uint32)]


class WalkOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("stream", ctypes.c_void_p), ("async_", ctypes.c_int),
                ("qid_base", ctypes.c_uint64), ("tune", ctypes.POINTER(Tune)),
                ("use_graph", ctypes.c_int), ("sampler", ctypes.c_int)]


SAMPLERS = {"its": 0, "dprs": 1, "zprs": 2}


class BatchOpts(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_uint64), ("max_batch_queries", ctypes.c_uint64),
                ("mode", ctypes.c_int), ("batch_queries", ctypes.c_uint64),
                ("batches", ctypes.c_uint32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_batch_requests", ctypes.c_uint32), ("small_max_queries", ctypes.c_uint32),
                ("express_max_queries", ctypes.c_uint32)]


class ReqStats(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("n", ctypes.c_uint64), ("length", ctypes.c_uint32),
                ("status", ctypes.c_int), ("steps", ctypes.c_uint64)]


def _bind(lib):
    u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    sig = {
        "fw_graph_upload": ([ctypes.POINTER(Csr), vp, vp, ctypes.POINTER(vp)], i32),
        "fw_graph_free": ([vp], i32),
        "fw_graph_info_get": ([vp, ctypes.POINTER(GraphInfo)], i32),
        "fw_node2vec_factors": ([u32, u32, u32, u32, ctypes.POINTER(Params)], i32),
        "fw_walk": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64, vp], i32),
        "fw_walk_ex": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64, vp,
                        ctypes.POINTER(WalkOpts)], i32),
        "fw_walk_noalloc": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64, vp, vp], i32),
        "fw_sync": ([vp, vp], i32),
        "fw_count_steps": ([vp, u64, u32, vp, ctypes.POINTER(u64)], i32),
        "fw_sample_tasks": ([i32, vp, u64, u32, u64, vp, vp], i32),
        "fw_walk_host": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64, vp,
                          ctypes.POINTER(BatchOpts)], i32),
        "fw_autotune": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64, vp,
                         ctypes.POINTER(Tune)], i32),
        "fw_server_create": ([vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)], i32),
        "fw_server_submit": ([vp, i32, ctypes.POINTER(Params), vp, u64, u32, u64,
                              ctypes.POINTER(u64)], i32),
        "fw_server_poll": ([vp, u64], i32),
        "fw_server_wait": ([vp, u64, vp, ctypes.POINTER(ReqStats)], i32),
        "fw_server_destroy": ([vp], i32),
        "fw_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


# torch's ROCm wheel ships its own HIP runtime under a different file name.
# Loading it first lets the dynamic linker resolve this library's HIP
# dependency to that same copy: two HIP runtimes in one process would each
# try to own the GPU, and the second would find none.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = _bind(ctypes.CDLL(str(LIB_PATH)))


def lib():
    return _lib


class FWError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.fw_last_error().decode(errors="replace")
        super().__init__(f"{what}: status {status}: {msg}")
        self.status = status


def _check(rc: int, what: str):
    if rc != OK:
        raise FWError(rc, what)


def node2vec_factors(p_num: int, p_den: int, q_num: int, q_den: int) -> tuple[int, int, int]:
    out = Params()
    _check(_lib.fw_node2vec_factors(p_num, p_den, q_num, q_den, ctypes.byref(out)),
           "fw_node2vec_factors")
    return out.f_ret, out.f_in, out.f_out


def make_params(factors=(1, 1, 1), schema=(), stop=(0, 1)) -> Params:
    """node2vec factors, MetaPath schema, PPR stop chance (num, den)."""
    p = Params()
    p.f_ret, p.f_in, p.f_out = factors
    p.stop_num, p.stop_den = stop
    p.schema_len = len(schema)
    for i, s in enumerate(schema):
        p.schema[i] = s
    return p


def make_tune(**kw) -> Tune:
    t = Tune()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


class Graph:
    """A CSR graph resident in HBM (owned by the library)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def upload(cls, offsets, adj, weights=None, labels=None) -> "Graph":
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        a = np.ascontiguousarray(adj, dtype=np.uint32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
        lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint8)
        csr = Csr(off.shape[0] - 1, a.shape[0], off.ctypes.data, a.ctypes.data)
        h = ctypes.c_void_p()
        _check(_lib.fw_graph_upload(ctypes.byref(csr), None if w is None else w.ctypes.data,
                                    None if lab is None else lab.ctypes.data, ctypes.byref(h)),
               "fw_graph_upload")
        return cls(h.value)

    @classmethod
    def of(cls, g) -> "Graph":
        """Uploads any object with offsets/adj/weights/labels arrays."""
        return cls.upload(g.offsets, g.adj, getattr(g, "weights", None),
                          getattr(g, "labels", None))

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None or not self._h.value:
            raise ValueError("graph was freed")
        return self._h

    def info(self) -> dict:
        gi = GraphInfo()
        _check(_lib.fw_graph_info_get(self.handle, ctypes.byref(gi)), "fw_graph_info_get")
        return {k: getattr(gi, k) for k, _ in GraphInfo._fields_}

    def free(self):
        if self._h is not None and self._h.value:
            _lib.fw_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def walk_ptr(graph: Graph, algo, prm: Params | None, starts_ptr: int, n: int, length: int,
             seed: int, out_ptr: int, mode="auto", stream=None, async_=False, qid_base=0,
             tune: Tune | None = None, use_graph=False, sampler="its") -> int:
    """Raw-pointer form of fw_walk_ex; returns the status."""
    o = WalkOpts()
    o.sampler = SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.stream = _stream_handle(stream)
    o.async_ = int(bool(async_))
    o.qid_base = qid_base
    o.tune = ctypes.pointer(tune) if tune is not None else None
    o.use_graph = int(bool(use_graph))
    a = ALGOS.get(algo, algo)
    return _lib.fw_walk_ex(graph.handle, a, None if prm is None else ctypes.byref(prm),
                           starts_ptr, n, length, seed, out_ptr, ctypes.byref(o))


def walk(graph: Graph, algo, prm: Params | None, starts, length: int, seed: int, out=None,
         mode="auto", stream=None, async_=False, qid_base=0, tune: Tune | None = None,
         use_graph=False, sampler="its"):
    """Runs len(starts) queries; returns the int32 tensor [n, length + 1]
    (FW_END reads as -1).  sampler: "its" (any mode), "dprs" or "zprs"
    (mode "plain")."""
    import torch
    if starts.device.type != "cuda":
        raise ValueError("starts must be a device tensor")
    if starts.dtype not in (torch.int32, torch.uint32):
        raise ValueError("starts must be int32 or uint32")
    starts = starts.contiguous()
    n = starts.shape[0]
    if out is None:
        out = torch.empty((n, length + 1), dtype=torch.int32, device=starts.device)
    if out.dtype not in (torch.int32, torch.uint32) or not out.is_contiguous() \
            or out.numel() != n * (length + 1):
        raise ValueError("out must be a contiguous int32 tensor of n * (length + 1) entries")
    if stream is None:
        stream = torch.cuda.current_stream(starts.device)
    rc = walk_ptr(graph, algo, prm, starts.data_ptr(), n, length, seed, out.data_ptr(), mode,
                  stream, async_, qid_base, tune, use_graph, sampler)
    _check(rc, "fw_walk_ex")
    return out


def walk_noalloc(graph: Graph, algo, prm: Params | None, starts, out, length: int, seed: int,
                 stream=None):
    """fw_walk_noalloc: enqueues the persistent walk into the caller's `out`
    (contiguous int32 [n, length + 1]) on `stream` without allocating and
    without waiting; fw_sync (sync()) reports a bad start vertex."""
    import torch
    if starts.device.type != "cuda" or out.device.type != "cuda":
        raise ValueError("starts and out must be device tensors")
    if starts.dtype not in (torch.int32, torch.uint32) or not starts.is_contiguous():
        raise ValueError("starts must be a contiguous int32 tensor")
    n = starts.shape[0]
    if out.dtype not in (torch.int32, torch.uint32) or not out.is_contiguous() \
            or out.numel() != n * (length + 1):
        raise ValueError("out must be a contiguous int32 tensor of n * (length + 1) entries")
    if stream is None:
        stream = torch.cuda.current_stream(starts.device)
    a = ALGOS.get(algo, algo)
    rc = _lib.fw_walk_noalloc(graph.handle, a, None if prm is None else ctypes.byref(prm),
                              starts.data_ptr(), n, length, seed, out.data_ptr(),
                              _stream_handle(stream))
    _check(rc, "fw_walk_noalloc")
    return out


def autotune(graph: Graph, algo, prm: Params | None, starts, length: int, seed: int,
             stream=None) -> dict:
    """Tunes the persistent and the staged form on the queries of `starts` (a
    device tensor holding a sample of the workload) and returns the faster
    configuration ("mode" names its form: 2 persistent, 3 staged)."""
    import torch
    starts = starts.contiguous()
    if stream is None:
        stream = torch.cuda.current_stream(starts.device)
    best = Tune()
    a = ALGOS.get(algo, algo)
    _check(_lib.fw_autotune(graph.handle, a, None if prm is None else ctypes.byref(prm),
                            starts.data_ptr(), starts.shape[0], length, seed,
                            _stream_handle(stream), ctypes.byref(best)), "fw_autotune")
    return {k: getattr(best, k) for k, _ in Tune._fields_}


def walk_host(graph: Graph, algo, prm: Params | None, starts, length: int, seed: int,
              device_budget_bytes: int = 0, max_batch_queries: int = 0, mode="auto"):
    """Runs the queries of `starts` (host uint32 array) with rows in host
    memory, in ping-pong batches that fit the device budget.  Returns
    (rows uint32[n, length + 1], queries per batch, batches)."""
    st = np.ascontiguousarray(starts, dtype=np.uint32)
    out = np.empty((st.shape[0], length + 1), dtype=np.uint32)
    o = BatchOpts()
    o.device_budget_bytes = device_budget_bytes
    o.max_batch_queries = max_batch_queries
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    a = ALGOS.get(algo, algo)
    _check(_lib.fw_walk_host(graph.handle, a, None if prm is None else ctypes.byref(prm),
                             st.ctypes.data, st.shape[0], length, seed, out.ctypes.data,
                             ctypes.byref(o)), "fw_walk_host")
    return out, int(o.batch_queries), int(o.batches)


TASK_SAMPLERS = {"its": 0, "dprs": 1, "zprs": 2, "its_buffered": 3, "alias": 4, "rejection": 5}


def sample_tasks(sampler, weights, size: int, seed: int, picks=None, stream=None):
    """Sampler microbenchmark: task j picks an index of weights[j*size:(j+1)*size]
    (a contiguous int32/uint32 device tensor); returns the int32 picks (-1 =
    END)."""
    import torch
    weights = weights.contiguous()
    n = weights.numel() // size
    if picks is None:
        picks = torch.empty(n, dtype=torch.int32, device=weights.device)
    if stream is None:
        stream = torch.cuda.current_stream(weights.device)
    smp = TASK_SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
    _check(_lib.fw_sample_tasks(smp, weights.data_ptr(), n, size, seed, picks.data_ptr(),
                                _stream_handle(stream)), "fw_sample_tasks")
    return picks


def count_steps(paths, stream=None) -> int:
    """Realised hops of a walk result: the entries of columns 1.. of the
    (n, length + 1) device tensor `paths` that are not END."""
    import torch
    paths = paths.contiguous()
    if stream is None:
        stream = torch.cuda.current_stream(paths.device)
    out = ctypes.c_uint64(0)
    _check(_lib.fw_count_steps(paths.data_ptr(), paths.shape[0], paths.shape[1] - 1,
                               _stream_handle(stream), ctypes.byref(out)), "fw_count_steps")
    return int(out.value)


def sync(graph: Graph, stream=None):
    _check(_lib.fw_sync(graph.handle, _stream_handle(stream)), "fw_sync")


class Server:
    """Continuous-batching walk server over one resident graph.

    submit() takes host start vertices (numpy) and returns a ticket; wait()
    returns the uint32 paths [n, length + 1] and the request's timestamps."""

    def __init__(self, graph: Graph, mem_budget_bytes: int = 1 << 30, max_inflight: int = 3,
                 max_batch_requests: int = 256, small_max_queries: int = 0,
                 express_max_queries: int = 0):
        self.graph = graph
        o = ServerOpts(mem_budget_bytes, max_inflight, max_batch_requests, small_max_queries,
                       express_max_queries)
        h = ctypes.c_void_p()
        _check(_lib.fw_server_create(graph.handle, ctypes.byref(o), ctypes.byref(h)),
               "fw_server_create")
        self._h = h
        self._shapes = {}

    def submit(self, algo, prm: Params | None, starts, length: int, seed: int) -> int:
        st = np.ascontiguousarray(starts, dtype=np.uint32)
        t = ctypes.c_uint64()
        a = ALGOS.get(algo, algo)
        _check(_lib.fw_server_submit(self._h, a, None if prm is None else ctypes.byref(prm),
                                     st.ctypes.data, st.shape[0], length, seed, ctypes.byref(t)),
               "fw_server_submit")
        self._shapes[t.value] = (st.shape[0], length + 1)
        return t.value

    def poll(self, ticket: int) -> bool:
        rc = _lib.fw_server_poll(self._h, ticket)
        if rc < 0:
            raise FWError(rc, "fw_server_poll")
        return rc == 1

    def wait(self, ticket: int, rows: bool = True):
        """Returns (rows as uint32 [n, length + 1], stats); rows=False skips
        the copy of the rows and returns None for them."""
        shape = self._shapes.pop(ticket)
        out = np.empty(shape, dtype=np.uint32) if rows else None
        st = ReqStats()
        _check(_lib.fw_server_wait(self._h, ticket, out.ctypes.data if rows else None,
                                   ctypes.byref(st)), "fw_server_wait")
        return out, {k: getattr(st, k) for k, _ in ReqStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            _lib.fw_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
