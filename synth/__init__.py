"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module generates graphs, edge attributes and start-vertex sets only; it
holds none of the random-walk method's arithmetic.  The heavy lifting is in
``fw_synth.cpp`` (built with g++ into ``libfwsynth.so`` next to this file).

The workload recipes in :data:`RECIPES` stand in for the paper's SNAP/LAW
graphs (Table 1 of the experiments section), which are not available: they are
power-law graphs of the same kind (R-MAT and Chung-Lu), with integer edge
weights and labels in {0..4} like the paper's labelled runs.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import subprocess
import weakref
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "fw_synth.cpp"
_LIB = _HERE / "libfwsynth.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile libfwsynth.so with g++ (host code only)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
               str(_SRC), "-o", str(tmp)]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB.exists():
        build(force=False)
    lib = ctypes.CDLL(str(_LIB))
    u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    pu64p = ctypes.POINTER(ctypes.POINTER(u64))
    pu32p = ctypes.POINTER(ctypes.POINTER(u32))
    vp = ctypes.c_void_p
    lib.synth_rmat.argtypes = [i32, u64, dbl, dbl, dbl, u64, i32, i32, pu64p, pu32p,
                               ctypes.POINTER(u64)]
    lib.synth_chung_lu.argtypes = [u64, u64, dbl, dbl, u64, i32, i32, pu64p, pu32p,
                                   ctypes.POINTER(u64)]
    lib.synth_free.argtypes = [vp]
    lib.synth_weights_uniform.argtypes = [vp, vp, u64, u32, u32, u64, i32, vp]
    lib.synth_weights_zipf.argtypes = [vp, vp, u64, dbl, u32, u64, i32, vp]
    lib.synth_labels_uniform.argtypes = [vp, vp, u64, u32, u64, i32, vp]
    lib.synth_uniform_ids.argtypes = [u64, u64, u64, i32, vp]
    _lib = lib
    return lib


def threads() -> int:
    env = os.environ.get("FW_SYNTH_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


def _adopt(ptr, n: int, ctype, dtype) -> np.ndarray:
    """Wrap a malloc'd buffer as a numpy array that frees it when collected."""
    lib = _load()
    if n == 0:
        lib.synth_free(ctypes.cast(ptr, ctypes.c_void_p))
        return np.zeros(0, dtype=dtype)
    buf = (ctype * n).from_address(ctypes.addressof(ptr.contents))
    weakref.finalize(buf, lib.synth_free, ctypes.cast(ptr, ctypes.c_void_p))
    return np.frombuffer(buf, dtype=dtype)


@dataclass
class Graph:
    """Host CSR graph: rows sorted ascending, no self-loops, no duplicates."""
    offsets: np.ndarray            # uint64[V+1]
    adj: np.ndarray                # uint32[E]
    weights: np.ndarray | None = None   # uint32[E] or None (unit weights)
    labels: np.ndarray | None = None    # uint8[E] or None
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_edges(self) -> int:
        return int(self.adj.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def _csr_call(fn, *args) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    po = ctypes.POINTER(ctypes.c_uint64)()
    pa = ctypes.POINTER(ctypes.c_uint32)()
    ne = ctypes.c_uint64(0)
    rc = fn(*args, threads(), ctypes.byref(po), ctypes.byref(pa), ctypes.byref(ne))
    if rc != 0:
        raise RuntimeError(f"synth generator failed with status {rc}")
    return po, pa, int(ne.value)


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True) -> Graph:
    lib = _load()
    po, pa, ne = _csr_call(lib.synth_rmat, scale, edge_factor, a, b, c, seed, int(permute))
    nv = 1 << scale
    off = _adopt(po, nv + 1, ctypes.c_uint64, np.uint64)
    adj = _adopt(pa, ne, ctypes.c_uint32, np.uint32)
    return Graph(off, adj, meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                                     a=a, b=b, c=c, seed=seed, permute=permute))


def chung_lu(n: int, draws: int, gamma: float, i0: float, seed: int = 1,
             permute: bool = True) -> Graph:
    lib = _load()
    po, pa, ne = _csr_call(lib.synth_chung_lu, n, draws, gamma, i0, seed, int(permute))
    off = _adopt(po, n + 1, ctypes.c_uint64, np.uint64)
    adj = _adopt(pa, ne, ctypes.c_uint32, np.uint32)
    return Graph(off, adj, meta=dict(kind="chung_lu", n=n, draws=draws, gamma=gamma, i0=i0,
                                     seed=seed, permute=permute))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def weights_uniform(g: Graph, lo: int, hi: int, seed: int) -> np.ndarray:
    out = np.empty(g.n_edges, dtype=np.uint32)
    rc = _load().synth_weights_uniform(_ptr(g.offsets), _ptr(g.adj), g.n_vertices, lo, hi,
                                       seed, threads(), _ptr(out))
    if rc:
        raise ValueError("bad uniform weight range")
    return out


def weights_zipf(g: Graph, s: float, cap: int, seed: int) -> np.ndarray:
    out = np.empty(g.n_edges, dtype=np.uint32)
    rc = _load().synth_weights_zipf(_ptr(g.offsets), _ptr(g.adj), g.n_vertices, s, cap, seed,
                                    threads(), _ptr(out))
    if rc:
        raise ValueError("bad zipf parameters")
    return out


def labels_uniform(g: Graph, k: int, seed: int) -> np.ndarray:
    out = np.empty(g.n_edges, dtype=np.uint8)
    rc = _load().synth_labels_uniform(_ptr(g.offsets), _ptr(g.adj), g.n_vertices, k, seed,
                                      threads(), _ptr(out))
    if rc:
        raise ValueError("bad label count")
    return out


def uniform_ids(n: int, nv: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    rc = _load().synth_uniform_ids(n, nv, seed, threads(), _ptr(out))
    if rc:
        raise ValueError("bad id range")
    return out


# ---------------------------------------------------------------------------
# Workload recipes.  Each names the graph, its attributes, the walk algorithm
# and the query set.  Node2vec factors are (f_ret, f_in, f_out) = L*(1/p, 1, 1/q)
# reduced to integers; they are given here as the p, q rationals.
# ---------------------------------------------------------------------------
RECIPES = {
    # node2vec p=2, q=1/2 on R-MAT scale 12: small enough for the oracle in full.
    "rmat12_n2v": dict(
        graph=dict(kind="rmat", scale=12, edge_factor=8, a=0.57, b=0.19, c=0.19, seed=12),
        weights=dict(kind="uniform", lo=1, hi=255, seed=1201),
        labels=None,
        walk=dict(algo="node2vec", p=(2, 1), q=(1, 2), length=20, seed=42,
                  starts="all"),
    ),
    # R-MAT scale 22, edge factor 16: the plain-batch-walker workload.
    "rmat22_n2v": dict(
        graph=dict(kind="rmat", scale=22, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=22),
        weights=dict(kind="zipf", s=1.2, cap=65535, seed=2201),
        labels=None,
        walk=dict(algo="node2vec", p=(1, 1), q=(2, 1), length=80, seed=42, starts="all"),
    ),
    "rmat22_deepwalk": dict(
        graph=dict(kind="rmat", scale=22, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=22),
        weights=dict(kind="zipf", s=1.2, cap=65535, seed=2201),
        labels=None,
        walk=dict(algo="deepwalk", length=80, seed=42, starts="all"),
    ),
    # PPR as in the experiments: |V| queries, all from the vertex of largest
    # degree, stop chance 1/5 per hop; 80 hops cap the (geometric) length.
    "rmat22_ppr": dict(
        graph=dict(kind="rmat", scale=22, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=22),
        weights=dict(kind="zipf", s=1.2, cap=65535, seed=2201),
        labels=None,
        walk=dict(algo="ppr", stop=(1, 5), length=80, seed=42, starts="max_degree"),
    ),
    # Chung-Lu gamma=2.1, 2^24 vertices, ~256M stored edges: MetaPath, unit weights.
    "chunglu24_metapath": dict(
        graph=dict(kind="chung_lu", n=1 << 24, draws=142_000_000, gamma=2.1, i0=4.0, seed=24),
        weights=None,
        labels=dict(kind="uniform", k=5, seed=2402),
        walk=dict(algo="metapath", schema=[0, 1, 2, 3, 4], length=20, seed=42,
                  starts="all"),
    ),
    # R-MAT scale 24 for the served request stream.
    "rmat24_serve": dict(
        graph=dict(kind="rmat", scale=24, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=2424),
        weights=dict(kind="uniform", lo=1, hi=255, seed=2421),
        labels=dict(kind="uniform", k=5, seed=2422),
        walk=None,
    ),
    # Chung-Lu gamma=2.0 shaped like a 227M-vertex / 2.71B-edge social graph.
    "chunglu227m_n2v": dict(
        graph=dict(kind="chung_lu", n=227_000_000, draws=1_620_000_000, gamma=2.0, i0=30.0,
                   seed=227),
        weights=dict(kind="uniform", lo=1, hi=1000, seed=22701),
        labels=None,
        walk=dict(algo="node2vec", p=(1, 2), q=(2, 1), length=80, seed=42,
                  starts=dict(kind="uniform", n=10_000_000, seed=22702)),
    ),
}


def make_graph(spec: dict) -> Graph:
    g = dict(spec)
    kind = g.pop("kind")
    if kind == "rmat":
        return rmat(**g)
    if kind == "chung_lu":
        return chung_lu(**g)
    raise ValueError(kind)


def _attach(g: Graph, recipe: dict) -> Graph:
    w = recipe.get("weights")
    if w is not None:
        if w["kind"] == "uniform":
            g.weights = weights_uniform(g, w["lo"], w["hi"], w["seed"])
        elif w["kind"] == "zipf":
            g.weights = weights_zipf(g, w["s"], w["cap"], w["seed"])
        else:
            raise ValueError(w["kind"])
    lab = recipe.get("labels")
    if lab is not None:
        g.labels = labels_uniform(g, lab["k"], lab["seed"])
    return g


def cache_dir() -> Path:
    return Path(os.environ.get("FW_GRAPH_CACHE", "/tmp/fw_graph_cache"))


def _key(recipe: dict) -> str:
    blob = json.dumps({"graph": recipe["graph"], "weights": recipe.get("weights"),
                       "labels": recipe.get("labels"), "v": 1}, sort_keys=True)
    return hashlib.sha1(blob.encode()).hexdigest()[:16]


def load_recipe_graph(name: str, use_cache: bool = True) -> Graph:
    """Generate (or read back from the on-disk cache) the graph of a recipe.
    FW_GRAPH_CACHE=off generates without reading or writing the cache."""
    recipe = RECIPES[name]
    if os.environ.get("FW_GRAPH_CACHE") == "off":
        use_cache = False
    d = cache_dir() / _key(recipe)
    parts = ["offsets", "adj", "weights", "labels"]
    if use_cache and (d / "meta.json").exists():
        meta = json.loads((d / "meta.json").read_text())
        arrs = {p: (np.load(d / f"{p}.npy", mmap_mode="r") if (d / f"{p}.npy").exists()
                    else None) for p in parts}
        return Graph(arrs["offsets"], arrs["adj"], arrs["weights"], arrs["labels"], meta)
    g = _attach(make_graph(recipe["graph"]), recipe)
    g.meta["recipe"] = name
    if use_cache:
        try:
            d.mkdir(parents=True, exist_ok=True)
            for p in parts:
                a = getattr(g, p)
                if a is not None:
                    np.save(d / f"{p}.npy", a)
            (d / "meta.json").write_text(json.dumps(g.meta))
        except OSError:
            pass
    return g


def recipe_starts(name: str, g: Graph) -> np.ndarray:
    st = RECIPES[name]["walk"]["starts"]
    if st == "all":
        return np.arange(g.n_vertices, dtype=np.uint32)
    if st == "max_degree":
        hub = int(np.argmax(g.degrees()))
        return np.full(g.n_vertices, hub, dtype=np.uint32)
    return uniform_ids(st["n"], g.n_vertices, st["seed"])


def degree_stats(g: Graph) -> dict:
    d = g.degrees().astype(np.float64)
    return dict(n_vertices=g.n_vertices, n_edges=g.n_edges, d_max=int(d.max()),
                d_mean=float(d.mean()), d2_over_d=float((d * d).sum() / max(d.sum(), 1)),
                zero_degree=int((d == 0).sum()))
