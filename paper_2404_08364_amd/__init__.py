"""MI355X (gfx950) dynamic-graph random walks: DeepWalk, node2vec and
MetaPath hops sampled on the fly over a CSR graph in HBM, bit-exact and
bufferless.

The native library is ``libflowwalk.so`` (HIP); :mod:`.flowwalk` is its
ctypes binding and is imported on first use, so that building does not need
the library to exist yet.
"""
import importlib

__all__ = ["flowwalk"]


def __getattr__(name):
    if name == "flowwalk":
        return importlib.import_module(".flowwalk", __name__)
    raise AttributeError(name)
