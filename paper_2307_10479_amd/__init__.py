"""MI355X (gfx950) search library for the Dynamic Exploration Graph.

The compute path is libdeg.so (hand-written HIP kernels behind the C ABI in
include/deg.h); `api` marshals torch tensors into it. Importing this package
does not touch the GPU; the first library call does, and it raises if the
library is not built or no GPU is visible.
"""
from . import api  # noqa: F401
from .api import (DeviceGraph, StopModel, VectorStore, knn_bruteforce, medoid,  # noqa: F401
                  search, search_batch, search_indexed)
