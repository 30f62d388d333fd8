"""Seeded synthetic input graphs (input generation only, no method arithmetic).

Both the CPU oracle (in tests) and the GPU path consume these edge lists.
Shapes follow the paper's workloads (Sec. 5.1, Tab. networks): Graph500
R-MAT graphs, heavy-tailed Chung-Lu graphs and a BTER-like community graph.
"""
from .gen import (build, rmat, chung_lu, bter, batch_shapes, chung_lu_c1, rmat_graph500)  # noqa: F401
