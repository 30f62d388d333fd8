"""MI355X-native wedge sampling for triangle statistics.

Kolda, Pinar, Plantenga, Seshadhri, Task, "Counting Triangles in Massive
Graphs with MapReduce" (arXiv 1301.5887): degrees and wedges per vertex,
exponential degree bins, uniform wedge samples per bin, exact closure tests,
per-bin and global clustering coefficients and triangle estimates.

The compute path is libwedge.so (HIP for gfx950, C ABI in include/wedge.h);
``paper_1301_5887_amd.wedge`` is its thin Python binding.
"""
__all__ = ["wedge"]
