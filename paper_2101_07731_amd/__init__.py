"""MI355X-native multivariate DTW nearest-neighbour search with lower-bound
filtering (TC-DTW, arXiv 2101.07731).

The compute lives in libtcdtw.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/tc_dtw.h); this package only marshals arguments.
Submodules load the library on first use and raise if it is missing.
"""

__all__ = ["pairs", "synth"]
