"""Extended RaBitQ on MI355X (gfx950): the data-parallel hot path of
arXiv 2409.09913 behind a C-ABI library (``liberq.so``).

``paper_2409_09913_amd.erq`` is the thin ctypes binding (argument marshalling
only); ``paper_2409_09913_amd.synth`` holds the seeded input generators.
Importing the package does not load the library; the binding loads it on first
use and raises if it is missing.
"""
__all__ = ["erq", "synth"]
