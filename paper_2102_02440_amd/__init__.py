"""MI355X-native hot path of online sketch-based query optimisation.

The fused selection scan + Fast-AGMS sketch build and the sketch-merging
join-size estimates run as hand-written HIP kernels behind a C ABI
(``libcompass.so``); ``paper_2102_02440_amd.compass`` is the Python binding.
"""
__version__ = "0.1.0"
