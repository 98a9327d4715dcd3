"""FP64 CPU oracle of the forward Gaussian-splatting rasterizer.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its Python binding.
"""
