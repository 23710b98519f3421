"""CPU oracle of the vertex-reuse geometry stage.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the GPU
library and its Python binding never do.
"""
