"""FP64 CPU oracle of the dual-tree-traversal Laplace FMM.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library.  The product package never
imports it.
"""
