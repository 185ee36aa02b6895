"""MI355X (gfx950) dual-tree-traversal fast multipole method, 3-D Laplace kernel.

The library (libfmm.so: host C++ tree/traversal + HIP kernels) is loaded on
first use through paper_1209_3516_amd.fmm; importing the package itself does
not touch the GPU.
"""
