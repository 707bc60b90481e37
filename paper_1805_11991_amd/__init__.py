"""hwcount: Hasse-Weil point counts of hyperelliptic curves over small finite
fields on MI355X (gfx950), after M. Raum, "Hyperelliptic Curves over Small
Finite Fields and GPU Accelerators" (arXiv:1805.11991).

The counting runs in hand-written HIP kernels behind the C ABI declared in
``include/hwcount.h`` (``libhwcount.so``); ``paper_1805_11991_amd.hwcount``
is the Python binding with the same names.
"""
