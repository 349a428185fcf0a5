"""Ensemble adaptive explicit/implicit tau-leaping on MI355X (gfx950).

``paper_1608_07058_amd.lx`` is the binding to the C-ABI library ``liblx.so``
(hand-written HIP kernels); ``paper_1608_07058_amd.workloads`` generates seeded
synthetic inputs.  Importing the package itself loads nothing.
"""
