"""MI355X-native orthogonal voxel finite element (OVFEM) elastic-wave stepper.

The compute path is the C-ABI library ``libovfem.so`` (HIP kernels for gfx950);
``paper_2404_13683_amd.ovfem`` is a thin ctypes binding over it.  The seeded input
generators live in ``paper_2404_13683_amd.workloads``.
"""
__all__ = ["ovfem", "workloads"]
