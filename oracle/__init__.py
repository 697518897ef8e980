"""Plain FP64 CPU oracle for the orthogonal voxel finite element (OVFEM) stepper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library, its
Python binding) may import, call, link or execute anything in this package.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code, table or helper with the HIP implementation; the
two meet only through the seeded inputs of ``paper_2404_13683_amd.workloads``.

Contents
--------
element     exact (rational) element matrices of the OVFEM voxel element
            (Sec. 2, Eqs. (4)-(8)) and of the conventional trilinear voxel
            element (Sec. 2, VFEM paragraph), element mass.
assembly    structured-grid element-by-element matvec, lumped/orthogonal mass,
            central-difference stepper (Sec. 2, Eq. (3)), receivers, energy,
            discrete adjoint and gradients, the error measure of Sec. 3 Eq. (18).
dispersion  Bloch (plane-wave) analysis of the assembled operators.

Precision: every floating-point step is FP64 (numpy float64); the reference
matrices themselves are built in exact rational arithmetic and converted once.
"""
