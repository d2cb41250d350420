"""MGRIT for the 2-D Riesz space-fractional diffusion equation on MI355X (gfx950).

The solver is the HIP library libmgrit.so behind the C ABI in include/mgrit.h;
`paper_1805_06688_amd.mgrit` is its ctypes binding and
`paper_1805_06688_amd.workloads` holds the seeded synthetic input generators.
Importing the package itself loads nothing.
"""
