"""POLFED hot path on AMD MI355X (gfx950): Python binding of libpolfed.

The compute lives in ``csrc/`` (HIP kernels + a C-ABI host library).  This
package only marshals arguments to it: ``paper_2005_09534_amd.polfed`` loads
``libpolfed.so`` through ctypes and fails loudly when it is missing.
``paper_2005_09534_amd.workloads`` draws the seeded synthetic spin chains.
Import the submodule you need; importing the package loads nothing.
"""
