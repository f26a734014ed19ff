"""MI355X-native semi-Lagrangian lattice Boltzmann hot path.

``paper_1910_13918_amd.sllbm`` is the ctypes binding of the C-ABI library
``libsllbm.so`` (HIP kernels for gfx950); ``paper_1910_13918_amd.solver`` wraps
it with torch-owned device buffers; ``paper_1910_13918_amd.workloads`` holds the
seeded synthetic problems.  Nothing is imported eagerly, so importing the
package never loads the GPU library.
"""
