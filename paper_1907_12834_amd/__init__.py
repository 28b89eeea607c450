"""MI355X-native spin-2 quantum-lattice-gas step (HIP kernels behind a C ABI).

Submodules: ``qlg`` (ctypes binding of libqlg.so), ``build`` (hipcc build),
``autograd`` (adjoint as a torch.autograd.Function).  Nothing is imported
eagerly, so the build module works before the library exists.
"""
