"""juqcs_gpu: MI355X-native state-vector gate engine (hot path of the Juelich
universal quantum computer simulator, arXiv:1912.03243).

Submodules
  workloads  seeded synthetic circuits and bitstrings (input generation only)
  juqcs      ctypes binding of the C-ABI library libjuqcs_gpu.so (loaded on
             first import of that module; it fails loudly if the library is
             missing)
"""
