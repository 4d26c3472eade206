"""MI355X-native 1D2V continuum-kinetic flashover step (arXiv 2303.14119).

Submodules:
  flashkin   ctypes binding of the HIP library (loads ``libflashkin.so`` and
             raises if it has not been built)
  workloads  seeded synthetic parameter sets and initial states
"""
