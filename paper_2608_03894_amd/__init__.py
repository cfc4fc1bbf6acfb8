"""MI355X-native (gfx950) DQMC hot path for the attractive Hubbard model on the
kagome lattice: FFT propagator wrap and delayed Ising-field updates behind the
C ABI of include/kdqmc.h.  ``kdqmc`` is the ctypes binding."""
