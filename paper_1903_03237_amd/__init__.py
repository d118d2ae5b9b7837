"""FastMNMF on AMD MI355X (gfx950): HIP kernels behind a C-ABI library.

Submodules (imported explicitly, nothing is loaded at package import):
  fmnmf   ctypes binding of libfmnmf.so (the C-ABI declared in include/fmnmf.h)
  synth   seeded synthetic mixtures and initial states
  serve   continuous-batching request loop on top of fmnmf_step_batch
"""
