"""MI355X (gfx950) batched HMM micro-problem solver for the Landau-Lifshitz
equation (Leitenmaier & Runborg).

Modules:
  inputs   seeded synthetic workloads (shared with the test oracle)
  llhmm    ctypes binding of libllhmm.so (include/llhmm.h)
  runner   workload -> device buffers -> solve
  build    hipcc build of libllhmm.so
"""
