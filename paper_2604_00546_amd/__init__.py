"""MI355X (gfx950) implementation of encrypted face-template search:
RNS-CKKS baby-step giant-step diagonal matrix-vector product against a
plaintext template database, followed by the homomorphic Chebyshev threshold
(arXiv 2604.00546).

Submodules:
  fr     -- binding of the C ABI in include/fr.h (libfrhip.so)
  synth  -- seeded synthetic workloads
  build  -- hipcc build of libfrhip.so
The binding is imported lazily so that CPU-only tooling can import `synth`.
"""
