"""libchaosvid: the real-time chaotic video cipher of arXiv 2302.07411
(Jiang, Yuan, Li, Lu) on AMD Instinct MI355X (gfx950).

- ``csrc/``      HIP kernels and the C-ABI host runtime (include/chaosvid.h)
- ``binding``    thin ctypes binding over libchaosvid.so
- ``inputs``     seeded synthetic frames, keys and confusion seeds
- ``build``      in-tree hipcc build of libchaosvid.so
"""
