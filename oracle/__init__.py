"""CPU FP64 oracle for the spectral projector of a symmetric banded matrix -- TEST INFRASTRUCTURE.

Nothing in the product path may import this package: only ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` use it.  It shares no code,
headers, tables or helpers with the HIP implementation in ``paper_1608_01164_amd``; the only
thing both sides consume is the seeded input generator in ``workloads``.

Modules
  eig        -- Sylvester-inertia counts, bisection, inverse iteration, Pi = V V^T (C core in eig_band.c)
  qdwh       -- the scalar QDWH weight schedule (a_k, b_k, c_k, l_k) and the exact-arithmetic map
  givens_qr  -- dense reference for the fast Givens QR of [A; I] (Algorithms 1 and 2)
  hodlr      -- reader and plain matvec for a HODLR matrix exported by the library
  norms      -- Lanczos estimate of the 2-norm of a symmetric operator, Frobenius helpers

Parity status of every function is listed in its docstring ("pinned by ...").
"""
