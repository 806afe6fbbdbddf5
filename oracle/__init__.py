"""Plain FP64 CPU oracle for the two-level Lippmann-Schwinger solver of
Zepeda-Nunez & Zhao, "Fast alternating bi-directional preconditioner for the
2D high-frequency Lippmann-Schwinger equation" (arXiv 1602.07652).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library and its Python binding never call it, and it shares no code
with them (only the seeded input generators in ``ls_inputs`` serve both).

Everything is complex128 / float64.  Each function cites the passage of the
paper it follows.  Readings of passages where the paper is silent or garbled
are stated where they are used.

Modules
-------
kernel    Green's function samples, modified trapezoidal weight, the
          operator H = I + w^2 G D (direct sum and zero-padded FFT), f.
sparsify  sparsifying stencils alpha/beta by SVD, A, C = A + w^2 B D.
slabs     layered decomposition, local matrices C^l with the smooth
          cut-off, Alg. 1 (Gauss-Seidel polarized traces), Alg. 2.
krylov    right-preconditioned GMRES and flexible GMRES.
solver    Alg. 3 (the Lippmann-Schwinger preconditioner) and the outer
          solve; dense reference solve.
disk      closed-form Bessel series for a homogeneous disk.
fno       the Fourier-neural-operator preconditioner / warm start: forward,
          analytic adjoint, relative loss, Adam.

Parity status: every function is pinned by a CPU test against something other
than itself (closed forms, brute force, invariants); see tests/test_oracle_*.py.
"""
from . import kernel, sparsify, slabs, krylov, solver, disk, fno  # noqa: F401
