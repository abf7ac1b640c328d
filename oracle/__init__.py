"""Plain FP64 CPU oracle for FFT-based homogenization of orders 0 and 1.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never imports, links or calls it, and it shares no code with the GPU
path: it has its own FFT (``fftref``), its own tensor algebra and its own
solvers, written directly from the paper (Dietrich, Merkert, Simeon,
"Derivation of higher-order terms in FFT-based numerical homogenization",
arXiv:1712.05145).

Modules
-------
fftref         own mixed-radix DFT/FFT (Sec. 2: the Fourier series of eq. (5))
tensors        Hooke's law (eq. (2)), reference medium C0 (Sec. 2), Voigt I/O
spectral       Green operator (formula below eq. (5)), theta (eq. (12)),
               displacement recovery (inverse of eq. (1)), spectral sym-gradient
solvers        Basic Scheme (fixed point of eq. (5)), CG on eq. (6)
               (Algorithm 1 and the Cauchy criterion after it), dense
               displacement Galerkin solve (the definition of the discrete
               solution, small grids only)
homogenization order-0 and order-1 problems (Sec. 3, Definition 1), effective
               stiffness, Voigt/Reuss/Hashin-Shtrikman bounds

Every numerical convention the paper leaves open (Nyquist modes, DFT sign,
CG inner product, unit loads, zero-RHS guard) is fixed, with its reading of
the paper, in the ``spectral`` and ``solvers`` docstrings.

Parity unpinned: the order-1 right-hand side on genuinely 3-D
microstructures is pinned only through identities (divergence of theta,
compatibility of recovered displacements, mean of g equal to C_eff
contracted with the gradient) and the laminate reduction; the pointwise
formulas of p_2 and g_2 themselves are checked by hand-computed single-voxel
cases only.
"""
