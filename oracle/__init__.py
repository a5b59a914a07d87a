"""CPU FP64 oracle for coil-sketched PICS reconstruction (test infrastructure).

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  It is TEST INFRASTRUCTURE: only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library and its Python binding) never
calls into it and shares no code with it.

Everything is NumPy/SciPy in float64 / complex128.  Each function cites the
passage of the paper (Oscanoa et al., "Coil Sketching for
computationally-efficient MR iterative reconstruction") it follows:

  * ``cartesian``  -- A = U F C for Cartesian sampling (Sec. 2.1, Eq. 2).
  * ``nufft``      -- A = W^1/2 F_n C with a Kaiser-Bessel gridding NUFFT
                      (Sec. 2.1, Eqs. 1-2, 5), plus the brute-force NDFT of
                      Eq. 1 used to pin it.
  * ``sketch``     -- PCA virtual coils and the structured sketch
                      S^t = S~^t (x) I_N with S~^t = blkdiag(I_V, S~_S^t)
                      (Sec. 2.3.2-2.3.3, Eqs. 11-13).
  * ``wavelet``    -- unitary periodized Daubechies-4 transform and the
                      l1-wavelet proximal step (Sec. 2.1, regularizer 2).
  * ``recon``      -- FISTA on the full problem (Eqs. 3-4) and Algorithm 1
                      (coil sketching, Eqs. 9-10) with FISTA inner solves.

Readings of passages the paper leaves open are listed in each module header.
"""
