"""CPU FP64 oracle for the Polar Express iteration (Amsel, Persson, Musco, Gower,
"The Polar Express: Optimal Matrix Sign Methods and Their Application to the
Muon Algorithm", arXiv 2505.16932).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product library
(``paper_2505_16932_amd`` and its HIP/C++ sources) never imports, links or calls
anything here, and nothing here imports the product: the two share no code.

Contents (each function cites the passage of the paper it follows):

* ``schedule``  -- the offline stage: degree-5 odd minimax polynomials by the
  simplified Remez exchange (Appendix E, Algorithm 3), composed greedily
  (Theorem 1), with the finite-precision modifications (Section 3.4, Appendix F).
* ``iteration`` -- the online stage in FP64: normalise, then
  X <- a X + (b A + c A^2) X with A = X X^T on the smaller side (Section 3.5).
* ``jacobi``    -- the exact polar factor U V^T from a one-sided (Hestenes)
  Jacobi SVD, the target of eq. (matrixsign).
* ``spectral``  -- spectral norms and the Appendix C identity relating the
  matrix error to the scalar composite on the spectrum.
* ``lowprec``   -- round-to-nearest-even bfloat16 / OCP e4m3 quantisers used to
  state what the low-precision paths compute.
* ``fastapply`` -- Algorithm 4 (Appendix G): the composite as Q X with Q a
  polynomial in the Gram matrix, restarted every k steps, first-segment shift.
* ``muon``      -- one Muon optimizer step (Section 1.1) around the iteration.
* ``spectral_init`` -- the spectrum-aware initialisation step for a large
  outlying singular value (appendix on large spectral gaps, k = 1).
* ``mlp``       -- FP64 forward/backward/update of the small l-predictor MLP
  and its spectrum-level labels.

Every function here is pinned by ``tests/test_oracle_*.py`` against values the
paper prints, closed forms, invariants, library routines or brute force.
"""
