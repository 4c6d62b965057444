"""FP64 CPU oracle for SMP-PCA (Wu, Bhojanapalli, Sanghavi, Dimakis, "Single Pass
PCA of Matrix Products", arXiv 1610.06656).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
numpy/scipy reference of what the GPU path computes. Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code, constants tables or helpers with the HIP path
(``paper_1610_06656_amd``), and it never imports that package.

Module map (each function cites the passage of the paper it follows):

* ``philox``    counter-based generator (Philox4x32-10, Salmon et al., SC'11)
* ``gaussian``  Box-Muller transform of two 24-bit uniforms
* ``sketch``    Alg. 1 step 2 / Section 2 "Step 1": Pi, sketches, column norms
* ``srht``      the subsampled randomized Hadamard transform as Pi (Section 4, Spark)
* ``sparse``    the sketch of matrices given as entries in any order (Section 1; Section 3 complexity)
* ``sample``    Eq. (1) and Alg. 1 step 3: q, q-hat, Omega, weights
* ``multinomial`` Appendix D "Sampling": row-wise multinomial draws of Omega
* ``estimate``  Eq. (2): rescaled-JL estimates on Omega
* ``waltmin``   Appendix A, Alg. 2: WAltMin init, trim, alternating solves
* ``evaluate``  Section 4 "spectral norm error" and the best rank-r error
* ``solve``     Alg. 1 end to end
* ``baselines`` the comparison methods of Section 4: SVD(A~^T B~) and LELA

Parity status: every function is pinned by a ``-m "not gpu"`` test except
those marked "parity unpinned" in their docstring.
"""

from . import philox, gaussian, sketch, sample, multinomial, estimate, waltmin, evaluate, solve, baselines, srht, sparse  # noqa: F401
