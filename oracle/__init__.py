"""FP64 CPU oracle for the randomized range finder, RSVD, ID and CUR.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import anything from this package.  The HIP library never links, loads or calls
it, and this package never imports the HIP library: the two share no code.

Every function follows the paper (Voronin & Martinsson, "RSVDPACK",
arXiv:1502.05366) and cites the section, equation or algorithm it writes out.
Precision is FP64 throughout.  Library primitives used as single steps are
numpy's matrix product and sort; every factorization (Householder QR,
one-sided Jacobi SVD, column-pivoted QR, triangular solves) is written out
here.

Modules
-------
philox   Philox4x32-10 block function and Box-Muller normals (the sketch).
dense    Householder QR, one-sided Jacobi SVD, k-step CPQR, triangular solves.
rsvd     Range finder with power scheme (Alg. 5, s=1), RSVD, QB-based ID,
         two-sided ID and CUR; plus the Fig. 1 and Alg. 4 variants used as
         cross-checks.
"""

from . import philox, dense, rsvd  # noqa: F401
