"""Plain FP64 CPU oracle for the approximate FIO inverse.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the HIP
library and its Python binding never do.  The oracle shares no code with the
HIP path: the two meet only in the seeded input generators of ``fio_inputs``.

Every function follows the paper's definitions and algorithm steps in the
paper's order, in plain numpy/scipy complex128, with no blocking, fusion or
reordering beyond the definitions:

  dd.py           double-double arithmetic (Knuth, Dekker) for phases modulo 1
  fio.py          grids, phase, kernel and dense K            (Section 1, eq. fio / fio_mat)
  cheb.py         Chebyshev grids and Lagrange bases          (Section 2.2)
  bf.py           explicit butterfly factors and their apply  (Section 2.2, eq. bf, bf_mid, bf_recursive)
  householder.py  textbook Householder QR / QRCP              (used by Section 3)
  hss.py          black-box HSS construction + postprocessing (Section 3, Def. hss_matrix)
  ulv.py          ULV factorization and solve                 (Section 2.4)
  solve.py        approximate inverse, refinement, PCG        (Section 4.1)

Parity status of each function is stated in its docstring; all functions are
pinned by the ``-m "not gpu"`` tests against closed forms, brute force or
invariants that do not reuse the function's own formulas.
"""
