"""CPU oracle for the MASTER mode-coupling matrices (TEST INFRASTRUCTURE ONLY).

This package is the slow, obviously correct reference that the HIP path is
checked against.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import, call, link or execute anything in it; the
product path (``paper_2602_15605_amd``) never does, and the two share no
code, headers, tables or helpers.

What it computes (Sec. 2, eqs. K_TT and K_EE; App. A, eqs. for Xi_TT, Xi_TE,
Xi_EE, Xi_EB and the BB remark):

    K^X_{l1 l2} = (2 l2 + 1)/(4 pi) * sum_{l3} (2 l3 + 1) W^X_{l3} S^X(l1, l2, l3)

    S^TT = (l1 l2 l3; 0 0 0)^2
    S^TE = [(1 + (-1)^L)/2] (l1 l2 l3; 0 0 0)(l1 l2 l3; -2 2 0)
    S^EE = S^BB = [(1 + (-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2
    S^EB = [(1 - (-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2,          L = l1 + l2 + l3

with W^TT = W_TT, W^TE = W_TP and W^EE = W^BB = W^EB = W_PP.

Tiers
-----
* ``racah``   -- the Wigner 3j symbol from its definition (the Racah sum) in
  exact integer/rational arithmetic, and the exact K for small l.
* ``bulk``    -- a long-double C implementation for large l: every 3j row
  over l3 by the Schulten--Gordon three-term recursion (two-sided, normalised
  by the orthogonality sum, sign fixed at the stretched end), then the plain
  l3 sum of the definition above.  It shares nothing with the method under
  test (no g(p) tables, no closed-form reduction of the (-2 2 0) symbol).

Every function here is pinned by ``tests/test_oracle_*.py`` against values
fixed by mathematics (library 3j values, textbook closed forms, orthogonality
sums, the full-sky identity, brute force at small l).
"""
