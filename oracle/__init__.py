"""CPU oracle for the F12 two-electron integral classes I1-I6 with the
range-separated correlation factor (Silkowski, Lesiuk, Moszynski,
arXiv:1412.5070).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The library in ``paper_1412_5070_amd`` never calls it, and it never calls the
library: the two share no code, tables or constants.

What it computes (plain definitions, each step citing the paper):
  * the integrals I_i = (ab|k_i(r12)|cd) over unnormalised primitive
    Cartesian Gaussians, contracted with the given coefficients (Sec. II.A,
    Eqs. (I1)-(I6), (basis));
  * via the Hermite (McMurchie-Davidson) expansion of each orbital product
    (Sec. II.B, Eq. (AB)) with the textbook three-term recursion for E;
  * the Hermite integrals R_tuv = d^t/dQx d^u/dQy d^v/dQz B_i (Eq. (ri))
    from the radial derivatives A_n = (R^-1 d/dR)^n B_i by the standard MD
    recurrence for a radial function;
  * the radial derivatives by direct quadrature of the universal one-
    dimensional representation of B_i (Sec. II.C, Eq. (bfinal)) with the
    kernel k_i evaluated pointwise from Eq. (rs12) and Eq. (ttdamp);
  * I5 by Green's identity, Eq. (I5_): I5 = 1/2 [I3(lap a, b) - I3(a, lap b)].

Precision: double-double (about 32 digits, ``oracle.dd``) for every step
from the quadrature to the contracted sum; inputs are binary64 and the
output is rounded to binary64.  Binary64 is not enough for this oracle:
D^n applied to the Gaussian-convolution in Eq. (bfinal) cancels like
(2 xi R^2)^(n/2) (demonstrated in tests/test_oracle_pins.py).

Parity unpinned: individual regularised S(alpha, beta, gamma) at negative
integer alpha (only sums inside a kernel are unique).  Every other function
here is pinned by a test against closed forms, library routines or
identities (see tests/test_oracle_pins.py).
"""
