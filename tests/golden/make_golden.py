"""Writes the golden fixtures of this folder from the exact oracle tier only.

    python tests/golden/make_golden.py

threej_small_exact.txt : (l1 l2 l3; 0 0 0) and (l1 l2 l3; -2 2 0) for
    0 <= l1, l2 <= 8, every l3 of the triangle, as "sign num/den" of the exact
    square (Racah sum, E57 eq. 3.7.3).
coupling_small_exact.txt : K^X for lmax = 6 and X in TT, TE, EE, BB, EB for the
    fixed window W_l = 1/(l+1) (l = 0..12) on all three spectra, each element
    rounded once to float64 (Sec. 2 eqs. K_TT, K_EE; App. A).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import racah  # noqa: E402


def main():
    with open(os.path.join(HERE, "threej_small_exact.txt"), "w") as f:
        f.write("# l1 l2 l3 m sign square   (symbol (l1 l2 l3; m -m 0), exact Racah sum)\n")
        for l1 in range(9):
            for l2 in range(9):
                for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                    for m in (0, -2):
                        sg, sq = racah.threej_sq_sign(l1, l2, l3, m, -m, 0)
                        f.write("%d %d %d %d %d %d/%d\n" % (l1, l2, l3, m, sg, sq.numerator, sq.denominator))
    lmax = 6
    W = [1.0 / (l + 1) for l in range(2 * lmax + 1)]
    with open(os.path.join(HERE, "coupling_small_exact.txt"), "w") as f:
        f.write("# spectrum l1 l2 K   (W_l = 1/(l+1), lmax = 6, exact sums rounded once)\n")
        for spec in racah.SPECTRA:
            K = racah.coupling_exact(lmax, W, spec)
            for l1 in range(lmax + 1):
                for l2 in range(lmax + 1):
                    f.write("%s %d %d %.17g\n" % (spec, l1, l2, K[l1][l2]))


if __name__ == "__main__":
    main()
