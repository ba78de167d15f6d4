"""Write paper_weight.txt: the weight function the paper prints in Section 3,
Phi(r) = (1 - r^((1 - r)^2))^4 for r < 1, evaluated at a few r in 50-digit
decimal arithmetic (power by exp and ln of the decimal module), so that the
stored values owe nothing to floating-point code under test.

Run from the repository root: python tests/golden/make_paper_weight.py
"""
import os
from decimal import Decimal, getcontext

getcontext().prec = 50
R_VALUES = ["0", "0.1", "0.25", "0.4", "0.5", "0.57", "0.75", "0.9", "0.99"]


def paper_weight(r):
    r = Decimal(r)
    if r == 0:
        return Decimal(1)          # 0^(1) = 0, so Phi(0) = 1
    e = (1 - r) ** 2
    power = (e * r.ln()).exp()     # r^e
    return (1 - power) ** 4


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "paper_weight.txt"), "w") as f:
        f.write("# Weight printed in Section 3 of the paper, Phi(r) = (1 - r^((1-r)^2))^4, r < 1.\n")
        f.write("# Written by tests/golden/make_paper_weight.py in 50-digit decimal arithmetic.\n")
        f.write("# r  Phi(r)\n")
        for r in R_VALUES:
            f.write("%s %s\n" % (r, format(paper_weight(r), ".20e")))


if __name__ == "__main__":
    main()
