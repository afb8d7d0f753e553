"""Writes heron_counts.txt: the exact step counts of min-norm Newton on the unit sphere.

For F(q) = q.q - 1 the min-norm step is radial and the radius follows r <- (r + 1/r) / 2 (Heron's
rule), so the number of steps until |r^2 - 1| < tol, from r0, follows from the recurrence alone. It is
evaluated here in exact rationals (no floating point, no oracle, no GPU). The paper prints no worked
numeric example of a projection, so this closed form stands in for one.
"""
from fractions import Fraction
import os


def steps(r0: str, tol: str, per_iteration: int = 1) -> int:
    r, k, t = Fraction(r0), 0, Fraction(tol)
    while not (abs(r * r - 1) < t):
        for _ in range(per_iteration):
            r = (r + 1 / r) / 2
        k += 1
    return k


if __name__ == "__main__":
    rows = [(r0, steps(r0, "1e-6")) for r0 in ("0.9", "0.5", "0.1", "0.01", "3")]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "heron_counts.txt")
    with open(out, "w") as f:
        f.write("# Newton steps on ||q||^2 - 1 until | ||q||^2 - 1 | < 1e-6, from ||q0|| = r0 (Heron's rule)\n")
        f.write("# written by tests/golden/make_golden.py from the recurrence in exact rationals\n")
        for r0, k in rows:
            f.write(f"{r0} {k}\n")
