"""Writes the closed-form energy fixtures used by tests/test_oracle_pins.py.

These values come from the bare pair potential U = l_B q_i q_j / r of the
paper's Sec. 5.1 (the Poisson-Boltzmann pair potential with kappa -> 0),
evaluated by hand-derived closed forms with Python's math module -- not by
the oracle and not by the GPU library.
"""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    with open(os.path.join(HERE, "two_ion_energy.txt"), "w") as f:
        f.write("# Two ions at (0,0,0) and (3,4,0): r = 5 exactly.\n")
        f.write("# E = l_B q1 q2 / r  (bare pair potential, paper Sec. 5.1, kappa -> 0)\n")
        for lB, q1, q2 in [(0.7, 1.0, -1.0), (7.117, 3.0, -1.0), (2.0, 2.0, 2.0)]:
            f.write("E(lB=%g,q1=%g,q2=%g) = %.17g\n" % (lB, q1, q2, lB * q1 * q2 / 5.0))
    a, lB = 1.25, 0.7
    e = lB / a * (-12.0 + 12.0 / math.sqrt(2.0) - 4.0 / math.sqrt(3.0))
    with open(os.path.join(HERE, "rocksalt_cube.txt"), "w") as f:
        f.write("# Eight charges +-1 alternating on the corners of a cube of edge a.\n")
        f.write("# 12 unlike pairs at a, 12 like pairs at a*sqrt(2), 4 unlike pairs at a*sqrt(3):\n")
        f.write("# E = (l_B/a) (-12 + 12/sqrt(2) - 4/sqrt(3))  (bare pair potential, paper Sec. 5.1)\n")
        f.write("a = %.17g\nlB = %.17g\nE = %.17g\n" % (a, lB, e))


if __name__ == "__main__":
    main()
