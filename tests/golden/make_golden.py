"""Writes the stored expected values under tests/golden (calls only oracle/)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import scalars  # noqa: E402

HEADER = """# Exact effective conductivity of the periodic array of squares at 25% volume
# fraction, sigma2 = 1 (Obnosov's formula, eq. J47a of the paper:
# sigma* = sqrt((1 + 3 sigma1)/(3 + sigma1))); branch cut [-3, -1/3].
# Values written by tests/golden/make_golden.py (calls oracle.scalars only).
# sigma1_re sigma1_im sigma_star_re sigma_star_im
"""

POINTS = [10.0, 100.0, 1000.0, 0.01, 0.0, 3 + 2j, -0.1 + 0.5j, 1.0]


def main():
    with open(os.path.join(HERE, "obnosov_square_array.txt"), "w") as f:
        f.write(HEADER)
        for s in POINTS:
            v = complex(scalars.obnosov_square_array(s))
            f.write(f"{complex(s).real:.17g} {complex(s).imag:.17g} {v.real:.17g} {v.imag:.17g}\n")


if __name__ == "__main__":
    main()
