"""Writes oracle/leja_points.txt: the first 501 Leja points on [-2, 2] as
exact hexadecimal doubles, produced by oracle.leja.generate_leja_points
(greedy max-product sequence; xi_0 = 2, ties to the smaller point)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle.leja import TABLE_FILE, generate_leja_points, MAX_DEGREE  # noqa: E402


def main(M: int = MAX_DEGREE + 1):
    pts = generate_leja_points(M)
    with open(TABLE_FILE, "w") as fh:
        fh.write("# Leja points on [-2, 2], greedy max-product order, xi_0 = 2,\n")
        fh.write("# ties to the smaller point; hex double, then decimal\n")
        for x in pts:
            fh.write("%s %.17g\n" % (float(x).hex(), x))


if __name__ == "__main__":
    main()
