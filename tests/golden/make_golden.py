"""Writes the stored colour-matrix fixtures from the oracle (run from the repo root).

The paper prints no numeric amplitude, colour-matrix or timing values (its
results are figures), so every stored value here is produced by this script
calling only ``oracle``.  Output: colour_matrix_n{4,5,6}.txt (full matrices)
and colour_matrix_n{7,8}_row0.txt (first rows; the rest follows by relabelling).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.color import color_entry, color_matrix, middle_permutations  # noqa: E402


def main():
    for n in (4, 5, 6):
        np.savetxt(os.path.join(HERE, f"colour_matrix_n{n}.txt"), color_matrix(n), fmt="%d",
                   header=f"C(n={n}) exact, N=3, Tr(T^a T^b)=delta^ab, lexicographic sigma")
    np.savetxt(os.path.join(HERE, "colour_matrix_n7_row0.txt"), color_matrix(7)[:1], fmt="%d",
               header="C(n=7) first row (sigma = identity)")
    perms = middle_permutations(8)
    row8 = np.array([[color_entry(8, perms[0], p) for p in perms]], dtype=np.int64)
    np.savetxt(os.path.join(HERE, "colour_matrix_n8_row0.txt"), row8, fmt="%d",
               header="C(n=8) first row (sigma = identity)")


if __name__ == "__main__":
    main()
