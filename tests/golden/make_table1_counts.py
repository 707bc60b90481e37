"""Writes table1_counts.txt: N_1 and N_2 of Table 1's curve over F_p and
F_{p^2} for the primes of Table 1, computed by the oracle only.

    python tests/golden/make_table1_counts.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CURVE = [17, 12, 16, 11, 10, 13, 12]      # 12X^6 + 13X^5 + 10X^4 + 11X^3 + 16X^2 + 12X + 17, constant first
PRIMES = [101, 211, 307, 401, 503, 1009, 1511, 2003, 3001]

if __name__ == "__main__":
    lines = ["# Table 1 (Sec. 4): Y^2 = 12X^6 + 13X^5 + 10X^4 + 11X^3 + 16X^2 + 12X + 17 over F_p and F_{p^2}",
             "# p N_1 N_2   (oracle point counts; the paper prints runtimes only)"]
    for p in PRIMES:
        row = np.array([[c % p for c in CURVE]], dtype=np.int16)
        N = oracle.count_curves(p, 2, row, kmax=2)[0]
        lines.append(f"{p} {int(N[0])} {int(N[1])}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "table1_counts.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
