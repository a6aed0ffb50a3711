"""Writes closed_forms.json: spectra the thesis states in closed form.

Sources (App. D, "Test Matrices"):
* 1-2-1: diagonal 2, off-diagonals 1, lambda_k = 2 - 2 cos(pi k / (n + 1)).
* Clement: zero diagonal, beta_k = sqrt(k (n - k)); integer eigenvalues
  +-(n-1), +-(n-3), ... (the printed "+-n, +-n-2" is read as +-(n-1), ...,
  consistent with the stated smallest magnitude 1 for even n, 0 for odd n).

Only the formulas are evaluated here; nothing calls the oracle or the GPU
library.  Run:  python tests/golden/make_golden.py
"""
import json
import math
import os

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")


def main():
    cases = []
    for n in (1, 2, 3, 4, 5, 8, 13):
        cases.append({
            "family": "121", "n": n, "d": 2.0, "e": 1.0,
            "eigenvalues": [2.0 - 2.0 * math.cos(math.pi * k / (n + 1)) for k in range(1, n + 1)],
            "cite": "App. D, 1-2-1 matrix: lambda_k = 2 - 2 cos(pi k/(n+1))",
        })
        cases.append({
            "family": "clement", "n": n,
            "eigenvalues": [float(-(n - 1) + 2 * (j - 1)) for j in range(1, n + 1)],
            "cite": "App. D, Clement matrix: integer spectrum +-(n-1), +-(n-3), ...",
        })
    with open(OUT, "w") as f:
        json.dump({"cases": cases}, f, indent=1)


if __name__ == "__main__":
    main()
