"""Writes exact_gap_k0.txt: the lowest zero-momentum levels of the spin chain
(eq. 3, J = 1) at h_perp = 1, h_par = 0.1 for N = 16, 20, 24, computed by the
oracle's sparse Lanczos exact diagonalisation (oracle/lanczos.py) and nothing
else.  These are the exact references of the gap metric: the truncated basis
dimension at which |Delta_TGBA - Delta_exact| <= 1e-6, Delta = E_{0,2} - E_{0,1}.

    python tests/golden/make_exact_gaps.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lanczos  # noqa: E402


def main():
    rows = []
    for N in (16, 20, 24):
        e = lanczos.k0_lowest(N, 1.0, 0.1, k=4)
        rows.append("%d 1.0 0.1 %.15f %.15f %.15f %.15f %.15f" % (N, e[0], e[1], e[2], e[3], e[1] - e[0]))
        print(rows[-1], flush=True)
    with open(os.path.join(HERE, "exact_gap_k0.txt"), "w") as f:
        f.write("# Exact lowest K = 0 levels of eq. 3 (J = 1), sparse Lanczos ED of the oracle\n")
        f.write("# (tests/golden/make_exact_gaps.py).  columns: N h_perp h_par E1 E2 E3 E4 gap=E2-E1\n")
        f.write("\n".join(rows) + "\n")


if __name__ == "__main__":
    main()
