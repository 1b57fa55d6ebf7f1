"""Write adjoint_24.txt: J and dJ/d(A, B, alpha, k) of the reduced adjoint
workload (24^3, bead spacing 7, one 2000-step period) from the FP64 gradient
oracle (checkpoints every 100 steps).  Calls only oracle/ and the workload
definitions.  Run from the repository root:

    python tests/golden/make_adjoint_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint  # noqa: E402
from paper_2202_12147_amd import workloads  # noqa: E402


def main():
    case = workloads.adjoint_case(reduced=True)
    J, g = adjoint.displacement_gradient(case, case["steps"], case["checkpoint"])
    with open(os.path.join(HERE, "adjoint_24.txt"), "w") as f:
        f.write("# FP64 gradient oracle (oracle/adjoint.py), workloads.adjoint_case(reduced=True):\n")
        f.write(f"# 24^3, tau 1, Guo, 3-point kernel, spacing 7, A = B = 1e-3, alpha = pi/3, T = 2000,"
                f" {case['steps']} steps, checkpoint {case['checkpoint']}\n")
        f.write("# J dJ/dA dJ/dB dJ/dalpha dJ/dk\n")
        f.write(" ".join(f"{v:.17e}" for v in [J, *g]) + "\n")


if __name__ == "__main__":
    main()
