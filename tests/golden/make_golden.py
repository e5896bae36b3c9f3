"""Write the stored reference numbers under tests/golden/ from the CPU oracle.

Calls only ``oracle/`` and the input generators.  Run from the repository
root: ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lshom_oracle as o  # noqa: E402
from paper_1004_1122_amd import microstructure as ms  # noqa: E402


def main():
    m = ms.square_inclusion()
    lam = m.lam()
    out = {"workload": "63x63 square inclusion, lambda 10 in 1, l0 5.5, E=(1,0)",
           "source": "oracle/lshom_oracle.py (CPU FP64), no GPU value"}
    res = o.cg(lam, 5.5, [1.0, 0.0], tol=1e-8)
    out["iterations_tol1e-8"] = res["iterations"]
    out["leff11_tol1e-8"] = float(o.leff(lam, res["e"])[0])
    L, iters = o.homogenize(lam, 5.5, tol=1e-12)
    out["leff_tensor_tol1e-12"] = L.tolist()
    out["iterations_tol1e-12"] = iters
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "square63.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
