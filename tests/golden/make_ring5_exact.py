"""Writes ring5_exact.json: exact ln Z, E, C and M of the five-site s=5/2 ring
(the anisotropic ring of Sec. 3.2 with n = 5, dim 7776) at B = 0.1 T and 1 T
along z, on a 60-point log grid 0.1..100 K, by full diagonalisation with the
dense Kronecker-product oracle (oracle/dense.py) only.

Run from the repository root: python tests/golden/make_ring5_exact.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import ftlm_workloads as W  # noqa: E402
from oracle import dense  # noqa: E402


def main():
    T = W.t_grid(60)
    out = {"system": "ring_sftlm(5, B): n=5, s=5/2, J=0.02 K, d=-20 K, dipolar, g=2",
           "T": T.tolist(), "fields_T": [0.1, 1.0], "curves": []}
    for B in (0.1, 1.0):
        sysm, _ = W.ring_sftlm(5, B)
        ex = dense.exact_thermo(sysm, T)
        out["curves"].append({k: ex[k].tolist() for k in ("lnZ", "E", "C", "M")})
        print("B", B, "E0", ex["E0"], flush=True)
    with open(os.path.join(HERE, "ring5_exact.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
