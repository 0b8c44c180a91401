"""Writes tests/golden/oracle_24cube.json: the oracle's FP64 exchange energy,
pair energies and exchange-matrix diagonal of the 24^3 smoke workload (4
orbitals, r = 16, K = 30).  Calls only the oracle and the input generator.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import txe_oracle as O  # noqa: E402
from paper_2401_04189_amd import workloads as W  # noqa: E402


def main():
    s = W.build_config("cfg1")
    st = O.Setup.from_system(s)
    pairs = {}
    vx, ex = O.apply(s.psi.numpy(), st, pairs_out=pairs)
    N = s.N
    e_pairs = [pairs[(i, j)] for i in range(N) for j in range(i, N)]
    w3 = O.weights3d(st.q)
    diag = [float((w3 * s.psi.numpy()[i] * vx[i]).sum()) for i in range(N)]
    out = {"workload": "cfg1: 24^3 grid on [-6,6]^3, 4 orbitals, r = 16, K = 30, symmetric",
           "writer": "tests/golden/make_golden.py (oracle only)",
           "E_x": ex, "e_pairs_upper_row_major": e_pairs, "exchange_diagonal": diag}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_24cube.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
