"""Writes ed_energies.json: exact lowest energies of open Hubbard chains in a
fixed (N, M, S) sector, from the oracle's exact diagonalisation only.

    python tests/golden/make_ed_energies.py

The ED itself is pinned by closed forms in tests/test_oracle_ed.py
(two-site chain and the U = 0 chain); the values here are regression pins
for the sweep tests.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ed  # noqa: E402

CASES = [  # (L, N, twoM, U, twoS)
    (4, 4, 0, 4.0, 0), (4, 4, 0, 4.0, 2),
    (5, 5, 1, 4.0, 1), (5, 5, 1, 4.0, 3),
    (6, 6, 0, 4.0, 0), (6, 6, 0, 4.0, 2),
    (8, 8, 0, 4.0, 0), (8, 8, 0, 4.0, 2),
]


def main():
    out = []
    for (L, N, twoM, U, twoS) in CASES:
        st = ed.sector_states(L, N, twoM)
        H = ed.hubbard_hamiltonian(L, 1.0, U, st)
        S2 = ed.s2_operator(L, st)
        P = ed.lowdin_projector(S2, twoS, twoM, N)
        E = ed.projected_ground_energy(H, P)
        out.append(dict(L=L, N=N, twoM=twoM, t=1.0, U=U, twoS=twoS, E=E, sector_dim=len(st)))
        print(out[-1])
    with open(os.path.join(HERE, "ed_energies.json"), "w") as f:
        json.dump({"_source": "oracle exact diagonalisation (make_ed_energies.py)",
                   "cases": out}, f, indent=1)


if __name__ == "__main__":
    main()
