"""Writes burgers_shock_reference_k10_ne160.txt: the reference solution of the
steep-gradient viscous Burgers problem (Section 5.1, "A solution with steep
gradient": u(x, 0) = sin(2 pi x) on [0, 1], zero Dirichlet ends,
kappa = 0.002) at t = 1 on 160 elements of degree 10 with the Lax-Friedrichs
flux, the discretization of the paper's reference.  The paper integrates it
with RK4 at dt = 5e-7; here the oracle's EXPRB32 at dt = 2e-3 and Krylov
tolerance 1e-12 (its temporal error, about 4e-9 by the dt^3 scaling of Table
expo-burgers-tconv-shock, is far below the errors the tables print).

Only the oracle is called.  Run from the repository root:
    python tests/golden/make_burgers_shock_reference.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

OUT = os.path.join(HERE, "burgers_shock_reference_k10_ne160.txt")


def main():
    m = oracle.Mesh(oracle.BURGERS1D, 160, 10, x0=0.0, x1=1.0, kappa=0.002,
                    bc=oracle.BC_DIRICHLET)
    q = np.sin(2.0 * math.pi * m.nodes()[0])
    for _ in range(500):
        q, _ = m.step(oracle.EXPRB32, 2e-3, q, tol=1e-12, m_min=5, m_max=64)
    with open(OUT, "w") as f:
        f.write("# steep-gradient viscous Burgers at t = 1, 160 elements of degree 10 (LF),\n")
        f.write("# nodal values in element order; written by make_burgers_shock_reference.py\n")
        for v in q:
            f.write(f"{v:.17e}\n")


if __name__ == "__main__":
    main()
