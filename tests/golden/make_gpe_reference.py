"""Write gpe_n4096_k10000.npz: the oracle's psi(T), J, F and gradient of the condensate
workload at its full size (n = 4096 on [-20, 20), g = 10, K = 10000, the seeded initial
controls).

    python tests/golden/make_gpe_reference.py      (about a minute)

It calls the oracle (oracle/gpe.py) and the input generator (problems/) only; the GPU parity
test reads the file instead of recomputing the 10^4-step forward and adjoint sweeps.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "gpe_n4096_k10000.npz")


def main():
    sys.path.insert(0, ROOT)
    import numpy as np

    import problems
    from oracle import gpe as G
    p = problems.gpe()
    g, J, F, psiK = G.adjoint_gradient(p.psi0, p.target, p.u0[0, :, 0], p.V0, p.V1, p.V2, p.g,
                                       p.L, p.T)
    np.savez_compressed(OUT, psiT=psiK, J=J, F=F, g=g)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
