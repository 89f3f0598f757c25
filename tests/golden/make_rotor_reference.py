"""Write rotor_b256_k20000.npz: the FP64 oracle's psi(T), lambda(0), J and F for every
instance of the rotor batch at its full size (256 rotors, d = 21, K = 20000, the seeded
initial controls), for the exponential map and the Crank-Nicolson map.

    python tests/golden/make_rotor_reference.py      (about 2 minutes on 8 cores)

It calls the oracle (oracle/finite.py) and the input generator (problems/) only; the GPU
parity tests read the file instead of recomputing 2 x 256 trajectories of 20000 steps.
"""
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "rotor_b256_k20000.npz")


def _one(args):
    b, step = args
    sys.path.insert(0, ROOT)
    import numpy as np

    import problems
    from oracle import finite as O
    p = problems.rotor()
    mk = O.step_unitaries if step == "exp" else O.step_unitaries_cn
    Us = mk(p.H0_of(b), p.Hc, p.u0[b], p.T / p.K)
    psiK = O.forward(Us, p.psi0)[-1]
    lam0 = O.backward(Us, p.target)[0]
    z = O.inner(psiK, p.target)
    return psiK, lam0, z.real, abs(z) ** 2


def main():
    import numpy as np
    sys.path.insert(0, ROOT)
    import problems
    B = problems.rotor().batch
    out = {}
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        for step in ("exp", "cn"):
            res = pool.map(_one, [(b, step) for b in range(B)])
            out[f"{step}_psiT"] = np.stack([r[0] for r in res])
            out[f"{step}_lam0"] = np.stack([r[1] for r in res])
            out[f"{step}_J"] = np.array([r[2] for r in res])
            out[f"{step}_F"] = np.array([r[3] for r in res])
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
