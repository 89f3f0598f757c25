"""GPU parity of the condensate's frozen-density propagator assembling (ism_options.gpe_frozen;
the reading of Sec. 4.C's propagator assembling, oracle/gpe_frozen.py) against the oracle's
lagged ISM iteration, FP64.

The first iteration's boundaries come from exact sweeps; every later one assembles the slice
maps on basis vectors with the density of the previous slice pass, so J history and controls
are compared over several iterations (the GPU's step maps fuse consecutive kinetic half
steps, the oracle's do not: rounding-level differences, bar 1e-10 on J and 1e-9 on u)."""
import sys

import numpy as np
import pytest

import problems
from oracle import gpe_frozen as FZ

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _run(p, iters, rho, N):
    from paper_1603_01237_amd import _lib
    ref = FZ.ism_bec_frozen_iterate(p.psi0, p.target, p.u0[0, :, 0], p.V0, p.V1, p.V2, p.g,
                                    p.L, p.T, rho, iters, N)
    with _lib.from_problem(p, precision="fp64", N=N, gpe_frozen=True) as h:
        Jh, done = h.iterate(iters, rho)
        u = h.get_controls()[0, :, 0]
    return ref, Jh, done, u


def test_frozen_paper_grid_n64_k512():
    """The paper's condensate scale: 64 grid points on [-10, 10], 2^9 steps, T = 8, N = 8."""
    _say("case frozen n64 K512 N8")
    p = problems.gpe(n=64, L=20.0, g=1.0, dt=8.0 / 512, K=512, N=8, x_target=3.0)
    ref, Jh, done, u = _run(p, 5, 0.1, 8)
    _say("J", Jh[:, 0], ref["J"], "u", _rel(u, ref["u"]))
    assert done == 5
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10
    assert _rel(u, ref["u"]) <= 1e-9


def test_frozen_n1024_small():
    _say("case frozen n1024 K12 N2")
    p = problems.gpe(n=1024, L=40.0, g=10.0, dt=2e-3, K=12, N=2, x_target=1.0)
    ref, Jh, done, u = _run(p, 2, 0.1, 2)
    _say("J", Jh[:, 0], ref["J"], "u", _rel(u, ref["u"]))
    assert done == 2
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10
    assert _rel(u, ref["u"]) <= 1e-9


def test_frozen_rejected_at_n4096():
    from paper_1603_01237_amd import _lib
    _say("case frozen n4096 rejected")
    n = 4096
    x = -20.0 + 40.0 / n * np.arange(n)
    psi = np.exp(-0.5 * x * x).astype(complex)
    with pytest.raises(_lib.IsmError) as e:
        _lib.Problem.create_gpe(n, 40.0, 1.0, 0.5 * x * x, -x, 0.5, psi, psi, 0.1, 4, 2,
                                gpe_frozen=True)
    assert e.value.code == _lib.ISM_E_UNSUPPORTED
