"""GPU parity of the Newton slice solver (ism_iterate_newton; Sec. 4.B) against the oracle
(oracle/newton.py), FP64.

A Newton-GMRES step divides gradient differences by 2 eps and then solves with the slice
Hessian, so it amplifies the rounding of the gradients by about cond / eps.  The bars below
come from the oracle's own sensitivity, measured by perturbing its slice gradients by a
relative 1e-15 (random): two spins (eps = 1e-5), controls after 5 iterations move 5e-8;
rotor (jmax 10, N = 16, m = 8, eps = 1e-3), controls after one iteration move 1e-6.  The
library's FP64 gradients agree with the oracle's to about 1e-14, so the bars are set at 20
to 100 times those figures."""
import sys

import numpy as np
import pytest

import problems
from oracle import newton as NW

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_newton_two_spins_five_iterations():
    from paper_1603_01237_amd import _lib
    _say("case newton spin2")
    p = problems.spin2(K=200, N=8, T=2.0)
    ref = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 5, 8, 10,
                                eps=1e-5)
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate_newton(5, 10, fd_eps=1e-5)
        u = h.get_controls()[0]
    _say("J", Jh[:, 0], ref["J"], "u", _rel(u, ref["u"]))
    assert done == 5
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-8
    assert _rel(u, ref["u"]) <= 1e-6


def test_newton_rotor_batch_one_iteration():
    from paper_1603_01237_amd import _lib
    _say("case newton rotor")
    p = problems.rotor(batch=2, jmax=10, K=300, N=16, T=2.0)
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate_newton(1, 8, fd_eps=1e-3)
        u = h.get_controls()
    assert done == 1
    for b in range(2):
        ref = NW.ism_newton_iterate(p.H0_of(b), p.Hc, p.psi0, p.target, p.u0[b], p.T, p.alpha, 1,
                                    16, 8, eps=1e-3)
        _say("instance", b, "u", _rel(u[b], ref["u"]), "J", Jh[0, b] - ref["J"][0])
        assert abs(Jh[0, b] - ref["J"][0]) <= 1e-12
        assert _rel(u[b], ref["u"]) <= 1e-4


def test_newton_gate_two_iterations():
    from paper_1603_01237_amd import _lib
    _say("case newton gate")
    base = problems.spin2(K=24, N=3, T=1.0)
    rng = np.random.default_rng(3)
    W = problems.haar_unitary(4, rng)
    u0 = rng.uniform(-1, 1, size=(1, 24, 2))
    p = problems.FiniteProblem("spin2_gate", base.H0, base.Hc, np.eye(4, dtype=complex), W, 1.0,
                               24, 3, u0, np.zeros(24), 0.5, 5, kind="gate")
    ref = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 2, 3, 6,
                                eps=1e-4)
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate_newton(2, 6, fd_eps=1e-4)
        u = h.get_controls()[0]
    _say("J", Jh[:, 0], ref["J"], "u", _rel(u, ref["u"]))
    assert done == 2
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-8
    assert _rel(u, ref["u"]) <= 1e-5


def test_newton_fid_stop_and_arguments():
    from paper_1603_01237_amd import _lib
    _say("case newton stop")
    p = problems.spin2(K=200, N=8, T=2.0)
    ref = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 8, 8, 10)
    k_stop = int(np.argmax(ref["F"] >= 0.95))
    assert ref["F"][k_stop] >= 0.95 and 0 < k_stop < 8
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate_newton(8, 10, fid_stop=0.95)
        assert done == k_stop and Jh.shape[0] == k_stop + 1
        with pytest.raises(_lib.IsmError) as e:
            h.iterate_newton(1, 0)
        assert e.value.code == _lib.ISM_E_ARG
    with _lib.from_problem(p, precision="fp32") as h:
        with pytest.raises(_lib.IsmError) as e:
            h.iterate_newton(1, 4)
        assert e.value.code == _lib.ISM_E_UNSUPPORTED
