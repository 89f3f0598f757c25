"""The allocation-free entry point ism_iterate_static against ism_iterate, through the C ABI.

Both run the same kernels in the same order, so on equal handles the J history, the
iteration count and the controls they leave must agree bitwise.  Two calls in a row share
the library's fixed device array, the second with a smaller problem and fewer iterations;
a request beyond the array's capacity is refused before anything runs.
"""
import sys

import numpy as np
import pytest

import problems

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(p, n_iter, rho, fid_stop, precision):
    from paper_1603_01237_amd import _lib
    with _lib.from_problem(p, precision=precision) as h:
        Js, ds = h.iterate_static(n_iter, rho, fid_stop=fid_stop)
        us = h.get_controls()
        Fs = h.fidelity()[1]
    with _lib.from_problem(p, precision=precision) as h:
        Jr, dr = h.iterate(n_iter, rho, fid_stop=fid_stop)
        ur = h.get_controls()
        Fr = h.fidelity()[1]
    return (Js, ds, us, Fs), (Jr, dr, ur, Fr)


def _check(stat, ref, n_iter):
    (Js, ds, us, Fs), (Jr, dr, ur, Fr) = stat, ref
    assert ds == dr
    rows = min(n_iter, ds + 1)
    assert np.array_equal(Js[:rows], Jr[:rows])
    assert np.all(np.isnan(Js[rows:]))            # rows the call did not write stay untouched
    assert np.array_equal(us, ur)
    assert np.array_equal(Fs, Fr)


def test_static_iterate_matches_iterate_two_calls():
    from paper_1603_01237_amd import _lib
    # first call: 8 rotors, 6 iterations, FP32 mixed
    _say("case no-alloc rotor B8 K300 N6 fp32")
    p = problems.rotor(batch=8, K=300, N=6, T=1.5)
    s, r = _pair(p, 6, p.rho, 2.0, "fp32")
    _check(s, r, 6)
    # second call, smaller: two spins, FP64, stopped early by the fidelity rule
    _say("case no-alloc spin2 K64 N4 fp64 fid_stop")
    q = problems.spin2(K=64, N=4)
    s, r = _pair(q, 40, 0.5, 0.9, "fp64")
    assert 0 < s[1] < 40
    _check(s, r, 40)


def test_static_iterate_capacity():
    from paper_1603_01237_amd import _lib
    _say("case no-alloc capacity")
    p = problems.rotor(batch=4, K=40, N=4, T=0.2)
    n_big = _lib.ISM_STATIC_HIST_MAX // 4 + 1
    with _lib.from_problem(p, precision="fp64") as h:
        u0 = h.get_controls()
        with pytest.raises(_lib.IsmError) as e:
            h.iterate_static(n_big, p.rho, record=False)
        assert e.value.code == _lib.ISM_E_BUDGET
        assert np.array_equal(h.get_controls(), u0)
        Jh, done = h.iterate_static(_lib.ISM_STATIC_HIST_MAX // 4, 0.0, fid_stop=0.0)
        assert done == 0 and np.all(np.isfinite(Jh[0]))
