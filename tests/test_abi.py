"""C-ABI checks that need no GPU: the library loads, exports every symbol of
include/libism.h, and rejects invalid arguments before touching the device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "libism.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ism_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1603_01237_amd import _lib
    L = _lib.lib()
    syms = _header_symbols()
    assert "ism_problem_create" in syms and "ism_iterate" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.EXPORTED)


def test_status_strings():
    from paper_1603_01237_amd import _lib
    for code in range(8):
        assert _lib.status_string(code)
    assert _lib.status_string(99) == "unknown status"


def _create(**kw):
    from paper_1603_01237_amd import _lib
    p = problems.spin2(K=10, N=2)
    args = dict(H0=p.H0, Hc=p.Hc, psi0=p.psi0, target=p.target, T=1.0, K=10, N=2)
    args.update(kw)
    return _lib.Problem.create(**args)


@pytest.mark.parametrize("kw", [
    {"step_map": 7},           # no such step map
    {"N": 11},                 # N > K
    {"N": 0},
    {"K": 0, "N": 0},
    {"T": -1.0},
    {"T": float("nan")},
    {"batch": 0},
])
def test_invalid_sizes_rejected(kw):
    from paper_1603_01237_amd import _lib
    with pytest.raises(_lib.IsmError) as e:
        _create(**kw)
    assert e.value.code == _lib.ISM_E_ARG


def test_non_hermitian_rejected():
    from paper_1603_01237_amd import _lib
    p = problems.spin2()
    H = p.H0.copy()
    H[0, 1] = 1.0
    with pytest.raises(_lib.IsmError) as e:
        _create(H0=H)
    assert e.value.code == _lib.ISM_E_ARG
    Hc = p.Hc.copy()
    Hc[1, 0, 1] = 0.3j          # sigma_y entry no longer conjugate-symmetric
    with pytest.raises(_lib.IsmError) as e:
        _create(Hc=Hc)
    assert e.value.code == _lib.ISM_E_ARG


def test_nan_inputs_rejected():
    from paper_1603_01237_amd import _lib
    p = problems.spin2()
    psi = p.psi0.copy()
    psi[1] = np.nan
    with pytest.raises(_lib.IsmError) as e:
        _create(psi0=psi)
    assert e.value.code == _lib.ISM_E_ARG
    with pytest.raises(_lib.IsmError) as e:
        _create(alpha=np.array([np.inf]))
    assert e.value.code == _lib.ISM_E_ARG
    with pytest.raises(_lib.IsmError) as e:
        _create(alpha=np.ones(3))      # alpha_len neither 1 nor K
    assert e.value.code == _lib.ISM_E_ARG


def test_null_pointers_rejected():
    from paper_1603_01237_amd import _lib
    L = _lib.lib()
    h = ct.c_void_p()
    o = _lib.Options()
    L.ism_default_options(ct.byref(o))
    assert L.ism_problem_create(ct.byref(h), 4, 1, None, None, None, None, 1.0, 4, 2, ct.byref(o)) == _lib.ISM_E_ARG
    assert L.ism_forward(None, None) == _lib.ISM_E_ARG
    assert L.ism_gradient(None, None) == _lib.ISM_E_ARG
    assert L.ism_iterate(None, 1, 0.1, 2.0, None, None) == _lib.ISM_E_ARG
    assert L.ism_iterate_inner(None, 1, 2, 0.1, 2.0, 0.0, None, None, None) == _lib.ISM_E_ARG
    assert L.ism_taylor_params(None, None, None) == _lib.ISM_E_ARG
    assert L.ism_fidelity(None, None, None) == _lib.ISM_E_ARG
    assert L.ism_set_controls(None, None) == _lib.ISM_E_ARG
    L.ism_problem_destroy(None)


def test_footprint_scales():
    from paper_1603_01237_amd import _lib
    a = _lib.footprint(21, 1, 20000, 128, 256)
    b = _lib.footprint(21, 1, 20000, 128, 128)
    assert a > b > 0
    assert _lib.footprint(21, 1, 100, 200, 1) == 0      # N > K
    assert _lib.footprint(256, 16, 2000, 64, 1, kind=_lib.GATE) > 0


def test_server_rejects_invalid_arguments_without_device():
    from paper_1603_01237_amd import _lib
    L = _lib.lib()
    h = ct.c_void_p()
    assert L.ism_server_create(ct.byref(h), 0, 1 << 30, 0, 4) == _lib.ISM_E_ARG   # no iterations
    assert L.ism_server_create(ct.byref(h), 0, 1 << 30, 5, 0) == _lib.ISM_E_ARG   # no slots
    assert L.ism_server_create(ct.byref(h), 0, 0, 5, 4) == _lib.ISM_E_ARG         # no budget
    assert L.ism_server_create(None, 0, 1 << 30, 5, 4) == _lib.ISM_E_ARG
    t = ct.c_uint64()
    assert L.ism_server_submit(None, None, -1.0, ct.byref(t)) == _lib.ISM_E_ARG
    assert L.ism_server_progress(None, None, None) == _lib.ISM_E_ARG
    r = _lib.Result()
    assert L.ism_server_poll(None, 1, ct.byref(r)) == _lib.ISM_E_ARG
    assert L.ism_server_take(None, 1, None, None) == _lib.ISM_E_ARG
    L.ism_server_destroy(None)
    c1 = L.ism_server_clock()
    c2 = L.ism_server_clock()
    assert c2 >= c1 > 0


def test_request_problems_of_trace_are_well_formed():
    trace = problems.serving_trace(n_req=60)
    kinds = set()
    for req in trace[:60]:
        if req["type"] == "gpe" or (req["type"] == "spin" and req["size"] == 256):
            continue                         # large set-up, covered on the GPU
        p = problems.request_problem(req)
        kinds.add(req["type"])
        assert p.K == req["K"] and p.N == req["N"]
        assert p.u0.shape[0] == 1 and p.u0.shape[1] == p.K
    assert {"spin", "rotor"} <= kinds
    arr = np.array([r["arrival"] for r in problems.serving_trace()])
    assert np.all(np.diff(arr) > 0)
    assert abs(len(arr) / arr[-1] - 200.0) < 20.0     # 2000 arrivals at a mean rate of 200/s


def test_build_refuses_kernels_with_a_dynamic_stack():
    """The build parses the compiler's resource report and refuses a kernel whose stack is
    sized at run time (its scratch would be allocated from the static size only)."""
    from paper_1603_01237_amd import build
    ok = ("k.hip:1:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]\n"
          "k.hip:1:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]\n")
    bad = ok + ("k.hip:9:1: remark: Function Name: _Z3barPd [-Rpass-analysis=kernel-resource-usage]\n"
                "k.hip:9:1: remark:     Dynamic Stack: True [-Rpass-analysis=kernel-resource-usage]\n")
    assert build._dynamic_stack_kernels(ok) == []
    assert build._dynamic_stack_kernels(bad) == ["_Z3barPd"]
