"""Benchmark: ISM iterations on the rotor batch (molecular-orientation stand-in).

Workload: 256 rigid rotors (j = 0..20, d = 21, H_b = B_b j(j+1) - u cos(theta),
B_b ~ U(0.8, 1.2)), T = 10, K = 20000 steps, N = 128 slices, psi0 = |0,0>, target =
top cos(theta) eigenvector in j <= 4, seeded controls u0 = 1 + U(-0.01, 0.01),
constant step rho = 1.  One benchmark step = one ISM iteration (Algorithm 1 with
one gradient step per slice): per-step generator data, slice propagator assembly,
boundary rebuild by 2N products, intermediate states, slice forward/adjoint sweeps
with the exact gradient, control update.  Inputs are resident in device memory
before the timed region.

value  = useful propagation steps/s of the FP32 mixed path = B * 2K * steps / time
         (forward + adjoint, per the metric), with the plain FP64 ISM measured on the
         same data beside it.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "propagation steps/s (fwd+adjoint) FP32 vs plain FP64 ISM; p50/p99 solve latency"
PEAK_ALU = 78.6e12       # non-packed FP32 and FP64 vector FMA rate: 256 CU x 64 lanes x 2 x 2.4 GHz

# HBM traffic of the dominant kernel, from two rocprofv3 counter runs of this script
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each divided by what the same counter
# reads per KiB actually moved by a plain streaming kernel of known size (--copy-calibration).
# It holds for the kernel sources it was taken on (sha256 over TRAFFIC_SOURCES); after any
# change to them the field is reported as null until the counters are taken again.
TRAFFIC_SOURCES = ["paper_1603_01237_amd/csrc/k_sparse.hip",
                   "paper_1603_01237_amd/csrc/ism_internal.h"]
TRAFFIC = {"kernel": "sp_assemble", "fetch_kib": 32521.2, "write_kib": 113344.0,
           "copy_fetch_per_kib": 0.50001, "copy_write_per_kib": 1.0,
           "sha256": "527323be7fd8d176ecfa1713a8d358728ed81f89894cd983b410778d0c318eed"}
COPY_BYTES = 1 << 30


def _sources_sha():
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(kernel):
    t = TRAFFIC
    if kernel != t["kernel"] or t["sha256"] is None or t["sha256"] != _sources_sha():
        return None
    return 1024.0 * (t["fetch_kib"] / t["copy_fetch_per_kib"]
                     + t["write_kib"] / t["copy_write_per_kib"])


def copy_calibration():
    """A plain streaming kernel of known size (reads COPY_BYTES, writes COPY_BYTES), for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = COPY_BYTES // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "elementwise neg", "read_bytes": COPY_BYTES,
                                           "write_bytes": COPY_BYTES, "launches": 3}}), flush=True)


def serving_sample(n_req, max_iter=20, iters_per_round=5, max_running=16, shapes="continuous"):
    """Replay of the first n_req requests of the seeded 200 req/s serving trace at their
    arrival times (FP32 mixed; stop at F >= 0.99 or max_iter iterations).  The trace offers
    far more work than the device serves (200 requests arrive within about a second), so the
    server is saturated from the start and solves/s over the replay is its sustainable rate
    for this request mix."""
    import numpy as np
    import problems
    from paper_1603_01237_amd import Server
    from paper_1603_01237_amd.serve import latency_summary, replay
    trace = problems.serving_trace(shapes=shapes)[:n_req]
    types = [f"{r['type']}{r['size']}" for r in trace]
    items = [(r["arrival"] - trace[0]["arrival"], problems.request_problem(r),
              dict(max_iter=max_iter, rho=problems.SERVE_RHO[r["type"]], fid_stop=0.99,
                   precision="fp32")) for r in trace]
    with Server(200 << 30, iters_per_round=iters_per_round, max_running=max_running) as s:
        recs, wall = replay(s, items, timeout=600.0, report_every=10.0,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
        st = s.stats()
    out = latency_summary(recs, wall)
    by_type = {}
    for t, r in zip(types, recs):
        by_type.setdefault(t, []).append(r["latency_s"])
    out["latency_s_by_type"] = {t: {"n": len(v), "p50": float(np.percentile(v, 50)),
                                    "p99": float(np.percentile(v, 99))}
                                for t, v in sorted(by_type.items())}
    out.update({"sustainable_solves_per_s": out["solves_per_s"],
                "offered_req_per_s": n_req / max(trace[-1]["arrival"] - trace[0]["arrival"], 1e-9),
                "handles": st["groups"], "merged_requests": st["merged"],
                "request_in_flight_frac": st["busy_s"] / wall if wall > 0 else None,
                "peak_device_GB": st["bytes_peak"] / 1e9,
                "mean_iters": float(sum(r["iters"] for r in recs) / max(len(recs), 1)),
                "reached_F099": int(sum(r["F"] >= 0.99 for r in recs)),
                "sample": f"first {n_req} requests of the seeded 200 req/s trace (spin d in "
                          "{4,16,64,256}, rotor j<=10/20/40, GPE n=1024/4096; " +
                          ("K log-uniform 1000..20000, N 16..128" if shapes == "continuous" else
                           "K in {1000,2000,5000,10000,20000}, N in {16,32,64,128}") +
                          "), arrival-time replay, FP32 mixed, stop at "
                          f"F>=0.99 or {max_iter} iterations (the trace's 200 capped to keep the "
                          "replay near a minute); request_in_flight_frac: share of the wall "
                          "time with at least one request running (not GPU utilisation)"})
    return out


def _sparse_row_costs(prob):
    """Per-row flop weights of one Taylor term: 4 flops per stored real nonzero (8 if complex)
    plus 4 for the term scaling and accumulation; returns (H rows sum, per-control rows sum)."""
    import numpy as np
    H0 = prob.H0_of(0)
    pattern = (np.abs(H0) > 0)
    cplx = np.any(np.abs(H0.imag) > 0)
    for c in range(prob.C):
        pattern |= np.abs(prob.Hc[c]) > 0
        cplx |= np.any(np.abs(prob.Hc[c].imag) > 0)
    w = 8 if cplx else 4
    h_rows = float(np.sum(w * pattern.sum(axis=1) + 4))
    c_rows = [float(np.sum(w * (np.abs(prob.Hc[c]) > 0).sum(axis=1))) for c in range(prob.C)]
    return h_rows, c_rows


def algorithmic_flops(prob, terms):
    """Algorithmic FP operations per launch of the two hot kernels of the sparse path;
    terms[b] = generator applications per step of instance b (m_b S_b for the Taylor map,
    n_b + 1 for Crank-Nicolson), as the library chose them."""
    h_rows, c_rows = _sparse_row_costs(prob)
    K, d, C = prob.K, prob.d, prob.C
    B = len(terms)
    mS = float(sum(terms))                          # sum over instances
    assemble = K * d * h_rows * mS                  # d basis vectors through every step
    slice_ = K * ((3 + C) * h_rows * mS             # forward, adjoint, reversal, Frechet
                  + sum(cr for cr in c_rows) * mS   # H_c applied to the adjoint terms
                  + B * C * 8 * d)                  # overlaps
    return {"sp_assemble": assemble, "sp_slice": slice_}


PEAK_MFMA = {"fp32": 157.3e12, "fp64": 78.6e12}    # dense MFMA, v_mfma_*_16x16x4
PEAK_CU_FP64 = 78.6e12 / 256                       # one CU (a sequential sweep is one workgroup)


def gate_gemm_flops(prob, d):
    """Algorithmic MFMA work of one ISM iteration of the dense path (path precision), 8 d^3
    flops per complex d x d x d product: the assembly chain P_j = U_j P_{j-1} (K - N
    products), the slice right-hand sides M_n^+ phi_{n+1} (N; density matrices: N more for
    the right factor M_n) and [X_j | Y_j] = P_{j-1} [phi_n | .] (K - N products of twice the
    width).  d is the unpadded dimension (the kernels pad to a multiple of 64)."""
    K, N = prob.K, prob.N
    extra = N if getattr(prob, "kind", "") == "density" else 0
    return 8.0 * d ** 3 * (3 * K - 2 * N + extra)


def gate_grad_flops(prob, prec):
    """Algorithmic work of one launch of the dense path's gradient kernel, summed over the K
    steps with the Krylov order m_j each step needs at its controls (the kernel's own rule:
    x = 2 tau (||H0 - s||_inf + sum_c |u_jc| ||H_c||_inf), terms until x^(m+2)/(m+3)! is
    below 1e-17 in FP64, min(1e-8, 1e-5/K) in FP32).  Per step and column of X_j, Y_j and per
    row r with w_r entries in the union pattern of H0 and the controls:
      16 m w_r        the Krylov sequences p_a = (tau H')^a y and r_b = (tau H')^b x
      2 (m+1)(m+2)    the weights t_b = sum_a conj(w_ab) p_a (real weight times complex)
      8 (m+1) w_r     S_w = sum_b conj(t_b) r_b(col_w)
and once per step and row, S_w being summed over the columns first:
      4 nnz_c(r)      Im(h S_w) per control entry of the row (summed over controls)."""
    import numpy as np
    K, d, C = prob.K, prob.d, prob.C
    H0 = prob.H0_of(0)
    dg = np.real(np.diag(H0))
    s = 0.5 * (dg.max() + dg.min())
    pat = np.abs(H0) > 0
    np.fill_diagonal(pat, True)
    nnz_c = 0
    for c in range(C):
        pat |= np.abs(prob.Hc[c]) > 0
        nnz_c += int((np.abs(prob.Hc[c]) > 0).sum())
    w_sum = float(pat.sum())
    h0norm = float(np.abs(H0 - s * np.eye(d)).sum(axis=1).max())
    cnorm = np.array([np.abs(prob.Hc[c]).sum(axis=1).max() for c in range(C)])
    tau = prob.T / K
    tol = 1e-17 if prec == "fp64" else min(1e-8, 1e-5 / K)
    cap = 16 if prec == "fp64" else 12
    u = prob.u0[0]
    total = 0.0
    for j in range(K):
        x = 2 * tau * (h0norm + float(np.abs(u[j]) @ cnorm))
        m, rem = 1, x * x / 6
        while m < cap and rem > tol:
            m += 1
            rem = rem * x / (m + 2)
        total += d * (16 * m * w_sum + d * 2 * (m + 1) * (m + 2) + 8 * (m + 1) * w_sum) + 4 * nnz_c
    return total


def gpe_sweep_flops(prob):
    """FFT work of the two sequential sweeps of one iteration: 2K steps of two length-n
    transforms at 5 n log2 n flops each (pointwise work not counted)."""
    import math
    return 2.0 * prob.K * 2 * 5 * prob.n * math.log2(prob.n) * prob.batch


def other_workloads(stream, iters_gate=2, iters_gpe=2,
                    which=("spins", "gate", "gpe", "rotor_cn", "rotor_inner", "rotor_newton",
                           "density")):
    """The paper's other benchmark shapes: the two-spin solve (latency), gate synthesis
    on MFMA, the condensate (sequential FFT sweeps), and the rotor batch with the
    Crank-Nicolson step map and with several gradient steps per slice problem."""
    import problems
    out = {}
    if "rotor_cn" in which:
        out.update(_rotor_cn_workload(stream))
    if "rotor_inner" in which:
        out.update(_rotor_inner_workload(stream))
    if "rotor_newton" in which:
        out.update(_rotor_newton_workload(stream))
    if "density" in which:
        out.update(_density_workload(stream))
        out.update(_density_cn_workload(stream))
    if "spins" in which:
        out.update(_spins_workload(stream))
    if "gate" in which:
        out.update(_gate_workload(stream, iters_gate))
    if "gpe" in which:
        out.update(_gpe_workload(stream, iters_gpe))
        out.update(_gpe_frozen_workload(stream))
    return out


def _rotor_cn_workload(stream, steps=3):
    """The benchmark's rotor batch with the Crank-Nicolson map (Sec. 3): each step is
    (I - L) then the Neumann series of (I + L)^{-1}, n terms from the norm bound."""
    import problems
    prob = problems.rotor()
    B = prob.batch
    r = {prec: run_gpu(prec, prob, steps, 1, stream, step_map="cn") for prec in ("fp32", "fp64")}
    ent = {"workload": f"rotor batch with the Crank-Nicolson map: {B} instances, d=21, "
                       f"K={prob.K}, N={prob.N}",
           "ms_per_iteration": {k: v["seconds"] / steps * 1e3 for k, v in r.items()},
           "useful_steps_per_s": {k: B * 2 * prob.K * steps / v["seconds"] for k, v in r.items()},
           "neumann_terms": {k: v["info"]["taylor_m"] for k, v in r.items()},
           "kernels_ms_per_iteration": {k: {n: t[1] / steps for n, t in v["kernels"].items()}
                                        for k, v in r.items()},
           "final_F_mean": {k: v["F_mean"] for k, v in r.items()}}
    for prec, v in r.items():
        launches, ms = v["kernels"]["sp_assemble"]
        # (n + 1) applications of tau/2 H per step: (I - L) and n Neumann terms
        fl = algorithmic_flops(prob, [t + 1 for t in v["info"]["terms"]])["sp_assemble"]
        ach = fl / (ms / launches * 1e-3)
        ent[f"roofline_{prec}"] = {"bound": "alu", "kernel": "sp_assemble", "achieved": ach / 1e12,
                                   "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s",
                                   "frac": ach / PEAK_ALU}
    return {"rotor_cn": ent}


def _rotor_inner_workload(stream, steps=3, ell=3):
    """The benchmark's rotor batch with ell gradient steps per slice problem and the Err rule
    (Algorithm 1 steps (c) and (e)): per iteration one assembly and boundary rebuild, ell
    slice passes with updates and one slice pass for Err.  Each inner step is rho/ell, so
    that an iteration moves the controls about as far as one plain step (ell steps of the
    full rho overshoot on this problem)."""
    import dataclasses
    import problems
    prob = problems.rotor()
    prob = dataclasses.replace(prob, rho=prob.rho / ell)
    B = prob.batch
    r = {prec: run_gpu(prec, prob, steps, 1, stream, n_inner=ell) for prec in ("fp32", "fp64")}
    passes = ell + 1
    ent = {"workload": f"rotor batch, {ell} gradient steps of rho/{ell} per slice problem + Err: "
                       f"{B} instances, d=21, K={prob.K}, N={prob.N}",
           "ms_per_iteration": {k: v["seconds"] / steps * 1e3 for k, v in r.items()},
           "slice_passes_per_iteration": passes,
           "slice_steps_per_s": {k: B * 2 * prob.K * passes * steps / v["seconds"]
                                 for k, v in r.items()},
           "kernels_ms_per_iteration": {k: {n: t[1] / steps for n, t in v["kernels"].items()}
                                        for k, v in r.items()},
           "Err_mean_per_iteration": {k: v["Err_mean"] for k, v in r.items()},
           "final_F_mean": {k: v["F_mean"] for k, v in r.items()}}
    for prec, v in r.items():
        launches, ms = v["kernels"]["sp_slice"]
        fl = algorithmic_flops(prob, v["info"]["terms"])["sp_slice"]
        ach = fl / (ms / launches * 1e-3)
        ent[f"roofline_slice_{prec}"] = {"bound": "alu", "kernel": "sp_slice", "achieved": ach / 1e12,
                                         "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s",
                                         "frac": ach / PEAK_ALU}
    return {"rotor_inner": ent}


def _density_workload(stream, steps=2):
    """The five-spin density-matrix run (Sec. 4.A, Liouville-von Neumann form, K = 2^15) on
    the dense MFMA path: one ISM iteration per step at N = 1, 2, 4, 8 slices (FP32 mixed) and
    at N = 8 in FP64; the efficiency t(1) / (N t(N)) is the single-GPU counterpart of the
    paper's parallel-efficiency table."""
    import problems
    p = problems.spin5_density()
    out = {"workload": f"five spins, density matrices (d=32), K={p.K}, one ISM iteration per "
                       f"step, constant step {p.rho:g}",
           "ms_per_iteration": {}, "kernels_ms_per_iteration": {}}
    for N in (1, 2, 4, 8):
        q = problems.spin5_density(N=N)
        r = run_gpu("fp32", q, steps, 1, stream)
        out["ms_per_iteration"][f"fp32_N{N}"] = r["seconds"] / steps * 1e3
        out["kernels_ms_per_iteration"][f"fp32_N{N}"] = {n: t[1] / steps for n, t in r["kernels"].items()}
        if N == 8:
            out["final_J_fp32_N8"] = r["J_mean"]
            launches, ms = r["kernels"]["gate_gemm"]
            ach = gate_gemm_flops(q, q.d) * steps / (ms * 1e-3)
            out["roofline_fp32_N8"] = {"bound": "mfma", "kernel": "gate_gemm (all batched GEMMs)",
                                       "achieved": ach / 1e12, "peak": PEAK_MFMA["fp32"] / 1e12,
                                       "unit": "TFLOP/s", "frac": ach / PEAK_MFMA["fp32"]}
    r = run_gpu("fp64", p, steps, 1, stream)
    out["ms_per_iteration"]["fp64_N8"] = r["seconds"] / steps * 1e3
    out["kernels_ms_per_iteration"]["fp64_N8"] = {n: t[1] / steps for n, t in r["kernels"].items()}
    t = out["ms_per_iteration"]
    # t(1) / (N t(N)): the paper's parallel efficiency, which on one GPU measures how the
    # slicing changes the per-iteration time (the chunked scans make it flat in N), not the
    # use of N processors
    out["slicing_time_ratio_fp32"] = {f"N{N}": t["fp32_N1"] / (N * t[f"fp32_N{N}"])
                                      for N in (1, 2, 4, 8)}
    out["useful_matrix_steps_per_s"] = {k: 2 * p.K / (v * 1e-3) for k, v in t.items()}
    return {"spin5_density": out}


def _gpe_frozen_workload(stream, iters=40, target=0.998):
    """The condensate at the paper's scale (64 grid points on [-10, 10], 2^9 steps, T = 8,
    g = 1, rho = 0.1; the moving-trap stand-in for Sec. 4.C's double well): iterations and time
    to reach J >= target with the frozen-density boundaries (B16) for N = 1..32 slices, and
    with the exact sweeps (the plain gradient method's iterates).  The counterpart of Table
    tabGP: iterations(N = 1) / iterations(N), and the wall time to the target against the
    sequential method."""
    import numpy as np
    import problems
    from paper_1603_01237_amd import _lib
    base = problems.gpe(n=64, L=20.0, g=1.0, dt=8.0 / 512, K=512, N=1, x_target=3.0)
    out = {"workload": "condensate, n=64 on [-10,10], K=512, T=8, g=1, rho=0.1, FP64; "
                       f"iterations to J >= {target}",
           "frozen": {}, "exact": {}}
    for frozen in (True, False):
        for N in (1, 2, 4, 8, 16, 32):
            with _lib.from_problem(base, precision="fp64", N=N, stream=stream,
                                   gpe_frozen=frozen) as h:
                t0 = time.perf_counter()
                Jh, done = h.iterate(iters, 0.1)
                dt = time.perf_counter() - t0
            J = Jh[:, 0]
            hit = np.nonzero(J >= target)[0]
            key = "frozen" if frozen else "exact"
            out[key][f"N{N}"] = {"iterations": int(hit[0]) if hit.size else None,
                                 "ms_per_iteration": dt / iters * 1e3,
                                 "J_final": float(J[-1])}
    for key in ("frozen", "exact"):
        for v in out[key].values():
            v["ms_to_target"] = (v["iterations"] * v["ms_per_iteration"]
                                 if v["iterations"] is not None else None)
    it1 = out["frozen"]["N1"]["iterations"]
    out["iteration_ratio_frozen"] = {k: (it1 / v["iterations"] if it1 and v["iterations"] else None)
                                     for k, v in out["frozen"].items()}
    # wall time to the target against the sequential method (exact sweeps, N = 1) on the
    # same GPU: what the assembled boundaries buy here
    t1 = out["exact"]["N1"]["ms_to_target"]
    out["speedup_vs_sequential"] = {k: (t1 / v["ms_to_target"] if t1 and v["ms_to_target"] else None)
                                    for k, v in out["frozen"].items()}
    return {"gpe_frozen_n64": out}


def _rotor_newton_workload(stream, iters=8, m=10, eps=1e-4, batch=16):
    """Newton-GMRES slice solver (Sec. 4.B, Table tabnewt) on the benchmark's rotors
    (first `batch` instances, K = 20000, FP64): J after each of `iters` iterations for
    N = 1, 2, 4, ..., 128, time per iteration, and N t per iteration (the paper's
    equivalent sequential time per iteration)."""
    import numpy as np
    import problems
    from paper_1603_01237_amd import _lib
    out = {"workload": f"rotor batch, first {batch} instances, d=21, K=20000, FP64, one "
                       f"Newton step per slice, GMRES m={m}, eps={eps}", "by_N": {}}
    for N in (1, 2, 4, 8, 16, 32, 64, 128):
        p = problems.rotor(batch=batch, N=N)
        with _lib.from_problem(p, precision="fp64", stream=stream) as h:
            t0 = time.perf_counter()
            Jh, done = h.iterate_newton(iters, m, fd_eps=eps)
            dt = time.perf_counter() - t0
        J = Jh.mean(axis=1)
        out["by_N"][f"N{N}"] = {"J_mean_per_iteration": [float(x) for x in J],
                                "ms_per_iteration": dt / max(done, 1) * 1e3,
                                "N_times_ms_per_iteration": N * dt / max(done, 1) * 1e3}
    return {"rotor_newton": out}


def _density_cn_workload(stream, steps=2):
    """The five-spin density-matrix run with the Crank-Nicolson map at tau = T / 2^15, N = 8
    (Sec. 3 scheme on the conjugation form): Cayley steps built as D_j = U_j - I by a Neumann
    series, the gradient from A x and A y, A = (I + L_j)^{-1}."""
    import problems
    p = problems.spin5_density()
    r = {prec: run_gpu(prec, p, steps, 1, stream, step_map="cn") for prec in ("fp32", "fp64")}
    return {"spin5_density_cn": {
        "workload": f"five spins, density matrices (d=32), Crank-Nicolson map, K={p.K} "
                    f"(tau = T/2^15), N={p.N}, one ISM iteration per step",
        "ms_per_iteration": {k: v["seconds"] / steps * 1e3 for k, v in r.items()},
        "useful_matrix_steps_per_s": {k: 2 * p.K * steps / v["seconds"] for k, v in r.items()},
        "kernels_ms_per_iteration": {k: {n: t[1] / steps for n, t in v["kernels"].items()}
                                     for k, v in r.items()},
        "final_J": {k: v["J_mean"] for k, v in r.items()}}}


def _spins_workload(stream):
    import problems
    out = {}
    p0 = problems.spin2()
    r = {prec: run_gpu(prec, p0, p0.iters, 1, stream, timing=False) for prec in ("fp64", "fp32")}
    out["spins_d4"] = {
        "workload": f"two coupled spins, d=4, K={p0.K}, N={p0.N}, {p0.iters} iterations (one solve)",
        "solve_ms": {k: v["seconds"] * 1e3 for k, v in r.items()},
        "useful_steps_per_s": {k: 2 * p0.K * p0.iters / v["seconds"] for k, v in r.items()},
        "final_F": {k: v["F_mean"] for k, v in r.items()}}
    return out


def _gate_workload(stream, iters_gate):
    import problems
    out = {}
    pg = problems.spin_chain_gate()
    r = {prec: run_gpu(prec, pg, iters_gate, 1, stream) for prec in ("fp32", "fp64")}
    dp = pg.d
    ent = {"workload": f"gate synthesis, 8-spin chain d={pg.d}, C={pg.C}, K={pg.K}, N={pg.N}",
           "ms_per_iteration": {k: v["seconds"] / iters_gate * 1e3 for k, v in r.items()},
           "useful_matrix_steps_per_s": {k: 2 * pg.K * iters_gate / v["seconds"]
                                         for k, v in r.items()},
           "kernels_ms_per_iteration": {k: {n: t[1] / iters_gate for n, t in v["kernels"].items()}
                                        for k, v in r.items()}}
    for prec, v in r.items():
        launches, ms = v["kernels"]["gate_gemm"]
        ach = gate_gemm_flops(pg, dp) * iters_gate / (ms * 1e-3)
        ent[f"roofline_{prec}"] = {"bound": "mfma", "kernel": "gate_gemm (all batched GEMMs)",
                                   "achieved": ach / 1e12, "peak": PEAK_MFMA[prec] / 1e12,
                                   "unit": "TFLOP/s", "frac": ach / PEAK_MFMA[prec]}
        # the gradient kernel: one effective launch per iteration (of the two Krylov bounds,
        # the one not needed exits at once); controls at u0 (the timed iterations move them
        # little, and m_j is recomputed at u0 here)
        launches, ms = v["kernels"]["gate_grad"]
        ach = gate_grad_flops(pg, prec) * iters_gate / (ms * 1e-3)
        ent[f"roofline_grad_{prec}"] = {"bound": "alu", "kernel": "gate_grad",
                                        "achieved": ach / 1e12, "peak": PEAK_ALU / 1e12,
                                        "unit": "TFLOP/s", "frac": ach / PEAK_ALU,
                                        "algorithmic_TFLOP_per_launch": gate_grad_flops(pg, prec) / 1e12}
    out["gate_d256"] = ent
    return out


def _gpe_workload(stream, iters_gpe):
    import problems
    out = {}
    pe = problems.gpe()
    r = {prec: run_gpu(prec, pe, iters_gpe, 1, stream) for prec in ("fp32", "fp64")}
    ent = {"workload": f"condensate, n={pe.n}, K={pe.K}, N={pe.N}, g={pe.g}",
           "ms_per_iteration": {k: v["seconds"] / iters_gpe * 1e3 for k, v in r.items()},
           "useful_steps_per_s": {k: 2 * pe.K * iters_gpe / v["seconds"] for k, v in r.items()},
           "kernels_ms_per_iteration": {k: {n: t[1] / iters_gpe for n, t in v["kernels"].items()}
                                        for k, v in r.items()}}
    for prec, v in r.items():
        launches, ms = v["kernels"]["gpe_sweep"]
        ach = gpe_sweep_flops(pe) * iters_gpe / (ms * 1e-3)
        ent[f"roofline_{prec}"] = {"bound": "alu, one CU (sequential sweep)",
                                   "kernel": "gpe fwd+adj sweeps", "achieved": ach / 1e9,
                                   "peak": PEAK_CU_FP64 / 1e9, "unit": "GFLOP/s",
                                   "frac": ach / PEAK_CU_FP64,
                                   "us_per_step": ms * 1e3 / iters_gpe / (2 * pe.K)}
    out["gpe_n4096"] = ent
    return out


def run_gpu(prec, prob, steps, warmup, stream_ptr, timing=True, step_map="exp", n_inner=None):
    """Warm-up iterations, controls reset to u0, then `steps` timed iterations (per-kernel
    HIP events on the handle's stream when `timing`).  With n_inner, the iterations take
    n_inner gradient steps per slice problem and evaluate Err (ism_iterate_inner)."""
    import torch
    from paper_1603_01237_amd import _lib
    h = _lib.from_problem(prob, precision=prec, stream=stream_ptr, step_map=step_map)
    if n_inner is None:
        h.iterate(warmup, prob.rho, record=False)
    else:
        h.iterate_inner(warmup, n_inner, prob.rho, record=False)
    h.set_controls(prob.u0)
    torch.cuda.synchronize()
    h.set_timing(timing)
    h.kernel_times()
    torch.cuda.synchronize()
    Eh = None
    t0 = time.perf_counter()
    if n_inner is None:
        h.iterate(steps, prob.rho, record=False)
    else:
        _, Eh, _ = h.iterate_inner(steps, n_inner, prob.rho, record=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = h.kernel_times()
    h.set_timing(False)
    info = h.info()
    if info["path"] == 0:
        try:
            m_b, S_b = h.taylor_params()
            info["terms"] = [m * S for m, S in zip(m_b, S_b)]
        except _lib.IsmError:     # one-launch solve: its series are chosen per step
            info["terms"] = None
    J, F = h.fidelity()
    h.close()
    out = {"seconds": t1 - t0, "kernels": kt, "info": info, "J_mean": float(J.mean()),
           "F_mean": float(F.mean())}
    if Eh is not None:
        out["Err_mean"] = [float(e) for e in Eh.mean(axis=1)]
    return out


def _cpu_info():
    """CPU model, logical CPUs and physical cores of this host (Linux /proc/cpuinfo)."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "physical_cores": len(cores) or None}


def _slice_worker(conn, H0, Hc, psi0, target, T, K, N, alpha, mine):
    """One process of the CPU-parallel ISM (the paper's one-process-per-slice layout, several
    slices per process): for its slices, the step propagators, step averages and slice
    propagator (Sec. 3, propagator assembling), then the slice gradients once the master has
    sent the intermediate states."""
    from threadpoolctl import threadpool_limits
    from oracle import finite as O
    s = O.slice_starts(K, N)
    tau = T / K
    with threadpool_limits(1):
        while True:
            msg = conn.recv()
            if msg is None:
                return
            if msg[0] == "build":
                u = msg[1]
                Us, Hh, Ms = {}, {}, {}
                for n in mine:
                    for j in range(s[n], s[n + 1]):
                        Us[j] = O.step_unitary(O.hamiltonian(H0, Hc, u[j]), tau)
                        Hh[j] = O.hhat(O.hamiltonian(H0, Hc, u[j]), Hc, tau)
                    Ms[n] = O.assemble([Us[j] for j in range(s[n], s[n + 1])], [0, s[n + 1] - s[n]])[0]
                conn.send(Ms)
            else:
                phi = msg[1]
                out = {}
                for n in mine:
                    UU = [None] * K
                    HH = [None] * K
                    for j in range(s[n], s[n + 1]):
                        UU[j], HH[j] = Us[j], Hh[j]
                    out[n] = O.ism_slice_gradient(UU, HH, u, alpha, phi[n], phi[n + 1], s[n],
                                                  s[n + 1], K)[0]
                conn.send(out)


def cpu_baseline(prob, n_inst, reps=5, warm=2):
    """The FP64 oracle timed on this host, on a bounded sample of the workload: one ISM
    iteration (Algorithm 1, one gradient step per slice) of instance 0, the median of `reps`
    repetitions after `warm` untimed ones.
      - single core: the oracle's ISM iteration in one thread;
      - P cores: the paper's CPU-parallel ISM, P = min(N, physical cores, 16) worker
        processes holding contiguous blocks of slices, the master doing the boundary rebuild
        (2N products) and the update."""
    import multiprocessing as mp
    import statistics
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import finite as O
    b = 0
    H0, u0 = prob.H0_of(b), prob.u0[b]

    def one_core():
        with threadpool_limits(1):
            g, *_ = O.ism_gradient(H0, prob.Hc, prob.psi0, prob.target, u0, prob.T, prob.alpha,
                                   prob.N)
            return u0 + prob.rho * g

    times = []
    for k in range(warm + reps):
        t0 = time.perf_counter()
        u1 = one_core()
        if k >= warm:
            times.append(time.perf_counter() - t0)
    t1 = statistics.median(times)
    info = _cpu_info()
    P = max(1, min(prob.N, info["physical_cores"] or os.cpu_count() or 1, 16))
    s = O.slice_starts(prob.K, prob.N)
    blocks = [list(range(w * prob.N // P, (w + 1) * prob.N // P)) for w in range(P)]
    ctx = mp.get_context("spawn")
    pipes, procs = [], []
    for w in range(P):
        a, c = ctx.Pipe()
        pr = ctx.Process(target=_slice_worker, args=(c, H0, prob.Hc, prob.psi0, prob.target,
                                                     prob.T, prob.K, prob.N, prob.alpha,
                                                     blocks[w]), daemon=True)
        pr.start()
        pipes.append(a)
        procs.append(pr)

    def p_cores():
        for a in pipes:
            a.send(("build", u0))
        Ms = {}
        for a in pipes:
            Ms.update(a.recv())
        Psi, Lam = O.boundaries([Ms[n] for n in range(prob.N)], prob.psi0, prob.target)
        phi = O.intermediate_states(Psi, Lam, s, prob.K)
        for a in pipes:
            a.send(("grad", phi))
        g = np.zeros_like(u0)
        for a in pipes:
            for n, gn in a.recv().items():
                g[s[n]:s[n + 1]] = gn
        return u0 + prob.rho * g

    ptimes = []
    try:
        for k in range(warm + reps):
            t0 = time.perf_counter()
            uP = p_cores()
            if k >= warm:
                ptimes.append(time.perf_counter() - t0)
    finally:
        for a in pipes:
            a.send(None)
        for pr in procs:
            pr.join(timeout=10)
    tP = statistics.median(ptimes)
    same = float(np.max(np.abs(uP - u1)))
    steps = 2 * prob.K                     # useful steps of one instance and iteration
    return {"value": steps / t1, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"instance 0 of {prob.batch}, 1 ISM iteration (K={prob.K}, N={prob.N}), "
                      f"FP64 NumPy, one thread; median of {reps} after {warm} warm-ups: "
                      f"{t1:.2f} s",
            "p_cores": {"value": steps / tP, "unit": "steps/s", "cores": P,
                        "sample": f"same iteration, {P} worker processes with contiguous "
                                  f"slice blocks, boundaries on the master; median "
                                  f"{tP:.2f} s; controls equal the single-core ones to "
                                  f"{same:.1e}"},
            "host": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=3, help="oracle instances timed (0: skip)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the two-spin, gate and condensate workloads")
    ap.add_argument("--serve", type=int, default=200,
                    help="requests of the serving trace replayed for p50/p99 latency (0: skip)")
    ap.add_argument("--only", choices=["spins", "gate", "gpe", "rotor_cn", "rotor_inner",
                                       "rotor_newton", "density"],
                    help="run only this secondary workload and print its figures (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the streaming kernel that scales the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU sharding of ISM slices and "
              "instances is a design (see the design notes), not part of this build",
              file=sys.stderr)
        sys.exit(2)
    # 16 hardware queues instead of HIP's default 4, so that the streams of concurrently
    # served requests run side by side (set before the HIP runtime initialises)
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    import torch
    import problems
    torch.cuda.init()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only:
        stream = torch.cuda.current_stream().cuda_stream
        print(json.dumps({"workloads": other_workloads(stream, which=(args.only,))}), flush=True)
        return
    stream = torch.cuda.current_stream().cuda_stream
    prob = problems.rotor(batch=args.batch)
    B = prob.batch
    res = {"fp32": run_gpu("fp32", prob, args.steps, args.warmup, stream)}
    if not args.no_fp64:
        res["fp64"] = run_gpu("fp64", prob, args.steps, args.warmup, stream)
    useful = B * 2 * prob.K * args.steps
    r32 = res["fp32"]
    value = useful / r32["seconds"]
    # roofline of the dominant kernel of the FP32 path (largest total time among the
    # kernels with an algorithmic flop count)
    kt = r32["kernels"]
    flops = algorithmic_flops(prob, r32["info"]["terms"])
    dom = max((k for k in kt if k in flops), key=lambda k: kt[k][1])
    launches, tot_ms = kt[dom]
    achieved = flops.get(dom, 0.0) / (tot_ms / launches * 1e-3) if dom in flops else 0.0
    per_launch = {k: {"launches": v[0], "avg_ms": v[1] / v[0],
                      "algorithmic_TFLOP": flops[k] / 1e12 if k in flops else None}
                  for k, v in kt.items()}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"rotor batch: {B} instances, j<=20 (d=21), K={prob.K}, "
                               f"N={prob.N}, T={prob.T}, one ISM iteration per step",
                   "precision": "FP32 mixed (FP64 generator data, overlaps, boundaries)"},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12,
                     "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_ALU,
                     "traffic": traffic_bytes(dom),
                     "avg_launch_ms": tot_ms / launches,
                     "algorithmic_flop_per_launch": flops.get(dom)},
        "kernels": per_launch,
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "taylor": {"m_max": r32["info"]["taylor_m"], "S_max": r32["info"]["taylor_S"],
                   "terms_mean": sum(r32["info"]["terms"]) / len(r32["info"]["terms"])},
        "final_F_mean": r32["F_mean"],
    }
    if "fp64" in res:
        r64 = res["fp64"]
        out["fp64_plain"] = {
            "value": useful / r64["seconds"], "ms_per_step": r64["seconds"] / args.steps * 1e3,
            "kernels_ms_per_step": {k: v[1] / args.steps for k, v in r64["kernels"].items()},
            "taylor": {"m": r64["info"]["taylor_m"], "S": r64["info"]["taylor_S"]},
            "final_F_mean": r64["F_mean"],
            "fp32_speedup": r64["seconds"] / r32["seconds"],
            "final_F_abs_diff_vs_fp32": abs(r64["F_mean"] - r32["F_mean"])}
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample)
    if not args.no_workloads:
        out["workloads"] = other_workloads(stream)
    if args.serve > 0:
        out["serving"] = serving_sample(args.serve)
        # the same replay with requests in a few standard shapes, which the server merges
        out["serving_standard_shapes"] = serving_sample(args.serve, shapes="standard")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
