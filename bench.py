"""Benchmark: converged PSR reactor-solves per second on one MI355X.

Workload: the 53-species / 325-reaction synthetic mechanism with energy
equation, 16384 reactors (the mixed-precision workload; seeded inputs from
psr_inputs).  One step = one psr_solve_batch call that solves the whole batch
from the same initial guess, with inputs already resident in HBM.

Printed JSON line (one): the mixed-precision persistent solver's rate as
`value`; the plain FP64 host-driven solver and the persistent FP64 solver on
the same inputs beside it, each timed the same way (warm-up, median of
--steps calls, workspace allocated beforehand); parity of every leg against
the oracle on the whole batch (or a seeded sample); a roofline object for the
dominant kernel (the persistent solve kernel); the residual kernel's
throughput on a batch of 1e6 reactors; the batched float LU at n = 201; the
65536-reactor three-mechanism workload and the 8192-reactor sooting workload
with oracle parity on samples; the single-Newton-iteration sweep; the
continuation sweeps; and the oracle's own throughput on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TFLOPS = 78.6   # FP64 vector = non-packed FP32 vector: 256 CU x 64 FMA/clk x 2 x 2.4 GHz
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_F32_TFLOPS = 157.3
EXP_FLOPS = 20.0         # an FP64 exp or log counted as its ~20 vector instructions
TOL = {0: 1e-8, 1: 1e-7}
FTOL = 1e-10             # scaled-residual bound of a converged reactor
PROFILES = os.path.join(ROOT, "profiles")
# Solver options of the 53/325 workload: damped Newton (natural criterion,
# lambda >= 1/16, 8 iterations per attempt), no continuation in tau, Newton
# retried once the pseudo-time step reaches tau.  That workload converges
# fully with them (the oracle: 1024 of 1024 sampled reactors, 66
# linearisations per reactor) against 132 linearisations and 99.4 % with the
# defaults, which the 100- to 201-unknown mechanisms need; the other legs use
# the defaults.
FAST_OPTS = dict(lambda_min=1.0 / 16.0, nw_max_it=8, ct_ratio=0.0, nw_h_ratio=1.0)


def residual_flops(N, I):
    """Algorithmic FP64 flops of one residual evaluation of one reactor: two
    exps per reaction (k_f and k_r), one log, ~19 flops per species (thermo,
    concentrations, residual rows) and ~14 per reaction (rate-constant
    exponent, equilibrium constant, concentration products, production
    rates)."""
    return 2.0 * I * EXP_FLOPS + EXP_FLOPS + 19.0 * N + 14.0 * I


def residual_bytes(N, n):
    """HBM bytes of one residual evaluation: x, Y_in, P, tau, T_in in; F and
    the scaled residual out."""
    return 8.0 * (n + N + 3) + 8.0 * (n + 1)


def jacobian_flops(n, I):
    """Analytic Jacobian: ~54 flops per reaction (rate derivatives and their
    scatter) and 2 n^2 for the density / temperature chain rule."""
    return 54.0 * I + 2.0 * n * n


def solve_flops(n):
    return 2.0 * n * n


def lu_flops(n):
    return 2.0 / 3.0 * n ** 3


def unit_flops(n, N, I):
    """(per linearisation, per round): a linearisation is a Jacobian and an
    LU factorisation, a round a residual and a pair of triangular solves."""
    return jacobian_flops(n, I) + lu_flops(n), residual_flops(N, I) + solve_flops(n)


def src_digest():
    """sha256 of the HIP sources: the profiles' counters hold only for the
    kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_11468_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the PMC summary in
    profiles/ (FETCH_SIZE and WRITE_SIZE passes, scaled by a plain copy of
    known size), or None when there is none for these sources."""
    path = os.path.join(PROFILES, "pmc_traffic.tsv")
    if not os.path.exists(path):
        return None
    digest = src_digest()
    with open(path) as fh:
        for line in fh:
            f = line.rstrip("\n").split("\t")
            if len(f) >= 5 and f[0] == kernel and f[1] == workload and f[2] == digest:
                return float(f[3]) + float(f[4])
    return None


def rate_kernel(P, B, steps=5, name="rate"):
    """psr_residual over B reactors of the 53/325 mechanism ('rate') or the
    200/1200 one ('rate200'), inputs resident in HBM, timed with HIP events on
    the launch stream."""
    import torch
    from psr_inputs import workload
    from tests.gpu_util import cond_dev, dev
    mech, cond, x0, energy = workload(name, B)
    M = P.Mechanism(mech)
    cd = cond_dev(cond)
    xd = dev(x0)
    F = torch.empty_like(xd)
    sc = torch.empty(B, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    P.residual(M, cd, energy, xd, F, sc)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        P.residual(M, cd, energy, xd, F, sc)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    N, I = mech["species_elems"].shape[0], mech["A"].shape[0]
    fl, by = residual_flops(N, I), residual_bytes(N, x0.shape[0])
    tf = fl * B / (ms / 1e3) / 1e12
    gbs = by * B / (ms / 1e3) / 1e9
    ok = bool(torch.isfinite(F).all().item())
    return {"kernel": "k_wresidual" if x0.shape[0] <= 64 else "k_residual",
            "mechanism": f"{N} species / {I} reactions", "reactors": B, "ms_per_launch": ms,
            "reactor_evals_per_s": B / (ms / 1e3), "flops_per_reactor": fl,
            "bytes_per_reactor": by, "achieved_tflops": tf, "peak_tflops": PEAK_ALU_TFLOPS,
            "frac_fp64": tf / PEAK_ALU_TFLOPS, "achieved_gbs": gbs, "peak_gbs": PEAK_HBM_GBS,
            "frac_hbm": gbs / PEAK_HBM_GBS, "finite": ok}


def newton_sweep(P, sizes, steps=3, fd_max=100_000):
    """One Newton iteration per reactor (residual, analytic Jacobian, FP64 LU
    factorisation, triangular solves) on the 101/542 mechanism at the paper's
    single-iteration conditions (isothermal 1800 K, tau = 50 ms, inlet
    0.15/0.18/0.67 fuel/oxidizer/diluent, every reactor alike), at each batch
    size; 'rate_jac' times the residual and Jacobian alone, 'rate_fd_jac' the
    residual and the finite-difference Jacobian (n + 1 residual evaluations,
    the paper's route; batches up to fd_max reactors).  The oracle's
    single-thread rate for the same iteration is measured on 20 reactors."""
    import ctypes as C
    import torch
    from psr_inputs import workload
    from paper_2005_11468_amd import _lib
    mech, cond, x0, energy = workload("newton101", 1)
    M = P.Mechanism(mech)
    N, I = mech["species_elems"].shape[0], mech["A"].shape[0]
    n = x0.shape[0]
    it_fl = residual_flops(N, I) + jacobian_flops(n, I) + lu_flops(n) + solve_flops(n)
    L = _lib.load()
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    out = {"mechanism": f"{N} species / {I} reactions, isothermal 1800 K, tau 50 ms",
           "flops_per_iteration": it_fl, "sizes": []}
    for B in sizes:
        d = "cuda:0"
        cd = {"P": torch.full((B,), float(cond["P"][0]), dtype=torch.float64, device=d),
              "tau": torch.full((B,), float(cond["tau"][0]), dtype=torch.float64, device=d),
              "T_in": torch.full((B,), float(cond["T_in"][0]), dtype=torch.float64, device=d),
              "Y_in": torch.from_numpy(cond["Y_in"]).to(d).expand(N, B).contiguous()}
        x = cd["Y_in"].clone()
        F = torch.empty_like(x)
        J = torch.empty((B, n, n), dtype=torch.float64, device=d)
        piv = torch.empty((B, n), dtype=torch.int32, device=d)
        info = torch.empty((B,), dtype=torch.int32, device=d)
        rhs = torch.empty((B, n), dtype=torch.float64, device=d)

        def rate_jac():
            P.residual(M, cd, energy, x, F, stream=stream)
            P.jacobian(M, cd, energy, x, J, stream=stream)

        def iteration():
            rate_jac()
            _lib.check(L.psr_lu_factor_batch(n, B, P.PSR_FP64, C.c_void_p(J.data_ptr()),
                                             C.c_void_p(piv.data_ptr()), C.c_void_p(info.data_ptr()), sp),
                       "psr_lu_factor_batch")
            torch.neg(F.t(), out=rhs)
            _lib.check(L.psr_lu_solve_batch(n, B, C.c_void_p(J.data_ptr()), C.c_void_p(piv.data_ptr()),
                                            C.c_void_p(rhs.data_ptr()), sp), "psr_lu_solve_batch")

        fd_work = torch.empty((3 * n * B,), dtype=torch.float64, device=d) if B <= fd_max else None

        def rate_fdjac():
            P.residual(M, cd, energy, x, F, stream=stream)
            P.jacobian_fd(M, cd, energy, x, J, work=fd_work, stream=stream)

        legs = [("rate_jac", rate_jac), ("iteration", iteration)]
        if fd_work is not None:
            legs.append(("rate_fd_jac", rate_fdjac))
        row = {"reactors": B}
        for name, fn in legs:
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[name] = {"ms": ms, "reactor_evals_per_s": B / (ms / 1e3)}
        row["iteration"]["achieved_tflops"] = it_fl * B / (row["iteration"]["ms"] / 1e3) / 1e12
        row["nonsingular"] = int((info == 0).sum().item())
        row["finite"] = bool(torch.isfinite(rhs).all().item())
        out["sizes"].append(row)
        print(f"newton101 B={B}: {row['iteration']['ms']:.3f} ms per iteration", file=sys.stderr, flush=True)
        del cd, x, F, J, piv, info, rhs, fd_work
        torch.cuda.empty_cache()
    try:
        from oracle import oracle as O
        om = O.Mechanism(mech)
        args = (cond["P"][0], cond["tau"][0], cond["T_in"][0], cond["Y_in"][:, 0], energy, x0[:, 0])
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            Fo = om.residual(*args)
            Jo = om.jacobian(*args)
            lo, po, io = O.lu_factor(Jo)
            O.lu_solve(lo, po, -Fo)
        t = time.perf_counter() - t0
        out["cpu_oracle"] = {"reactor_evals_per_s": reps / t, "cores": 1, "kind": "oracle",
                             "sample": f"{reps} reactor-iterations, single-threaded FP64 C oracle"}
    except Exception as e:  # the oracle is a reported baseline only
        out["cpu_oracle"] = {"error": str(e)}
    return out


def lu_large(P, n=201, B=9830, steps=3):
    """psr_lu_factor_batch with float factors on B seeded random n x n
    matrices (the 200/1200 mechanism's matrix size and reactor count of the
    uneven workload): one wavefront per matrix, register panel, trailing
    updates on the FP32 matrix cores; each timed launch factors a fresh copy
    (the copy is outside the events)."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(2011)
    A0 = torch.randn((B, n, n), dtype=torch.float64, device="cuda:0", generator=g)
    A = torch.empty_like(A0)
    piv = torch.empty((B, n), dtype=torch.int32, device="cuda:0")
    info = torch.empty((B,), dtype=torch.int32, device="cuda:0")
    import ctypes as C
    from paper_2005_11468_amd import _lib
    L = _lib.load()
    stream = torch.cuda.current_stream()
    total = 0.0
    for it in range(steps + 1):
        A.copy_(A0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _lib.check(L.psr_lu_factor_batch(n, B, P.PSR_MIXED, C.c_void_p(A.data_ptr()), C.c_void_p(piv.data_ptr()),
                                         C.c_void_p(info.data_ptr()), C.c_void_p(stream.cuda_stream)),
                   "psr_lu_factor_batch")
        e1.record(stream)
        torch.cuda.synchronize()
        if it > 0:
            total += e0.elapsed_time(e1)
    ms = total / steps
    flops = 2.0 / 3.0 * n ** 3 * B
    tf = flops / (ms / 1e3) / 1e12
    ok = int((info == 0).sum().item())
    del A0, A
    return {"kernel": "k_lu_factor_wave", "n": n, "matrices": B, "ms_per_launch": ms,
            "alg_flops": flops, "achieved_tflops": tf, "peak_tflops": PEAK_MFMA_F32_TFLOPS,
            "frac_mfma_f32": tf / PEAK_MFMA_F32_TFLOPS, "nonsingular": ok}


def timed_solves(P, groups, x0s, opts, steps, warmup, ws=None):
    """Time psr_solve_batch over `groups` (x reset to x0s before each call,
    outside the timed interval): `warmup` untimed calls, then `steps` calls,
    each bracketed by HIP events on the launching stream.  The workspace is
    allocated once, before the timed calls.  Returns (median ms, all ms,
    stats of the last call, workspace)."""
    import torch
    stream = torch.cuda.current_stream()
    st = None
    for _ in range(max(1, warmup)):
        for g, x0 in zip(groups, x0s):
            g["x"].copy_(x0)
        st, ws = P.solve_batch(groups, opts, workspace=ws, stats=True)
    times = []
    for _ in range(steps):
        for g, x0 in zip(groups, x0s):
            g["x"].copy_(x0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st, ws = P.solve_batch(groups, opts, workspace=ws, stats=True)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), times, st, ws


def oracle_parity(O, mech, cond, energy, idx, x, status, xo, so, tol, opts=None):
    """Per-reactor parity of GPU results on the oracle sample idx (the same
    reading as the tests): agree within tol; a GPU-only root within tol of
    the oracle's last iterate is the same state (the oracle reached it but
    its convergence test failed by rounding); any other branch mismatch or
    GPU-only root is verified by an oracle restart at the GPU root: it
    converges, either with its first linear solve (the oracle's own
    convergence test accepts the GPU root; trace species may then differ by
    up to the step-norm weight atol_Y + rtol |Y|) or to within tol of the GPU
    root; oracle-only roots counted as misses.  Returns counts and the
    fraction of the GPU-converged sample reactors that are verified steady
    states."""
    from tests.gpu_util import rel_err
    n_sp = mech["species_elems"].shape[0]
    xg, sg = x[:, idx], status[idx]
    conv_o, conv_g = so["status"] == 0, sg == 0
    both = conv_o & conv_g
    err = rel_err(xg, xo, n_sp)
    agree = both & (err <= tol)
    om = O.Mechanism(mech)
    opts = O.default_opts(**(opts or {}))
    verified, unverified, same_state = 0, 0, 0
    for j in np.flatnonzero(conv_g & ~agree):
        b = int(idx[j])
        if not conv_o[j] and err[j] <= tol:
            same_state += 1
            continue
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], energy)
        xr, st = om.solve(*args, xg[:, j], opts)
        e = rel_err(xg[:, j:j + 1], xr[:, None], n_sp)[0]
        ok = st.status == 0 and (st.n_lin <= 1 or e <= tol)
        verified += int(ok)
        unverified += int(not ok)
        if not ok:
            print(f"unverified GPU root: reactor {b}, oracle restart status {st.status}, "
                  f"{st.n_lin} linear solves, rel err {e:.2e}", file=sys.stderr, flush=True)
    ng = int(conv_g.sum())
    return {"sample": int(len(idx)), "oracle_converged": int(conv_o.sum()), "gpu_converged": ng,
            "agree": int(agree.sum()), "max_rel_err": float(err[agree].max()) if agree.any() else None,
            "branch_mismatch": int((both & ~agree).sum()), "gpu_only": int((conv_g & ~conv_o).sum()),
            "verified_other_roots": verified, "unverified": unverified,
            "gpu_only_at_oracle_state": same_state,
            "oracle_only": int((conv_o & ~conv_g).sum()),
            "valid_fraction": (int(agree.sum()) + verified + same_state) / ng if ng else 0.0}


def cpu_cores():
    """Host cores this process may use, at most 16 (the GPU machine's CPU share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def uneven(P, steps=1, warmup=1, sample=64, cores=16):
    """The three-mechanism workload: 65536 reactors (30/200, 100/600, 200/1200
    species / reactions, 32768 / 22938 / 9830) in one mixed-precision
    persistent psr_solve_batch call, which runs as one fused launch over one
    device queue (longest residence time first, largest n first); oracle
    parity on a seeded sample of each group over its whole residence-time
    range."""
    import torch
    from psr_inputs import uneven_workload
    from tests.gpu_util import cond_dev, dev
    gl, names, x0s, host = [], [], [], []
    for name, mech, cond, x0 in uneven_workload(1.0):
        B = x0.shape[1]
        gl.append(dict(mech=P.Mechanism(mech), cond=cond_dev(cond), energy=True, x=dev(x0),
                       status=torch.empty(B, dtype=torch.int32, device="cuda:0"),
                       n_lin=torch.empty(B, dtype=torch.int32, device="cuda:0")))
        names.append(f"{mech['species_elems'].shape[0]}/{mech['A'].shape[0]}")
        x0s.append(dev(x0))
        host.append((mech, cond, x0))
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    ms, times, st, ws = timed_solves(P, gl, x0s, o, steps, warmup)
    print(f"uneven: {st.converged}/{st.reactors} converged, {ms:.1f} ms", file=sys.stderr, flush=True)
    out = {"reactors": int(st.reactors), "converged": int(st.converged), "ms_per_solve": ms,
           "ms_all": times, "kernel_ms": st.kernel_ms, "lin_total": int(st.lin_total),
           "jac_total": int(st.jac_total), "fp64_fallbacks": int(st.fp64_fallbacks), "groups": {}}
    valid = 0.0
    for nm, g, (mech, cond, x0) in zip(names, gl, host):
        x = g["x"].cpu().numpy()
        status = g["status"].cpu().numpy()
        conv = int((status == 0).sum())
        row = {"reactors": int(x.shape[1]), "converged": conv}
        if sample > 0:
            from oracle import oracle as O
            idx = np.sort(np.random.default_rng(2025).choice(x.shape[1], sample, replace=False))
            t0 = time.perf_counter()
            xo, so = O.solve_batch(mech, cond, x0, True, idx=idx, processes=cores)
            row["parity"] = oracle_parity(O, mech, cond, True, idx, x, status, xo, so, TOL[1])
            row["parity"]["oracle_s"] = time.perf_counter() - t0
            valid += conv * row["parity"]["valid_fraction"]
            print(f"uneven {nm}: parity {row['parity']}", file=sys.stderr, flush=True)
        else:
            valid += conv
        out["groups"][nm] = row
    out["valid_converged_per_s"] = valid / (ms / 1e3)
    return out


def soot(P, steps=1, warmup=1, sample=32, cores=16):
    """The sooting workload (150 species / 900 reactions + 6 soot moments,
    n = 157, fuel-rich inlet), all 8192 reactors, mixed-precision persistent
    solve; oracle parity on a seeded sample."""
    import torch
    from psr_inputs import workload
    from tests.gpu_util import cond_dev, dev
    mech, cond, x0, _ = workload("soot")
    B = x0.shape[1]
    M = P.Mechanism(mech)
    cd, x0d = cond_dev(cond), dev(x0)
    g = dict(mech=M, cond=cd, energy=True, x=x0d.clone(),
             status=torch.empty(B, dtype=torch.int32, device="cuda:0"),
             n_lin=torch.empty(B, dtype=torch.int32, device="cuda:0"))
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    ms, times, st, ws = timed_solves(P, [g], [x0d], o, steps, warmup)
    print(f"soot: {st.converged}/{B} converged, {ms:.1f} ms", file=sys.stderr, flush=True)
    out = {"reactors": B, "n": int(x0.shape[0]), "converged": int(st.converged), "ms_per_solve": ms,
           "ms_all": times, "kernel_ms": st.kernel_ms, "lin_total": int(st.lin_total),
           "jac_total": int(st.jac_total), "fp64_fallbacks": int(st.fp64_fallbacks)}
    # the workgroup engine's own roofline line: the same per-unit counts as
    # the headline (LU + Jacobian per linearisation, residual + solve per
    # round), over the persistent kernel's duration
    N, I, n = mech["species_elems"].shape[0], mech["A"].shape[0], int(x0.shape[0])
    fl = st.jac_total * (lu_flops(n) + jacobian_flops(n, I)) + st.lin_total * (residual_flops(N, I) + solve_flops(n))
    tf = fl / (st.kernel_ms / 1e3) / 1e12
    out["roofline"] = {"kernel": "k_persistent<true,true>", "bound": "alu", "alg_flops": fl, "achieved": tf,
                       "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_ALU_TFLOPS}
    valid = float(st.converged)
    if sample > 0:
        from oracle import oracle as O
        x = g["x"].cpu().numpy()
        status = g["status"].cpu().numpy()
        idx = np.sort(np.random.default_rng(2026).choice(B, sample, replace=False))
        t0 = time.perf_counter()
        xo, so = O.solve_batch(mech, cond, x0, True, idx=idx, processes=cores)
        out["parity"] = oracle_parity(O, mech, cond, True, idx, x, status, xo, so, TOL[1])
        out["parity"]["oracle_s"] = time.perf_counter() - t0
        valid *= out["parity"]["valid_fraction"]
        print(f"soot: parity {out['parity']}", file=sys.stderr, flush=True)
    out["valid_converged_per_s"] = valid / (ms / 1e3)
    return out


def continuation(P, chains=4096):
    """The paper's continuation protocol (temperature 1500 -> 2000 K at 5 ms,
    then residence time 5 -> 95 ms at 1750 K, each step warm-started from the
    one before) on isothermal reactors of the 53-species mechanism, every
    reactor its own chain: mixed-precision persistent psr_sweep_batch."""
    import torch
    from psr_inputs.configs import sweep_workload
    from tests.gpu_util import cond_dev, dev
    out = {"chains": chains}
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    for param in ("T_in", "tau"):
        mech, cond, x0, values = sweep_workload(param, chains)
        M = P.Mechanism(mech)
        x0d, vd = dev(x0), dev(values)
        g = dict(mech=M, cond=cond_dev(cond), energy=False, x=x0d.clone(),
                 status=torch.empty(chains, dtype=torch.int32, device="cuda:0"))
        _, xp, sp, ws = P.sweep_batch(g, param, vd, o)  # warm-up (same inputs)
        g["x"].copy_(x0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, xp, sp, _ = P.sweep_batch(g, param, vd, o, workspace=ws, x_path=xp, status_path=sp)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[param] = {"steps": int(values.shape[0]), "converged": int(st.converged),
                      "reactor_solves": int(st.reactors), "kernel_ms": st.kernel_ms, "wall_ms": wall * 1e3,
                      "converged_per_s": st.converged / wall}
        print(f"sweep {param}: {st.converged}/{st.reactors} converged in {wall * 1e3:.1f} ms",
              file=sys.stderr, flush=True)
    return out


def soot_sweeps(P, chains=256):
    """The Section 5 sweeps on sooting reactors at a prescribed temperature
    (energy mode 2; 150/900 soot mechanism, chain 0 at equivalence ratio
    2.5): temperature 1500 -> 2000 K at 5 ms and residence time 5 -> 95 ms at
    1750 K, mixed-precision persistent psr_sweep_batch, then psr_soot_outputs
    along each path; reports throughput and chain 0's soot volume fraction
    (ppm), number density (cm^-3) and diameter (nm) per step (Figs. 1-2)."""
    import torch
    from psr_inputs.configs import FIXED_T, soot_sweep_workload
    from tests.gpu_util import cond_dev, dev
    out = {"chains": chains}
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    for param in ("T_in", "tau"):
        mech, cond, x0, values = soot_sweep_workload(param, chains)
        M = P.Mechanism(mech)
        x0d, vd = dev(x0), dev(values)
        g = dict(mech=M, cond=cond_dev(cond), energy=FIXED_T, x=x0d.clone(),
                 status=torch.empty(chains, dtype=torch.int32, device="cuda:0"))
        _, xp, sp, ws = P.sweep_batch(g, param, vd, o)  # warm-up (same inputs)
        g["x"].copy_(x0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, xp, sp, _ = P.sweep_batch(g, param, vd, o, workspace=ws, x_path=xp, status_path=sp)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        soot0 = torch.stack([P.soot_outputs(M, xp[k])[:, 0] for k in range(values.shape[0])]).cpu().numpy()
        out[param] = {"steps": int(values.shape[0]), "converged": int(st.converged),
                      "reactor_solves": int(st.reactors), "wall_ms": wall * 1e3,
                      "converged_per_s": st.converged / wall,
                      "chain0": {"values": values[:, 0].tolist(), "status": sp[:, 0].cpu().numpy().tolist(),
                                 "f_v_ppm": (soot0[:, 0] * 1e6).tolist(), "N_per_cm3": soot0[:, 1].tolist(),
                                 "d_nm": (soot0[:, 2] * 1e7).tolist()}}
        print(f"soot sweep {param}: {st.converged}/{st.reactors} converged in {wall * 1e3:.1f} ms",
              file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="reactors for the oracle baseline (0: the whole batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lu-large", action="store_true")
    ap.add_argument("--uneven-sample", type=int, default=48,
                    help="oracle parity sample per group of the 65536-reactor workload (-1: skip the leg)")
    ap.add_argument("--soot-sample", type=int, default=32,
                    help="oracle parity sample of the 8192-reactor sooting workload (-1: skip the leg)")
    ap.add_argument("--soot-sweep-chains", type=int, default=256,
                    help="chains of the sooting sweeps at a prescribed temperature (0: skip)")
    ap.add_argument("--sweep-chains", type=int, default=4096,
                    help="chains of the continuation sweeps (0: skip)")
    ap.add_argument("--newton-sizes", default="100,1000,10000,100000,1000000",
                    help="batch sizes of the one-Newton-iteration sweep, comma separated ('' or 0: skip)")
    ap.add_argument("--tune-sample", type=int, default=4096,
                    help="reactors the autotuner times each launch shape on (0: automatic shape)")
    ap.add_argument("--rate-reactors", type=int, default=1_000_000,
                    help="batch size of the residual-kernel measurement (0: skip)")
    ap.add_argument("--only-legs", action="store_true",
                    help="profiling runs: skip the headline solver legs and the oracle, print only "
                         "the other legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2005_11468_amd as P
    from psr_inputs import workload
    from tests.gpu_util import cond_dev, dev

    if args.only_legs:
        out = {"rate_kernel": rate_kernel(P, args.rate_reactors) if args.rate_reactors > 0 else None,
               "lu_large": lu_large(P) if not args.no_lu_large else None}
        print(json.dumps(out))
        return

    mech, cond, x0, energy = workload(args.workload)
    B = x0.shape[1]
    N = mech["species_elems"].shape[0]
    n = x0.shape[0]
    I = mech["A"].shape[0]
    M = P.Mechanism(mech)
    cd = cond_dev(cond)
    x0d = dev(x0)
    group = [dict(mech=M, cond=cd, energy=energy, x=x0d.clone(),
                  status=torch.empty(B, dtype=torch.int32, device="cuda:0"),
                  n_lin=torch.empty(B, dtype=torch.int32, device="cuda:0"))]
    cores = cpu_cores()

    mixed = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT, **FAST_OPTS)
    tune = None
    if args.tune_sample > 0:
        # launch shape picked by the autotuner on a prefix of the batch (setup,
        # outside the timed region)
        t0 = time.perf_counter()
        r = P.autotune(group, mixed, sample=args.tune_sample)
        tune = {"engine": r.engine, "rpw": r.rpw, "grid_per_cu": r.grid_per_cu,
                "candidates": r.candidates, "sample": min(args.tune_sample, B),
                "sample_ms": r.ms, "default_shape_sample_ms": r.default_ms,
                "tuning_s": time.perf_counter() - t0}

    # every solver leg timed the same way: warm-up, then the median of
    # `steps` calls, workspace allocated before the timed calls
    legs = {}
    for name, opts in (("mixed_persistent", mixed),
                       ("fp64_plain", P.default_opts(precision=P.PSR_FP64, scheduler=P.PSR_PLAIN, **FAST_OPTS)),
                       ("fp64_persistent", P.default_opts(precision=P.PSR_FP64, scheduler=P.PSR_PERSISTENT,
                                                          **FAST_OPTS))):
        ms, times, st, _ = timed_solves(P, group, [x0d], opts, args.steps, args.warmup)
        legs[name] = {"ms": ms, "ms_all": times, "st": st, "x": group[0]["x"].cpu().numpy(),
                      "status": group[0]["status"].cpu().numpy()}
        print(f"{name}: {st.converged}/{B} converged, median {ms:.2f} ms", file=sys.stderr, flush=True)

    # oracle on the workload (the CPU baseline, and the parity reference of
    # every timed leg)
    cpu = None
    parity = {}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        S = args.cpu_sample or B
        idx = np.sort(np.random.default_rng(2024).choice(B, S, replace=False)) if S < B else np.arange(B)
        t0 = time.perf_counter()
        xo, so = O.solve_batch(mech, cond, x0, energy, idx=idx, processes=cores,
                               opts=O.default_opts(**FAST_OPTS))
        tcpu = time.perf_counter() - t0
        conv_o = int((so["status"] == 0).sum())
        cpu = {"value": conv_o / tcpu, "unit": "reactor-solves/s", "cores": cores, "kind": "oracle",
               "nproc": os.cpu_count(), "cpu_model": cpu_model(),
               "per_core": conv_o / tcpu / cores,
               "sample": f"{S} of {B} reactors, single-threaded FP64 C oracle (gcc -O2), one process "
                         f"per core over a round-robin split, {tcpu:.1f} s wall"}
        for name, leg in legs.items():
            tol = TOL[1] if name.startswith("mixed") else TOL[0]
            parity[name] = oracle_parity(O, mech, cond, energy, idx, leg["x"], leg["status"], xo, so, tol,
                                         FAST_OPTS)
            print(f"parity {name}: {parity[name]}", file=sys.stderr, flush=True)

    def rate_of(name):
        leg = legs[name]
        conv = int((leg["status"] == 0).sum())
        frac = parity[name]["valid_fraction"] if name in parity else 1.0
        return conv * frac / (leg["ms"] / 1e3)

    value = rate_of("mixed_persistent")
    value_plain = rate_of("fp64_plain")
    value_fp64p = rate_of("fp64_persistent")

    rate = rate200 = None
    if args.rate_reactors > 0:
        rate = rate_kernel(P, args.rate_reactors)
        rate200 = rate_kernel(P, args.rate_reactors, name="rate200")
    lu_big = lu_large(P) if not args.no_lu_large else None
    unev = uneven(P, sample=args.uneven_sample, cores=cores) if args.uneven_sample >= 0 else None
    soot_leg = soot(P, sample=args.soot_sample, cores=cores) if args.soot_sample >= 0 else None
    sizes = [int(v) for v in args.newton_sizes.split(",") if v.strip() and int(v) > 0]
    newton = newton_sweep(P, sizes) if sizes else None
    sweep_leg = continuation(P, args.sweep_chains) if args.sweep_chains > 0 else None
    soot_sweep_leg = soot_sweeps(P, args.soot_sweep_chains) if args.soot_sweep_chains > 0 else None

    # roofline of the dominant kernel (the persistent solve kernel): the
    # solver's own counts of linearisations and rounds times the algorithmic
    # flops of each, over the kernel time from the library's HIP events on
    # the launching stream
    st_m = legs["mixed_persistent"]["st"]
    lin_f, rnd_f = unit_flops(n, N, I)
    flops = st_m.jac_total * lin_f + st_m.lin_total * rnd_f
    achieved = flops / (st_m.kernel_ms / 1e3) / 1e12
    kname = "k_wpersist<64,true>" if n <= 64 else "k_persistent<true,false>"
    traffic = measured_traffic(kname, f"{args.workload}:{B}")
    out = {
        "metric": "converged PSR solves/sec (1 GPU), mixed-prec batched vs plain FP64, rel err<=1e-7",
        "value": value, "unit": "reactor-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": legs["mixed_persistent"]["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "mixed: 53 species / 325 reactions + energy, 16384 reactors",
                   "reactors": B, "species": N, "reactions": I, "unknowns": n,
                   "precision": "mixed (FP32 LU + FP64 refinement, FP64 residual)",
                   "scheduler": "persistent work queue", "launch_shape": tune,
                   "solver_options": FAST_OPTS},
        "fp64_plain": {"value": value_plain, "ms_per_step": legs["fp64_plain"]["ms"],
                       "ms_all": legs["fp64_plain"]["ms_all"],
                       "converged": int((legs["fp64_plain"]["status"] == 0).sum()),
                       "rounds": legs["fp64_plain"]["st"].rounds,
                       "speedup_mixed_over_plain": value / value_plain if value_plain else None},
        "fp64_persistent": {"value": value_fp64p, "ms_per_step": legs["fp64_persistent"]["ms"],
                            "ms_all": legs["fp64_persistent"]["ms_all"],
                            "converged": int((legs["fp64_persistent"]["status"] == 0).sum()),
                            "speedup_mixed_over_fp64_persistent": value / value_fp64p if value_fp64p else None},
        "solver": {"converged": int((legs["mixed_persistent"]["status"] == 0).sum()), "reactors": B,
                   "ms_all": legs["mixed_persistent"]["ms_all"],
                   "lin_total": st_m.lin_total, "lin_max": st_m.lin_max, "jac_total": st_m.jac_total,
                   "fp64_fallbacks": st_m.fp64_fallbacks},
        "roofline": {"kernel": kname, "bound": "alu", "achieved": achieved,
                     "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": traffic, "kernel_ms": st_m.kernel_ms, "alg_flops": flops,
                     "flops_per_linearisation": lin_f, "flops_per_round": rnd_f,
                     "linearisations": int(st_m.jac_total), "rounds": int(st_m.lin_total)},
        "rate_kernel": rate,
        "rate_kernel_200sp": rate200,
        "lu_large": lu_big,
        "uneven": unev,
        "soot": soot_leg,
        "newton101": newton,
        "continuation": sweep_leg,
        "soot_sweeps": soot_sweep_leg,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
