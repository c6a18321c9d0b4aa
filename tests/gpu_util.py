"""Helpers shared by the GPU tests: device copies of seeded inputs and the
parity metric (max relative error with a floor for trace mass fractions)."""
import numpy as np

FLOOR_Y = 1e-20


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def cond_dev(cond):
    return {k: dev(np.asarray(v, dtype=np.float64)) for k, v in cond.items()}


def rel_err(a, b, n_species, floor=FLOOR_Y):
    """max over components of |a - b| / max(|b|, floor) (floor on species
    only); soot rows (ln M_r, after the temperature row) compare M_r = exp(ln M_r)
    relatively: |exp(a - b) - 1|."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    m = n_species + 1
    den = np.abs(b[:m]).copy()
    den[:n_species] = np.maximum(den[:n_species], floor)
    e = np.abs(a[:m] - b[:m]) / den
    if a.shape[0] > m:
        e = np.concatenate([e, np.abs(np.expm1(a[m:] - b[m:]))], axis=0)
    return np.max(e, axis=0)


def solve_gpu(mech_obj, cond, x0, energy, **opts):
    import torch
    import paper_2005_11468_amd as P
    B = x0.shape[1]
    x = dev(x0)
    status = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    nlin = torch.zeros((B,), dtype=torch.int32, device="cuda:0")
    o = P.default_opts(**opts)
    st, _ = P.solve_batch([dict(mech=mech_obj, cond=cond_dev(cond), energy=energy, x=x,
                                status=status, n_lin=nlin)], o)
    torch.cuda.synchronize()
    return x.cpu().numpy(), status.cpu().numpy(), nlin.cpu().numpy(), st


def parity(oracle_mod, mech, cond, energy, x, status, xo, so, tol, *, max_branch_frac=0.02,
           max_miss_frac=0.0, label=""):
    """Per-reactor parity of GPU results x, status against the oracle's xo, so
    (same initial guesses).

    Several steady states can be correct for one reactor (a non-isothermal
    PSR can have an ignited and an extinguished branch), and which one the
    hybrid method reaches can turn on rounding at a decision point (a Newton
    attempt converging in its last allowed iteration on one side only).  So:
      * reactors both sides converged either agree within `tol` (relative,
        rel_err), or form a branch mismatch;
      * every GPU root that is not within `tol` of an oracle root (branch
        mismatches, reactors only the GPU converged) must be a steady state
        by the oracle's own solve: the oracle, restarted at the GPU root,
        converges, either with its first linear solve (its own convergence
        test accepts the GPU root as it is; a trace species may then differ
        from the oracle's root by up to its step-norm weight atol_Y + rtol
        |Y|) or to within `tol` of the GPU root (on the stiffest reactors the
        scaled residual's rounding floor sits near the 1e-10 bound and the
        restart takes more Newton steps);
      * a reactor only the GPU converged whose state is within `tol` of the
        oracle's last iterate is the same state: the oracle reached it but
        did not pass its convergence test (on the sooting sweeps at 1900 K
        and above, Jacobians with condition numbers near 1e60 leave species
        below atol_Y determined only to atol_Y, and the final full Newton
        step can leave such a species' row off balance, which the test then
        sees or not by rounding);
      * branch mismatches may be at most max_branch_frac of the jointly
        converged reactors (at least one allowed), and reactors only the
        oracle converged at most max_miss_frac of the oracle-converged ones
        (at least one when max_miss_frac > 0; none when it is 0).
    Returns the counts (and prints them)."""
    n_sp = mech["species_elems"].shape[0]
    conv_o, conv_g = so["status"] == 0, status == 0
    both = conv_o & conv_g
    assert np.all(status >= 0), label
    err = rel_err(x, xo, n_sp) if x.shape[1] else np.zeros(0)
    agree = both & (err <= tol)
    branch = np.flatnonzero(both & ~agree)
    gpu_only = np.flatnonzero(conv_g & ~conv_o)
    miss = np.flatnonzero(conv_o & ~conv_g)
    O = oracle_mod.Mechanism(mech)
    opts = oracle_mod.default_opts()
    same_state = 0
    for b in np.concatenate([branch, gpu_only]).astype(int):
        if not conv_o[b] and err[b] <= tol:
            # the oracle ended at the GPU's root (within tol) without passing
            # its own convergence test
            same_state += 1
            continue
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], energy)
        xr, st = O.solve(*args, x[:, b], opts)
        assert st.status == 0, (label, "GPU root not verified", int(b), st.status, st.n_lin)
        e = rel_err(x[:, b:b + 1], xr[:, None], n_sp)[0]
        assert st.n_lin <= 1 or e <= tol, (label, "oracle restart moved", int(b), e)
    nb = int(both.sum())
    assert len(branch) <= max(1, int(max_branch_frac * nb)), (label, "branch mismatches", branch)
    allowed = max(1, int(max_miss_frac * conv_o.sum())) if max_miss_frac > 0 else 0
    assert len(miss) <= allowed, (label, "oracle-only roots", miss)
    out = dict(reactors=int(len(status)), oracle=int(conv_o.sum()), gpu=int(conv_g.sum()),
               agree=int(agree.sum()), branch=len(branch), gpu_only=len(gpu_only), miss=len(miss),
               gpu_only_at_oracle_state=same_state,
               max_err=float(err[agree].max()) if agree.any() else 0.0)
    print(f"{label}: {out}", flush=True)
    return out
