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
