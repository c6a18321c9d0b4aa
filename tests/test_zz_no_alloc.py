"""The allocation-free finite-difference Jacobian (psr_jacobian_fd_noalloc),
called through the C ABI: its Jacobians equal those of psr_jacobian_fd with a
caller-owned work buffer, bit for bit (same kernels), on two calls in a row
with the second batch smaller than the first; a batch whose work arrays
exceed the static scratch is rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_fd(L, M, cond_c, x, J, work, stream):
    return L.psr_jacobian_fd(M.handle, C.byref(cond_c), C.c_void_p(x.data_ptr()), C.c_void_p(J.data_ptr()),
                             C.c_void_p(work.data_ptr()), stream)


def _call_noalloc(L, M, cond_c, x, J, stream):
    return L.psr_jacobian_fd_noalloc(M.handle, C.byref(cond_c), C.c_void_p(x.data_ptr()),
                                     C.c_void_p(J.data_ptr()), stream)


def _inputs(B):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", B)
    # half the reactors at a perturbed state, half at the inlet guess
    rng = np.random.default_rng(B)
    x = x0.copy()
    N = mech["species_elems"].shape[0]
    x[:N, ::2] = rng.dirichlet(np.ones(N), x[:, ::2].shape[1]).T
    x[N, ::2] = rng.uniform(1200.0, 2200.0, x[:, ::2].shape[1])
    return mech, cond, x, energy


def test_noalloc_fd_jacobian_matches_caller_work():
    import torch
    import paper_2005_11468_amd as P
    from paper_2005_11468_amd import _lib
    from tests.gpu_util import cond_dev, dev
    assert torch.cuda.is_available()
    L = _lib.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for B in (300, 37):  # the second call smaller than the first
        mech, cond, x0, energy = _inputs(B)
        M = P.Mechanism(mech)
        n = M.n_unknowns(energy)
        cd = cond_dev(cond)
        cond_c = P._conditions(cd, energy)
        x = dev(x0)
        J_ref = torch.empty((B, n, n), dtype=torch.float64, device="cuda:0")
        work = torch.empty((3 * n * B,), dtype=torch.float64, device="cuda:0")
        print(f"psr_jacobian_fd vs psr_jacobian_fd_noalloc: B={B} n={n}", flush=True)
        assert _call_fd(L, M, cond_c, x, J_ref, work, stream) == 0, L.psr_last_error()
        J = torch.full((B, n, n), float("nan"), dtype=torch.float64, device="cuda:0")
        assert _call_noalloc(L, M, cond_c, x, J, stream) == 0, L.psr_last_error()
        torch.cuda.synchronize()
        a, b = J.cpu().numpy(), J_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), np.argwhere(a != b)[:4]


def test_noalloc_fd_jacobian_rejects_batches_beyond_the_scratch():
    import torch
    import paper_2005_11468_amd as P
    from paper_2005_11468_amd import _lib
    L = _lib.load()
    mech, cond, x0, energy = _inputs(8)
    M = P.Mechanism(mech)
    n = M.n_unknowns(energy)
    B = (4 << 20) // (3 * n) + 1  # 3 n B just above the scratch
    d = "cuda:0"
    cd = {"P": torch.full((B,), 101325.0, dtype=torch.float64, device=d),
          "tau": torch.full((B,), 1e-3, dtype=torch.float64, device=d),
          "T_in": torch.full((B,), 500.0, dtype=torch.float64, device=d),
          "Y_in": torch.zeros((M.n_species, B), dtype=torch.float64, device=d)}
    cond_c = P._conditions(cd, energy)
    x = torch.zeros((n, B), dtype=torch.float64, device=d)
    J = torch.empty((1,), dtype=torch.float64, device=d)  # never written: the call fails first
    r = L.psr_jacobian_fd_noalloc(M.handle, C.byref(cond_c), C.c_void_p(x.data_ptr()), C.c_void_p(J.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert r == _lib.PSR_EINVAL
    assert b"scratch" in L.psr_last_error()
