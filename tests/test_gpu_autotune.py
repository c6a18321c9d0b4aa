"""GPU checks of the launch-shape options (rpw, grid_per_cu) and of the
autotuner psr_autotune, through the C ABI.  The shape of a launch decides
only how reactors are packed onto the GPU; each reactor's arithmetic is the
same, so results must agree bit for bit with the automatic shape."""
import numpy as np
import pytest

from tests.gpu_util import cond_dev, dev, solve_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


@pytest.fixture(scope="module")
def energy():
    from psr_inputs import workload
    return workload("energy", 333)  # ragged against every rpw and the grid


def _same(a, b):
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[0], b[0])


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheduler", [0, 1])
def test_wave_shapes_bitwise(P, energy, precision, scheduler):
    mech, cond, x0, en = energy
    M = P.Mechanism(mech)
    ref = solve_gpu(M, cond, x0, en, precision=precision, scheduler=scheduler, engine=2)
    assert np.mean(ref[1] == 0) > 0.9
    for rpw, grid in ((1, 0), (2, 0), (4, 1), (1, 2), (2, 1)):
        print(f"wave engine rpw={rpw} grid_per_cu={grid}", flush=True)
        got = solve_gpu(M, cond, x0, en, precision=precision, scheduler=scheduler, engine=2,
                        rpw=rpw, grid_per_cu=grid)
        _same(got, ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_block_engine_grid_bitwise(P, energy, precision):
    mech, cond, x0, en = energy
    M = P.Mechanism(mech)
    ref = solve_gpu(M, cond, x0, en, precision=precision, scheduler=P.PSR_PERSISTENT, engine=1)
    assert np.mean(ref[1] == 0) > 0.9
    for grid in (1, 2):
        got = solve_gpu(M, cond, x0, en, precision=precision, scheduler=P.PSR_PERSISTENT,
                        engine=1, grid_per_cu=grid)
        _same(got, ref)


def test_autotune_picks_caches_and_leaves_inputs(P, energy, tmp_path):
    import torch
    mech, cond, x0, en = energy
    M = P.Mechanism(mech)
    B = x0.shape[1]
    x = dev(x0)
    status = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    g = [dict(mech=M, cond=cond_dev(cond), energy=en, x=x, status=status)]
    cache = str(tmp_path / "tune.txt")
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    r = P.autotune(g, o, sample=200, cache_path=cache)
    torch.cuda.synchronize()
    # the caller's arrays are not touched
    np.testing.assert_array_equal(x.cpu().numpy(), x0)
    assert np.all(status.cpu().numpy() == -1)
    assert r.candidates >= 2 and r.ms > 0 and r.solves_per_s > 0 and r.default_ms > 0
    assert (o.engine, o.rpw, o.grid_per_cu) == (r.engine, r.rpw, r.grid_per_cu)
    assert o.engine in (0, 1) and o.rpw in (0, 1, 2, 4) and 0 <= o.grid_per_cu <= 32
    # second call: a cache hit, same choice, nothing timed
    o2 = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT)
    r2 = P.autotune(g, o2, sample=200, cache_path=cache)
    assert r2.candidates == 0
    assert (o2.engine, o2.rpw, o2.grid_per_cu) == (o.engine, o.rpw, o.grid_per_cu)
    assert len(open(cache).read().strip().splitlines()) == 1
    # a solve with the tuned shape equals one with the same engine's automatic shape
    tuned = solve_gpu(M, cond, x0, en, precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT,
                      engine=o.engine, rpw=o.rpw, grid_per_cu=o.grid_per_cu)
    auto = solve_gpu(M, cond, x0, en, precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT,
                     engine=o.engine)
    _same(tuned, auto)
    assert np.mean(tuned[1] == 0) > 0.9


def test_autotune_block_engine_only(P, tmp_path):
    """A mechanism the wavefront engine cannot hold (n > 64): only the grid
    is tuned, and a sample larger than the batch means the whole batch."""
    import torch
    from psr_inputs import uneven_workload
    name, mech, cond, x0 = [w for w in uneven_workload(1.0) if w[0] == "uneven_b"][0]
    idx = np.arange(40)
    cond = {k: np.ascontiguousarray(v[..., idx]) for k, v in cond.items()}
    x0 = np.ascontiguousarray(x0[:, idx])
    M = P.Mechanism(mech)
    x = dev(x0)
    status = torch.full((40,), -1, dtype=torch.int32, device="cuda:0")
    g = [dict(mech=M, cond=cond_dev(cond), energy=True, x=x, status=status)]
    o = P.default_opts(precision=P.PSR_MIXED, scheduler=P.PSR_PERSISTENT, max_lin=60)
    r = P.autotune(g, o, sample=1000)
    assert r.candidates == 3 and o.engine == 0 and o.rpw == 0
    np.testing.assert_array_equal(x.cpu().numpy(), x0)
