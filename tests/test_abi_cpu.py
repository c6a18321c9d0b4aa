"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/psr.h declares, and rejects invalid mechanisms before
any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "psr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2005_11468_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("psr_create_mechanism", "psr_residual", "psr_solve_batch", "psr_jacobian",
                 "psr_lu_factor_batch", "psr_lu_solve_batch", "psr_workspace_bytes",
                 "psr_last_error", "psr_default_opts", "psr_destroy_mechanism",
                 "psr_num_unknowns"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_opts_match_the_oracle(lib):
    from oracle import oracle as O
    import paper_2005_11468_amd as P
    g = P.default_opts()
    o = O.default_opts()
    for name, _ in O.Opts._fields_:
        assert getattr(g, name) == getattr(o, name), name
    assert g.precision == P.PSR_FP64 and g.scheduler == P.PSR_PLAIN


def _desc(mech):
    from paper_2005_11468_amd import _lib
    keep = {k: np.ascontiguousarray(v) for k, v in mech.items() if isinstance(v, np.ndarray)}
    dpp = lambda x: x.astype(np.float64).ctypes.data_as(_lib.dp)
    arrs = dict(ew=np.ascontiguousarray(mech["elem_weight"], np.float64),
                se=np.ascontiguousarray(mech["species_elems"], np.int32),
                nasa=np.ascontiguousarray(mech["nasa7"], np.float64),
                ri=np.ascontiguousarray(mech["reac_idx"], np.int32),
                rn=np.ascontiguousarray(mech["reac_nu"], np.int32),
                pi=np.ascontiguousarray(mech["prod_idx"], np.int32),
                pn=np.ascontiguousarray(mech["prod_nu"], np.int32),
                A=np.ascontiguousarray(mech["A"], np.float64),
                beta=np.ascontiguousarray(mech["beta"], np.float64),
                Ea=np.ascontiguousarray(mech["Ea"], np.float64))
    d = _lib.MechDesc(arrs["se"].shape[1], arrs["se"].shape[0], arrs["ri"].shape[0],
                      arrs["ew"].ctypes.data_as(_lib.dp), arrs["se"].ctypes.data_as(_lib.ip),
                      arrs["nasa"].ctypes.data_as(_lib.dp), 300.0, 3000.0,
                      arrs["ri"].ctypes.data_as(_lib.ip), arrs["rn"].ctypes.data_as(_lib.ip),
                      arrs["pi"].ctypes.data_as(_lib.ip), arrs["pn"].ctypes.data_as(_lib.ip),
                      arrs["A"].ctypes.data_as(_lib.dp), arrs["beta"].ctypes.data_as(_lib.dp),
                      arrs["Ea"].ctypes.data_as(_lib.dp))
    return d, arrs


def _create(lib, mech):
    d, keep = _desc(mech)
    h = C.c_void_p()
    st = lib.psr_create_mechanism(C.byref(d), C.byref(h))
    return st, lib.psr_last_error().decode()


def test_rejects_unbalanced_reaction(lib):
    from tests import tiny_mechs as tm
    m = tm.association()
    m["reac_idx"][0] = [0, -1, -1]  # 2 A -> C: two carbons in, one out, no hydrogen in
    m["reac_nu"][0] = [2, 0, 0]
    st, msg = _create(lib, m)
    assert st == 1 and "balanced" in msg


def test_rejects_species_on_both_sides(lib):
    from tests import tiny_mechs as tm
    m = tm.association()
    m["prod_idx"][0, :2] = [2, 0]
    m["prod_nu"][0, :2] = [1, 1]
    st, msg = _create(lib, m)
    assert st == 1 and "both sides" in msg


def test_rejects_bad_index_and_coefficients(lib):
    from tests import tiny_mechs as tm
    m = tm.association()
    m["reac_idx"][0, 0] = 7
    st, msg = _create(lib, m)
    assert st == 1 and "out of range" in msg
    m = tm.association()
    m["reac_nu"][0, 0] = 0
    st, msg = _create(lib, m)
    assert st == 1 and "coefficient" in msg
    m = tm.association()
    m["A"][0] = -1.0
    st, msg = _create(lib, m)
    assert st == 1 and "Arrhenius" in msg


def test_rejects_null_and_empty(lib):
    h = C.c_void_p()
    assert lib.psr_create_mechanism(None, C.byref(h)) == 1
    from paper_2005_11468_amd import _lib
    o = _lib.SolveOpts()
    lib.psr_default_opts(C.byref(o))
    assert lib.psr_workspace_bytes(None, 0, C.byref(o)) == 0
    assert lib.psr_solve_batch(None, 0, C.byref(o), None, 0, None, None) == 1
    o.precision = 7
    assert lib.psr_solve_batch(None, 0, C.byref(o), None, 0, None, None) == 1


def test_rejects_bad_soot_description(lib):
    """Soot descriptions are validated before anything touches the device:
    the precursor and growth species must be pure carbon and distinct, the
    indices in range, the densities positive."""
    from paper_2005_11468_amd import _lib
    from psr_inputs import SOOT_CONSTANTS, mechanism
    mech = mechanism("soot")
    good = dict(mech["soot"])
    not_carbon = int(np.flatnonzero(mech["species_elems"][:, 1] > 0)[0])  # a species with hydrogen
    cases = [(dict(good, precursor=not_carbon), "pure carbon"),
             (dict(good, growth=good["precursor"]), "coincide"),
             (dict(good, growth=10 ** 6), "out of range"),
             (dict(good, carbon=5), "out of range"),
             (dict(good, soot_density=0.0), "density"),
             (dict(good, A_nuc=float("nan")), "non-finite")]
    for sd, words in cases:
        d, keep = _desc(mech)
        s = _lib.SootDesc(*(sd[k] for k, _ in _lib.SootDesc._fields_))
        d.soot = C.pointer(s)
        h = C.c_void_p()
        st = lib.psr_create_mechanism(C.byref(d), C.byref(h))
        msg = lib.psr_last_error().decode()
        assert st == 1 and words in msg, (sd, msg)
    assert set(SOOT_CONSTANTS) <= set(good)


def test_launch_shape_options_are_validated_on_the_host(lib):
    """rpw outside {0, 1, 2, 4} or grid_per_cu outside 0..32 is rejected
    before any device work, by both the solve and the autotuner."""
    from paper_2005_11468_amd import _lib
    g = (_lib.Group * 1)()
    res = _lib.TuneResult()
    for bad in (dict(rpw=3), dict(rpw=8), dict(grid_per_cu=-1), dict(grid_per_cu=33)):
        o = _lib.SolveOpts()
        lib.psr_default_opts(C.byref(o))
        assert o.rpw == 0 and o.grid_per_cu == 0
        for k, v in bad.items():
            setattr(o, k, v)
        assert lib.psr_solve_batch(g, 1, C.byref(o), None, 0, None, None) == _lib.PSR_EINVAL
        assert lib.psr_autotune(g, 1, C.byref(o), 16, None, C.byref(res), None) == _lib.PSR_EINVAL
        assert b"option out of range" in lib.psr_last_error()
    o = _lib.SolveOpts()
    lib.psr_default_opts(C.byref(o))
    assert lib.psr_autotune(g, 1, C.byref(o), 0, None, C.byref(res), None) == _lib.PSR_EINVAL
    assert b"sample" in lib.psr_last_error()
    assert lib.psr_autotune(g, 0, C.byref(o), 16, None, C.byref(res), None) == _lib.PSR_EINVAL


def test_sweep_arguments_are_validated_on_the_host(lib):
    """psr_sweep_batch rejects a null group, an unknown parameter, fewer
    than one step and null values before any device work."""
    from paper_2005_11468_amd import _lib
    g = (_lib.Group * 1)()
    o = _lib.SolveOpts()
    lib.psr_default_opts(C.byref(o))
    v = (C.c_double * 4)()
    cases = [(None, 0, 1, v, "null group"), (g, 2, 1, v, "parameter"), (g, -1, 1, v, "parameter"),
             (g, 0, 0, v, "n_steps"), (g, 1, 1, None, "null values"), (g, 0, 1, v, "mechanism")]
    for grp, param, steps, vals, words in cases:
        st = lib.psr_sweep_batch(grp, param, steps, C.cast(vals, C.c_void_p) if vals else None,
                                 C.byref(o), None, 0, None, None, None, None)
        assert st == _lib.PSR_EINVAL and words in lib.psr_last_error().decode(), words


def test_fd_jacobian_rejects_null_arguments_on_the_host(lib):
    """psr_jacobian_fd checks the mechanism and conditions before any
    device work: a null mechanism or null conditions is PSR_EINVAL."""
    from paper_2005_11468_amd import _lib
    c = _lib.Conditions()
    for cond in (None, C.byref(c)):
        st = lib.psr_jacobian_fd(None, cond, None, None, None, None)
        assert st == _lib.PSR_EINVAL and "null" in lib.psr_last_error().decode()


def test_soot_outputs_and_energy_mode_are_validated_on_the_host(lib):
    """psr_soot_outputs rejects a null mechanism or buffer; the solve and
    residual calls reject an energy mode outside 0, 1, 2 (checked before any
    device work: a null mechanism is reported first, so the mode is checked
    through the ABI's own argument validation only where no device is
    needed)."""
    from paper_2005_11468_amd import _lib
    buf = (C.c_double * 8)()
    assert lib.psr_soot_outputs(None, 1, C.cast(buf, C.c_void_p), C.cast(buf, C.c_void_p), None) == _lib.PSR_EINVAL
    assert b"null" in lib.psr_last_error()
    import paper_2005_11468_amd as P
    with pytest.raises(ValueError):
        P._energy(3)
    assert [P._energy(e) for e in (False, True, 0, 1, 2)] == [0, 1, 0, 1, 2]
