"""Host-side checks of the C-ABI library: it loads, exports every symbol include/colloc.h
declares, validates arguments on the host, and its own collocation tables agree with the
oracle's (two independent constructions).  No device calls."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2607_12201_amd import colloc, workloads
from oracle.tables import collocation_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "colloc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|size_t|void)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(colloc.LIB_PATH):
        pytest.fail("libcolloc.so is not built; run __graft_entry__.build()")
    return colloc.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(colloc.EXPORTS) == declared


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        colloc._lib_saved = colloc._lib
        try:
            colloc._lib = None
            colloc.load(str(tmp_path / "nope.so"))
        finally:
            colloc._lib = colloc._lib_saved


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_library_tables_match_oracle(lib, K):
    tau, a = colloc.library_tables(K)
    tau_o, a_o, _ = collocation_tables(K, "radau")
    assert np.max(np.abs(tau - tau_o)) < 1e-14
    assert np.max(np.abs(a - a_o)) < 1e-11 * np.max(np.abs(a_o))


def _desc_array(insts):
    keep = []

    def i32(x):
        arr = np.ascontiguousarray(np.asarray(x, np.int32).ravel())
        keep.append(arr)
        return arr.ctypes.data_as(C.POINTER(C.c_int32))

    def f64(x):
        arr = np.ascontiguousarray(np.asarray(x, np.float64).ravel())
        keep.append(arr)
        return arr.ctypes.data_as(C.POINTER(C.c_double))

    ds = (colloc.InstanceDesc * len(insts))()
    for q, inst in enumerate(insts):
        d = ds[q]
        d.n_s, d.n_r, d.n_p, d.N = inst["n_s"], inst["n_r"], inst["n_p"], inst["N"]
        d.react, d.prod, d.param = i32(inst["react"]), i32(inst["prod"]), i32(inst["param"])
        d.logk_fixed, d.h, d.z0 = f64(inst["logk_fixed"]), f64(inst["h"]), f64(inst["z0"])
        d.n_meas = len(inst["meas_y"])
        d.meas_elem, d.meas_species = i32(inst["meas_elem"]), i32(inst["meas_species"])
        d.meas_tau, d.meas_y, d.meas_sigma = f64(inst["meas_tau"]), f64(inst["meas_y"]), f64(inst["meas_sigma"])
        d.theta_lo, d.theta_hi = f64(inst["theta_lo"]), f64(inst["theta_hi"])
    return ds, keep


def _create(lib, insts, K=3):
    ds, keep = _desc_array(insts)
    h = C.c_void_p()
    rc = lib.colloc_create(ds, len(insts), K, C.byref(h))
    return rc, h


def test_create_and_layout(lib):
    insts = workloads.multistart_batch(3, 200, 400)
    rc, h = _create(lib, insts)
    assert rc == 0
    lay = colloc.Layout()
    assert lib.colloc_layout_get(h, C.byref(lay)) == 0
    Ns = [i["N"] for i in insts]
    assert lay.n_inst == 3 and lay.b == 8 and lay.n_elem == sum(Ns)
    assert lay.n_total == sum(N * 8 + 2 for N in Ns) and lay.m_total == sum(N * 8 for N in Ns)
    assert [lay.x_off[q] for q in range(3)] == [0, Ns[0] * 8 + 2, Ns[0] * 8 + 2 + Ns[1] * 8 + 2]
    assert lib.colloc_table_bytes(h) % 256 == 0 and lib.colloc_table_bytes(h) > 0
    w64 = lib.colloc_workspace_bytes(h, colloc.FP64)
    w32 = lib.colloc_workspace_bytes(h, colloc.FP32_IR)
    # FP32_IR keeps room for its per-instance FP64 re-factorization
    assert w64 == w32 > 0
    assert lib.colloc_workspace_bytes(h, 7) == 0
    assert lib.colloc_state_bytes(h) > 0
    sl = colloc.StateLayout()
    assert lib.colloc_state_layout_get(h, C.byref(sl)) == 0
    assert sl.x == 0 and sl.s >= lay.n_total * 8 and sl.info > sl.dx
    assert lib.colloc_destroy(h) == 0


def _bad(inst, **kw):
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in inst.items()}
    out.update(kw)
    return out


@pytest.mark.parametrize("case", ["species", "param", "h", "sigma", "tau", "elem", "bounds",
                                  "shape_mismatch", "K"])
def test_create_rejects_bad_input(lib, case):
    base = workloads.ab_reversible(0)
    K = 3
    if case == "species":
        insts = [_bad(base, react=np.array([[0, -1], [5, -1]], np.int32))]
    elif case == "param":
        insts = [_bad(base, param=np.array([0, 2], np.int32))]
    elif case == "h":
        h = base["h"].copy(); h[3] = 0.0
        insts = [_bad(base, h=h)]
    elif case == "sigma":
        s = base["meas_sigma"].copy(); s[0] = -1.0
        insts = [_bad(base, meas_sigma=s)]
    elif case == "tau":
        t = base["meas_tau"].copy(); t[0] = 1.5
        insts = [_bad(base, meas_tau=t)]
    elif case == "elem":
        e = base["meas_elem"].copy(); e[0] = base["N"]
        insts = [_bad(base, meas_elem=e)]
    elif case == "bounds":
        insts = [_bad(base, theta_hi=base["theta_lo"].copy())]
    elif case == "shape_mismatch":
        insts = [base, workloads.tiny_network(0)]
    else:
        insts, K = [base], 9
    rc, h = _create(lib, insts, K)
    assert rc == colloc.EINVAL
    assert not h.value


def _synthetic(n_s, n_r, N=2, seed=0):
    """A structurally valid instance without simulated data (host validation only)."""
    rng = np.random.default_rng(seed)
    react = rng.integers(-1, n_s, size=(n_r, 2)).astype(np.int32)
    react[:, 0] = rng.integers(0, n_s, size=n_r)
    prod = rng.integers(0, n_s, size=(n_r, 2)).astype(np.int32)
    return dict(n_s=n_s, n_r=n_r, n_p=n_r, N=N, react=react, prod=prod, param=np.arange(n_r, dtype=np.int32),
                logk_fixed=np.zeros(n_r), h=np.full(N, 0.1), z0=np.ones(n_s), meas_elem=np.zeros(1, np.int32),
                meas_species=np.zeros(1, np.int32), meas_tau=np.ones(1), meas_y=np.ones(1),
                meas_sigma=np.ones(1), theta_lo=np.full(n_r, -5.0), theta_hi=np.full(n_r, 5.0))


def test_create_picks_the_tiled_path_for_large_blocks(lib, monkeypatch):
    # 60 species, 60 parameters: 360-row element blocks, beyond the register-resident kernels;
    # accepted (tiled path) unless the register path is demanded
    inst = workloads.random_network(0, n_s=60, n_r=60, N=4, n_obs=2, n_times=2)
    rc, h = _create(lib, [inst])
    assert rc == colloc.OK
    lib.colloc_destroy(h)
    monkeypatch.setenv("COLLOC_FACTOR_PATH", "register")
    rc, h = _create(lib, [inst])
    assert rc == colloc.EUNSUPPORTED


def test_create_reports_unsupported_shapes(lib):
    # 3000 reactions: the line-search trial kernel's per-candidate rate constants exceed LDS
    rc, h = _create(lib, [_synthetic(40, 3000)])
    assert rc == colloc.EUNSUPPORTED


def test_null_handle_calls_are_rejected(lib):
    assert lib.colloc_destroy(None) == colloc.EINVAL
    assert lib.colloc_workspace_bytes(None, 0) == 0
    assert lib.kkt_factor(None, None, 0, None, None) == colloc.EINVAL
    assert lib.ipm_step(None, None, None, None, None) == colloc.EINVAL


def test_status_codes_and_option_defaults():
    """The binding's status codes follow the header's enum (a full filter has its own code), and
    the wall-clock limit defaults to off."""
    assert (colloc.RUNNING, colloc.SOLVED, colloc.TIMEOUT, colloc.ENONFINITE, colloc.EFILTER) == (0, 1, 4, 6, 8)
    o = colloc.default_opts()
    assert o.max_wall_s == 0.0 and o.ir_max == 10 and o.ir_tol == 1e-14
