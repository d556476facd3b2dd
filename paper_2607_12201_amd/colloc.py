"""Thin ctypes binding of libcolloc (include/colloc.h).  Argument marshalling only: every step
of the computation runs in the library's HIP kernels.  Device buffers are torch CUDA tensors
(memory and streams only).  There is no fallback: a missing library raises at load time."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcolloc.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
RUNNING, SOLVED, ACCEPTABLE, MAXITER, TIMEOUT, ENOTPD, ENONFINITE, RESTORATION_REQUIRED, EFILTER = range(9)
STATUS_NAMES = {RUNNING: "running", SOLVED: "solved", ACCEPTABLE: "acceptable", MAXITER: "maxiter",
                TIMEOUT: "timeout", ENOTPD: "enotpd", ENONFINITE: "enonfinite",
                RESTORATION_REQUIRED: "restoration_required", EFILTER: "efilter"}
FP64, FP32_IR = 0, 1
PHASES = ("eval", "level0", "cr", "border", "solve", "step", "linesearch", "assembly", "schur")
MAX_LS = 48
FILTER_CAP = 128

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class InstanceDesc(C.Structure):
    _fields_ = [
        ("n_s", C.c_int32), ("n_r", C.c_int32), ("n_p", C.c_int32), ("N", C.c_int32),
        ("react", _i32p), ("prod", _i32p), ("param", _i32p), ("logk_fixed", _f64p),
        ("h", _f64p), ("z0", _f64p), ("n_meas", C.c_int32),
        ("meas_elem", _i32p), ("meas_species", _i32p), ("meas_tau", _f64p), ("meas_y", _f64p),
        ("meas_sigma", _f64p), ("theta_lo", _f64p), ("theta_hi", _f64p),
    ]


class IpmOpts(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("acceptable_tol", C.c_double), ("acceptable_iter", C.c_int32),
        ("max_iter", C.c_int32), ("mu_init", C.c_double), ("tau_r", C.c_double),
        ("kappa_eps", C.c_double), ("kappa_mu", C.c_double), ("theta_mu", C.c_double),
        ("tau_min", C.c_double), ("kappa_sigma", C.c_double), ("s_max", C.c_double),
        ("bound_push", C.c_double), ("bound_frac", C.c_double), ("delta_w0", C.c_double),
        ("delta_min", C.c_double), ("delta_max", C.c_double), ("kappa_w_minus", C.c_double),
        ("kappa_w_plus", C.c_double), ("kappa_w_plus_bar", C.c_double),
        ("gamma_theta", C.c_double), ("gamma_phi", C.c_double), ("s_theta", C.c_double),
        ("s_phi", C.c_double), ("eta_phi", C.c_double), ("delta_sw", C.c_double),
        ("gamma_alpha", C.c_double), ("max_ls", C.c_int32), ("precision", C.c_int32),
        ("ir_max", C.c_int32), ("pad_", C.c_int32), ("ir_tol", C.c_double), ("max_wall_s", C.c_double),
    ]


INFO_DTYPE = np.dtype([
    ("status", "<i4"), ("iter", "<i4"), ("phase", "<i4"), ("ls_trials", "<i4"),
    ("factor_tries", "<i4"), ("acc_count", "<i4"), ("filter_len", "<i4"), ("ir_sweeps", "<i4"),
    ("mu", "<f8"), ("tau", "<f8"), ("delta_w", "<f8"), ("delta_last", "<f8"),
    ("alpha_pr", "<f8"), ("alpha_du", "<f8"), ("obj", "<f8"), ("inf_pr", "<f8"),
    ("inf_du", "<f8"), ("E0", "<f8"), ("theta_cv", "<f8"), ("phi", "<f8"),
    ("theta_max", "<f8"), ("theta_min", "<f8"), ("dphi", "<f8"), ("alpha_min", "<f8"),
    ("Emu", "<f8"), ("s_d", "<f8"), ("s_c", "<f8"), ("ir_fallbacks", "<i4"), ("pad_", "<i4"),
    ("t_start", "<f8"),
])


class Layout(C.Structure):
    _fields_ = [
        ("n_inst", C.c_int32), ("n_s", C.c_int32), ("n_r", C.c_int32), ("n_p", C.c_int32),
        ("K", C.c_int32), ("b", C.c_int32), ("n_elem", C.c_int64), ("n_total", C.c_int64),
        ("m_total", C.c_int64), ("jac_len", C.c_int64), ("hess_len", C.c_int64),
        ("x_off", C.POINTER(C.c_int64)), ("g_off", C.POINTER(C.c_int64)),
        ("elem_off", C.POINTER(C.c_int64)), ("N", _i32p),
    ]


class StateLayout(C.Structure):
    _fields_ = [(n, C.c_size_t) for n in ("x", "s", "y", "vL", "vU", "zL", "zU", "dx", "ds", "dy", "info",
                                          "fth", "fph")]


EXPORTS = [
    "colloc_create", "colloc_destroy", "colloc_layout_get", "colloc_table_bytes", "colloc_upload",
    "colloc_workspace_bytes", "colloc_state_bytes", "colloc_eval", "colloc_derivs",
    "kkt_assemble", "kkt_factor", "kkt_solve", "kkt_matvec", "colloc_ipm_default_opts",
    "ipm_init", "ipm_step", "colloc_state_layout_get", "colloc_timing_enable",
    "colloc_timing_read", "colloc_tables", "ipm_graph_create", "ipm_graph_launch",
    "ipm_graph_destroy", "colloc_tile_options", "colloc_tile_set", "colloc_tile_get",
    "colloc_eval_noalloc", "colloc_forward_init",
]
NOALLOC_MAX_ELEMS = (1 << 19) // 13

_lib = None


def load(path: str = LIB_PATH):
    """Load libcolloc.so (build it with paper_2607_12201_amd.build).  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcolloc.so is not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, i32, i64, sz, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    sig = {
        "colloc_create": (i32, [C.POINTER(InstanceDesc), i32, i32, C.POINTER(vp)]),
        "colloc_destroy": (i32, [vp]),
        "colloc_layout_get": (i32, [vp, C.POINTER(Layout)]),
        "colloc_table_bytes": (sz, [vp]),
        "colloc_upload": (i32, [vp, vp, vp]),
        "colloc_workspace_bytes": (sz, [vp, i32]),
        "colloc_state_bytes": (sz, [vp]),
        "colloc_eval": (i32, [vp, vp, vp, vp, vp, vp]),
        "colloc_eval_noalloc": (i32, [vp, vp, vp, vp, vp]),
        "colloc_derivs": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "kkt_assemble": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]),
        "kkt_factor": (i32, [vp, vp, i32, vp, vp]),
        "kkt_solve": (i32, [vp, vp, i32, vp, vp, i32, f64, vp, vp]),
        "kkt_matvec": (i32, [vp, vp, vp, vp, vp]),
        "colloc_ipm_default_opts": (None, [C.POINTER(IpmOpts)]),
        "ipm_init": (i32, [vp, vp, vp, vp, C.POINTER(IpmOpts), vp]),
        "ipm_step": (i32, [vp, vp, vp, C.POINTER(IpmOpts), vp]),
        "colloc_forward_init": (i32, [vp, vp, vp, vp, vp]),
        "colloc_state_layout_get": (i32, [vp, C.POINTER(StateLayout)]),
        "colloc_timing_enable": (i32, [vp, i32]),
        "colloc_timing_read": (i32, [vp, _f64p, C.POINTER(i64), i32]),
        "colloc_tables": (i32, [i32, _f64p, _f64p]),
        "ipm_graph_create": (i32, [vp, vp, vp, C.POINTER(IpmOpts), i32, vp, C.POINTER(vp)]),
        "ipm_graph_launch": (i32, [vp, vp]),
        "ipm_graph_destroy": (i32, [vp]),
        "colloc_tile_options": (i32, [vp, i32, C.POINTER(i32), i32]),
        "colloc_tile_set": (i32, [vp, i32, i32]),
        "colloc_tile_get": (i32, [vp, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, what):
    if rc != OK:
        raise RuntimeError(f"{what} failed with code {rc}")


def default_opts(**kw) -> IpmOpts:
    o = IpmOpts()
    load().colloc_ipm_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def library_tables(K: int):
    tau = np.zeros(K + 1)
    a = np.zeros((K + 1) * (K + 1))
    _check(load().colloc_tables(K, tau.ctypes.data_as(_f64p), a.ctypes.data_as(_f64p)), "colloc_tables")
    return tau, a.reshape(K + 1, K + 1)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Problem:
    """A batch of instances of one shape class on the current CUDA device."""

    def __init__(self, instances, K: int = 3, device: str = "cuda", upload: bool = True):
        """upload=False builds a host-only handle (sizes and layouts; no device call)."""
        import torch

        self.torch = torch
        self.lib = load()
        if isinstance(instances, dict):
            instances = [instances]
        self.instances = instances
        self.K = K
        self.device = device
        self._keep = []
        descs = (InstanceDesc * len(instances))()
        for q, inst in enumerate(instances):
            d = descs[q]
            d.n_s, d.n_r, d.n_p, d.N = (int(inst[k]) for k in ("n_s", "n_r", "n_p", "N"))
            d.react = self._i32(inst["react"])
            d.prod = self._i32(inst["prod"])
            d.param = self._i32(inst["param"])
            d.logk_fixed = self._f64(inst["logk_fixed"])
            d.h = self._f64(inst["h"])
            d.z0 = self._f64(inst["z0"])
            d.n_meas = len(inst["meas_y"])
            d.meas_elem = self._i32(inst["meas_elem"])
            d.meas_species = self._i32(inst["meas_species"])
            d.meas_tau = self._f64(inst["meas_tau"])
            d.meas_y = self._f64(inst["meas_y"])
            d.meas_sigma = self._f64(inst["meas_sigma"])
            d.theta_lo = self._f64(inst["theta_lo"])
            d.theta_hi = self._f64(inst["theta_hi"])
        h = C.c_void_p()
        _check(self.lib.colloc_create(descs, len(instances), K, C.byref(h)), "colloc_create")
        self.h = h
        lay = Layout()
        _check(self.lib.colloc_layout_get(h, C.byref(lay)), "colloc_layout_get")
        self.n_inst, self.ns, self.nr, self.np_, self.b = lay.n_inst, lay.n_s, lay.n_r, lay.n_p, lay.b
        self.n_elem, self.n_total, self.m_total = lay.n_elem, lay.n_total, lay.m_total
        self.jac_len, self.hess_len = lay.jac_len, lay.hess_len
        self.x_off = np.array([lay.x_off[q] for q in range(self.n_inst)])
        self.g_off = np.array([lay.g_off[q] for q in range(self.n_inst)])
        self.Ns = np.array([lay.N[q] for q in range(self.n_inst)])
        tb = self.lib.colloc_table_bytes(h)
        self.table_bytes = int(tb)
        if upload:
            self.table = torch.empty(tb + 256, dtype=torch.uint8, device=device)
            off = (-self.table.data_ptr()) % 256
            self.table_view = self.table[off:off + tb]
            _check(self.lib.colloc_upload(h, _ptr(self.table_view), _stream()), "colloc_upload")
        sl = StateLayout()
        _check(self.lib.colloc_state_layout_get(h, C.byref(sl)), "colloc_state_layout_get")
        self.state_layout = {n: getattr(sl, n) for n, _ in StateLayout._fields_}

    def _i32(self, a):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32).ravel())
        self._keep.append(arr)
        return arr.ctypes.data_as(_i32p)

    def _f64(self, a):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
        self._keep.append(arr)
        return arr.ctypes.data_as(_f64p)

    def close(self):
        if getattr(self, "h", None):
            self.lib.colloc_destroy(self.h)
            self.h = None
        self.table = self.table_view = None   # the device tables go with the handle

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ----------------------------------------------------------------------
    def device_bytes(self, precision=FP64):
        """Device memory of this batch: tables + interior-point state + workspace."""
        return (self.table_bytes + 256 + int(self.lib.colloc_state_bytes(self.h)) +
                int(self.lib.colloc_workspace_bytes(self.h, precision)))

    def workspace(self, precision=FP64):
        n = self.lib.colloc_workspace_bytes(self.h, precision)
        return self.torch.zeros(n, dtype=self.torch.uint8, device=self.device)

    def state(self):
        n = self.lib.colloc_state_bytes(self.h)
        return self.torch.zeros(n, dtype=self.torch.uint8, device=self.device)

    def vec(self, n, fill=0.0):
        return self.torch.full((int(n),), fill, dtype=self.torch.float64, device=self.device)

    def pack_x(self, xs):
        """Concatenate per-instance primal vectors (numpy) into one device vector."""
        return self.torch.tensor(np.concatenate(xs), dtype=self.torch.float64, device=self.device)

    # -- a1/a2 ---------------------------------------------------------------------------
    def eval(self, x, ws):
        obj = self.vec(self.n_inst)
        g = self.vec(self.m_total)
        _check(self.lib.colloc_eval(self.h, _ptr(x), _ptr(obj), _ptr(g), _ptr(ws), _stream()), "colloc_eval")
        return obj, g

    def eval_noalloc(self, x, obj, g):
        """colloc_eval without a workspace (static library scratch); outputs are the caller's."""
        return self.lib.colloc_eval_noalloc(self.h, _ptr(x), _ptr(obj), _ptr(g), _stream())

    def derivs(self, x, y):
        grad = self.vec(self.n_total)
        jac = self.vec(self.jac_len)
        hess = self.vec(self.hess_len)
        _check(self.lib.colloc_derivs(self.h, _ptr(x), _ptr(y), _ptr(grad), _ptr(jac), _ptr(hess),
                                      _stream()), "colloc_derivs")
        return grad, jac, hess

    # -- a3/a4/a5 ------------------------------------------------------------------------
    def assemble(self, ws, jac, hess, sigma_x, sigma_s, delta_w, r_x, r_s, r_y, precision=FP64):
        rhs = self.vec(self.n_total)
        _check(self.lib.kkt_assemble(self.h, _ptr(jac), _ptr(hess), _ptr(sigma_x), _ptr(sigma_s),
                                     _ptr(delta_w), _ptr(r_x), _ptr(r_s), _ptr(r_y), _ptr(ws),
                                     precision, _ptr(rhs), _stream()), "kkt_assemble")
        return rhs

    def factor(self, ws, precision=FP64):
        info = self.torch.zeros(self.n_inst, dtype=self.torch.int32, device=self.device)
        _check(self.lib.kkt_factor(self.h, _ptr(ws), precision, _ptr(info), _stream()), "kkt_factor")
        return info

    def solve(self, ws, rhs, precision=FP64, ir_max=0, ir_tol=0.0, sweeps=False):
        """dx = K^{-1} rhs with the last factor; with ir_max > 0 FP64 refinement sweeps follow.
        sweeps=True also returns the per-instance sweep counts (negative: not converged)."""
        dx = self.vec(self.n_total)
        sw = self.torch.zeros(self.n_inst, dtype=self.torch.int32, device=self.device)
        _check(self.lib.kkt_solve(self.h, _ptr(ws), precision, _ptr(rhs), _ptr(dx), ir_max, ir_tol,
                                  _ptr(sw), _stream()), "kkt_solve")
        return (dx, sw) if sweeps else dx

    def matvec(self, ws, v):
        out = self.vec(self.n_total)
        _check(self.lib.kkt_matvec(self.h, _ptr(ws), _ptr(v), _ptr(out), _stream()), "kkt_matvec")
        return out

    # -- starting states ---------------------------------------------------------------------
    def forward_init(self, theta):
        """Collocation-consistent x = [z | theta] of every instance at theta ([n_inst, n_p] or
        the concatenation), and the per-instance Newton status (0 = converged)."""
        th = self.torch.as_tensor(theta, dtype=self.torch.float64, device=self.device).contiguous().reshape(-1)
        x = self.torch.empty(self.n_total, dtype=self.torch.float64, device=self.device)
        stat = self.torch.zeros(self.n_inst, dtype=self.torch.int32, device=self.device)
        _check(self.lib.colloc_forward_init(self.h, _ptr(th), _ptr(x), _ptr(stat), _stream()),
               "colloc_forward_init")
        return x, stat

    # -- a6 ------------------------------------------------------------------------------
    def ipm_init(self, x0, state, ws, opts):
        _check(self.lib.ipm_init(self.h, _ptr(x0), _ptr(state), _ptr(ws), C.byref(opts), _stream()),
               "ipm_init")

    def ipm_step(self, state, ws, opts):
        _check(self.lib.ipm_step(self.h, _ptr(state), _ptr(ws), C.byref(opts), _stream()), "ipm_step")

    def graph_create(self, state, ws, opts, steps=1):
        """Capture `steps` ipm_step calls into a HIP graph on the current (non-default) stream."""
        g = C.c_void_p()
        _check(self.lib.ipm_graph_create(self.h, _ptr(state), _ptr(ws), C.byref(opts), steps,
                                         _stream(), C.byref(g)), "ipm_graph_create")
        return g

    def graph_launch(self, g):
        _check(self.lib.ipm_graph_launch(g, _stream()), "ipm_graph_launch")

    def graph_destroy(self, g):
        _check(self.lib.ipm_graph_destroy(g), "ipm_graph_destroy")

    # -- tuning hook ---------------------------------------------------------------------
    TILE_KERNELS = ("level0", "chain", "border")

    def tile_options(self, which):
        buf = (C.c_int32 * 8)()
        n = self.lib.colloc_tile_options(self.h, self.TILE_KERNELS.index(which), buf, 8)
        if n < 0:
            raise RuntimeError(f"colloc_tile_options failed with code {n}")
        return [int(buf[i]) for i in range(min(n, 8))]

    def tile_set(self, which, ts):
        _check(self.lib.colloc_tile_set(self.h, self.TILE_KERNELS.index(which), int(ts)), "colloc_tile_set")

    def tile_get(self, which):
        return int(self.lib.colloc_tile_get(self.h, self.TILE_KERNELS.index(which)))

    def state_vec(self, state, name, n=None):
        off = self.state_layout[name]
        if n is None:
            n = {"x": self.n_total, "dx": self.n_total, "zL": self.n_inst * self.np_,
                 "zU": self.n_inst * self.np_}.get(name, self.m_total)
        return state[off:off + 8 * int(n)].view(self.torch.float64)

    def info(self, state):
        off = self.state_layout["info"]
        raw = state[off:off + INFO_DTYPE.itemsize * self.n_inst].cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=INFO_DTYPE)

    # -- timing --------------------------------------------------------------------------
    def timing(self, enable=True):
        _check(self.lib.colloc_timing_enable(self.h, 1 if enable else 0), "colloc_timing_enable")

    def timing_read(self):
        ms = np.zeros(len(PHASES))
        ln = np.zeros(len(PHASES), dtype=np.int64)
        _check(self.lib.colloc_timing_read(self.h, ms.ctypes.data_as(_f64p),
                                           ln.ctypes.data_as(C.POINTER(C.c_int64)), len(PHASES)),
               "colloc_timing_read")
        return dict(zip(PHASES, ms)), dict(zip(PHASES, ln))
