"""Python binding of libholb.so (the C ABI declared in include/holb.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory and the stream.  The module
raises at import time if the built library is missing, so the product path
can never fall back to anything else.

Two layers:
  * holb_* functions with the C names, taking ctypes-compatible arguments;
  * Sim / Batch classes that own a torch workspace and marshal fields.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libholb.so")

ABI_VERSION = 4
FRAMES_AUTO, FRAMES_CELL, FRAMES_PLANE, FRAMES_CELL_U = 0, 1, 2, 3
EOS_VDW, EOS_CS = 0, 1
OK, EINVAL, ESIZE, EHIP, ENUMERIC, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6
D2Q37, D3Q39 = 0, 1
SRC_BODY, SRC_THERMAL, SRC_PTENSOR = 1, 2, 4
STORE_F32, STORE_F16DEV, STORE_BF16DEV = 0, 1, 2
STORAGE_BYTES = {STORE_F32: 4, STORE_F16DEV: 2, STORE_BF16DEV: 2}


class holb_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("tau_hat", ctypes.c_double),
        ("sources", ctypes.c_uint32),
        ("isothermal", ctypes.c_int32),
        ("g", ctypes.c_double * 3),
        ("prandtl", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_T", ctypes.c_double),
        ("sc_G", ctypes.c_double),
        ("ptensor_k", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("theta0", ctypes.c_double), ("u0", ctypes.c_double * 3),
        ("walls", ctypes.c_int32),
        ("theta_wall", ctypes.c_double * 2),
        ("u_wall", (ctypes.c_double * 3) * 2),
        ("frames", ctypes.c_int32),
        ("eos", ctypes.c_int32),
        ("grad_lag", ctypes.c_int32),
    ]


class HolbError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__("%s failed (%d): %s" % (what, code, msg))
        self.code = code


# One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname
# as the system one).  Importing torch first makes the dynamic linker bind
# this library to that already-loaded runtime instead of loading a second one,
# which would not see the GPU that torch has opened.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError("libholb.so is not built (expected %s); run `python -m "
                      "paper_2411_10751_amd.build` first" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.POINTER
_vp = ctypes.c_void_p
_sig = {
    "holb_last_error": ([], ctypes.c_char_p),
    "holb_lattice_info": ([ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32),
                           _P(ctypes.c_double), _P(ctypes.c_double)], ctypes.c_int32),
    "holb_workspace_size": ([_P(holb_config), _P(ctypes.c_size_t)], ctypes.c_int32),
    "holb_create": ([_P(holb_config), _vp, ctypes.c_size_t, _vp, _P(_vp)], ctypes.c_int32),
    "holb_init": ([_vp, _vp, _vp, _vp], ctypes.c_int32),
    "holb_step": ([_vp, ctypes.c_int64], ctypes.c_int32),
    "holb_fields": ([_vp, _vp, _vp, _vp], ctypes.c_int32),
    "holb_reduce": ([_vp, _P(ctypes.c_double)], ctypes.c_int32),
    "holb_reduce_noalloc": ([_vp, _P(ctypes.c_double)], ctypes.c_int32),
    "holb_error_flags": ([_vp, _P(ctypes.c_uint32)], ctypes.c_int32),
    "holb_state_bytes": ([_vp, _P(ctypes.c_size_t)], ctypes.c_int32),
    "holb_get_state": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int32),
    "holb_set_state": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int32),
    "holb_tune": ([_vp, _P(ctypes.c_int32)], ctypes.c_int32),
    "holb_set_variant": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "holb_timing_start": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "holb_batch_timing_start": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "holb_batch_timing_stop": ([_vp, _P(ctypes.c_double), _P(ctypes.c_int64), _P(ctypes.c_int64), ctypes.c_char_p,
                                ctypes.c_size_t], ctypes.c_int32),
    "holb_timing_stop": ([_vp, _P(ctypes.c_double), _P(ctypes.c_int64), _P(ctypes.c_int64), ctypes.c_char_p,
                          ctypes.c_size_t], ctypes.c_int32),
    "holb_num_variants": ([_vp, _P(ctypes.c_int32)], ctypes.c_int32),
    "holb_destroy": ([_vp], ctypes.c_int32),
    "holb_batch_workspace_size": ([_P(holb_config), ctypes.c_int32, _P(ctypes.c_size_t)], ctypes.c_int32),
    "holb_batch_create": ([_P(holb_config), ctypes.c_int32, _vp, ctypes.c_size_t, _vp, _P(_vp)],
                          ctypes.c_int32),
    "holb_batch_init": ([_vp, _P(_vp), _P(_vp), _P(_vp)], ctypes.c_int32),
    "holb_batch_step": ([_vp, ctypes.c_int64], ctypes.c_int32),
    "holb_batch_fields": ([_vp, ctypes.c_int32, _vp, _vp, _vp], ctypes.c_int32),
    "holb_batch_reduce": ([_vp, ctypes.c_int32, _P(ctypes.c_double)], ctypes.c_int32),
    "holb_batch_tune": ([_vp, _P(ctypes.c_int32)], ctypes.c_int32),
    "holb_batch_set_variant": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "holb_batch_destroy": ([_vp], ctypes.c_int32),
}
for _name, (_args, _res) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res
    globals()[_name] = _fn


def last_error():
    return _lib.holb_last_error().decode()


def check(code, what):
    if code != OK:
        raise HolbError(code, what, last_error())
    return code


def make_config(cfg):
    """holb_config from a plain dict (the keys of the workload recipes)."""
    c = holb_config()
    c.abi_version = ABI_VERSION
    c.lattice = int(cfg["lattice"])
    c.nx, c.ny, c.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
    c.tau_hat = float(cfg["tau_hat"])
    c.sources = int(cfg.get("sources", 0))
    c.isothermal = int(cfg.get("isothermal", 0))
    g = list(cfg.get("g", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    for a in range(3):
        c.g[a] = float(g[a])
    c.prandtl = float(cfg.get("prandtl", 1.0))
    c.eos_a = float(cfg.get("eos_a", 0.0))
    c.eos_b = float(cfg.get("eos_b", 0.0))
    c.eos_T = float(cfg.get("eos_T", 0.0))
    c.sc_G = float(cfg.get("sc_G", -1.0))
    c.ptensor_k = float(cfg.get("ptensor_k", 0.0))
    c.storage = int(cfg.get("storage", STORE_F32))
    c.rho0 = float(cfg.get("rho0", 1.0))
    c.theta0 = float(cfg.get("theta0", 1.0))
    u0 = list(cfg.get("u0", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    for a in range(3):
        c.u0[a] = float(u0[a])
    c.walls = int(cfg.get("walls", 0))
    tw = cfg.get("theta_wall", (1.0, 1.0))
    c.theta_wall[0], c.theta_wall[1] = float(tw[0]), float(tw[1])
    uw = cfg.get("u_wall", ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
    for w in range(2):
        uu = list(uw[w]) + [0.0, 0.0, 0.0]
        for a in range(3):
            c.u_wall[w][a] = float(uu[a])
    c.frames = int(cfg.get("frames", 0))
    c.eos = int(cfg.get("eos", 0))
    c.grad_lag = int(cfg.get("grad_lag", 0))
    return c


def lattice_info(lattice):
    """(c[Q,3] int, w[Q], c0sq) in the library's velocity order."""
    Q = ctypes.c_int32()
    D = ctypes.c_int32()
    c = (ctypes.c_int32 * (3 * 39))()
    w = (ctypes.c_double * 39)()
    c0 = ctypes.c_double()
    check(holb_lattice_info(lattice, ctypes.byref(Q), ctypes.byref(D), c, w, ctypes.byref(c0)),
          "holb_lattice_info")
    q = Q.value
    return (np.array(c[:3 * q], dtype=np.int64).reshape(q, 3), np.array(w[:q]), c0.value)


def workspace_size(cfg):
    c = make_config(cfg)
    n = ctypes.c_size_t()
    check(holb_workspace_size(ctypes.byref(c), ctypes.byref(n)), "holb_workspace_size")
    return n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _torch():
    import torch
    return torch


def _warn_storage(cfg):
    """BF16 storage keeps 8 significand bits: against the FP64 reference it
    stays within 2e-3 on smooth walled flows, but not at liquid-vapour
    interfaces (pressure-tensor source) or over long periodic thermal runs,
    with any frames.  Say so when such a run is created."""
    if int(cfg.get("storage", 0)) != STORE_BF16DEV:
        return
    src = int(cfg.get("sources", 0))
    if src & SRC_PTENSOR or (src & SRC_THERMAL and not int(cfg.get("walls", 0))):
        import warnings
        warnings.warn("BF16 deviation storage exceeds a 2e-3 relative error against the FP64 reference on "
                      "droplet interfaces and long periodic thermal runs; FP16 or FP32 storage is advised",
                      stacklevel=3)


class Sim:
    """One simulation on one GPU.  Owns its workspace (a torch uint8 tensor)."""

    def __init__(self, cfg, device="cuda", stream=None):
        torch = _torch()
        self.cfg = dict(cfg)
        self.D = 2 if int(cfg["lattice"]) == D2Q37 else 3
        self.shape = (int(cfg["ny"]), int(cfg["nx"])) if self.D == 2 else (
            int(cfg["nz"]), int(cfg["ny"]), int(cfg["nx"]))
        self.N = int(np.prod(self.shape))
        self.device = torch.device(device)
        self._c = make_config(cfg)
        nbytes = ctypes.c_size_t()
        check(holb_workspace_size(ctypes.byref(self._c), ctypes.byref(nbytes)), "holb_workspace_size")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(holb_create(ctypes.byref(self._c), _ptr(self.ws), nbytes.value,
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "holb_create")
        self._h = h
        _warn_storage(cfg)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            holb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape):
        torch = _torch()
        t = torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == tuple(shape), (t.shape, shape)
        return t

    def init(self, rho, u, theta):
        r = self._dev(rho, self.shape)
        uu = self._dev(u, (self.D,) + self.shape)
        t = self._dev(theta, self.shape)
        check(holb_init(self._h, _ptr(r), _ptr(uu), _ptr(t)), "holb_init")
        self._keep = (r, uu, t)  # keep alive until the stream has consumed them

    def step(self, n=1):
        check(holb_step(self._h, int(n)), "holb_step")

    def fields(self):
        torch = _torch()
        r = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((self.D,) + self.shape, dtype=torch.float32, device=self.device)
        t = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        check(holb_fields(self._h, _ptr(r), _ptr(u), _ptr(t)), "holb_fields")
        return r, u, t

    def reduce(self):
        out = (ctypes.c_double * 5)()
        check(holb_reduce(self._h, out), "holb_reduce")
        return np.array(out[:])

    def reduce_noalloc(self):
        out = (ctypes.c_double * 5)()
        check(holb_reduce_noalloc(self._h, out), "holb_reduce_noalloc")
        return np.array(out[:])

    def error_flags(self):
        f = ctypes.c_uint32()
        check(holb_error_flags(self._h, ctypes.byref(f)), "holb_error_flags")
        return f.value

    def state_bytes(self):
        n = ctypes.c_size_t()
        check(holb_state_bytes(self._h, ctypes.byref(n)), "holb_state_bytes")
        return n.value

    def get_state(self):
        torch = _torch()
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        check(holb_get_state(self._h, _ptr(buf), buf.numel()), "holb_get_state")
        return buf

    def set_state(self, buf):
        check(holb_set_state(self._h, _ptr(buf), buf.numel()), "holb_set_state")

    def tune(self):
        v = ctypes.c_int32()
        check(holb_tune(self._h, ctypes.byref(v)), "holb_tune")
        return v.value

    def set_variant(self, v):
        check(holb_set_variant(self._h, int(v)), "holb_set_variant")

    def num_variants(self):
        n = ctypes.c_int32()
        check(holb_num_variants(self._h, ctypes.byref(n)), "holb_num_variants")
        return n.value

    def timing_start(self, max_steps):
        check(holb_timing_start(self._h, int(max_steps)), "holb_timing_start")

    def timing_stop(self):
        """(summed ms, launches, cells per launch, kernel name) of the dominant
        kernel over the steps timed since timing_start."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        cells = ctypes.c_int64()
        name = ctypes.create_string_buffer(256)
        check(holb_timing_stop(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(cells), name, 256),
              "holb_timing_stop")
        return ms.value, n.value, cells.value, name.value.decode()


class Batch:
    """Many independent periodic D2Q37 runs advanced by one launch per step."""

    def __init__(self, cfgs, device="cuda", stream=None):
        torch = _torch()
        self.cfgs = [dict(c) for c in cfgs]
        self.n = len(cfgs)
        self.device = torch.device(device)
        arr = (holb_config * self.n)(*[make_config(c) for c in cfgs])
        self._arr = arr
        nbytes = ctypes.c_size_t()
        check(holb_batch_workspace_size(arr, self.n, ctypes.byref(nbytes)), "holb_batch_workspace_size")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(holb_batch_create(arr, self.n, _ptr(self.ws), nbytes.value,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "holb_batch_create")
        self._h = h
        self.shapes = [(int(c["ny"]), int(c["nx"])) for c in cfgs]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            holb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rhos, us, thetas):
        torch = _torch()
        keep = []
        pr, pu, pt = [], [], []
        for r, u, t, shp in zip(rhos, us, thetas, self.shapes):
            rr = torch.as_tensor(r, dtype=torch.float32, device=self.device).contiguous()
            uu = torch.as_tensor(u, dtype=torch.float32, device=self.device).contiguous()
            tt = torch.as_tensor(t, dtype=torch.float32, device=self.device).contiguous()
            assert tuple(rr.shape) == shp and tuple(uu.shape) == (2,) + shp and tuple(tt.shape) == shp
            keep += [rr, uu, tt]
            pr.append(rr.data_ptr()); pu.append(uu.data_ptr()); pt.append(tt.data_ptr())
        A = ctypes.c_void_p * self.n
        check(holb_batch_init(self._h, A(*pr), A(*pu), A(*pt)), "holb_batch_init")
        self._keep = keep

    def step(self, n=1):
        check(holb_batch_step(self._h, int(n)), "holb_batch_step")

    def fields(self, run):
        torch = _torch()
        shp = self.shapes[run]
        r = torch.empty(shp, dtype=torch.float32, device=self.device)
        u = torch.empty((2,) + shp, dtype=torch.float32, device=self.device)
        t = torch.empty(shp, dtype=torch.float32, device=self.device)
        check(holb_batch_fields(self._h, int(run), _ptr(r), _ptr(u), _ptr(t)), "holb_batch_fields")
        return r, u, t

    def reduce(self, run):
        out = (ctypes.c_double * 5)()
        check(holb_batch_reduce(self._h, int(run), out), "holb_batch_reduce")
        return np.array(out[:])

    def tune(self):
        v = ctypes.c_int32()
        check(holb_batch_tune(self._h, ctypes.byref(v)), "holb_batch_tune")
        return v.value

    def set_variant(self, v):
        check(holb_batch_set_variant(self._h, int(v)), "holb_batch_set_variant")

    def timing_start(self, max_steps):
        check(holb_batch_timing_start(self._h, int(max_steps)), "holb_batch_timing_start")

    def timing_stop(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        cells = ctypes.c_int64()
        name = ctypes.create_string_buffer(256)
        check(holb_batch_timing_stop(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(cells), name, 256),
              "holb_batch_timing_stop")
        return ms.value, n.value, cells.value, name.value.decode()
