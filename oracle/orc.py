"""ctypes binding of the FP64 CPU oracle (holb_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
benchmark's CPU-baseline leg to check the HIP path.  The product never imports
it.  Arrays are numpy float64; fields use the layout rho[N], u[D, N],
theta[N] with cell = x + nx*(y + ny*z) (numpy shape (nz, ny, nx) flattened).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "holb_oracle.c")

D2Q37 = 0
D3Q39 = 1
EOS_VDW = 0
EOS_CS = 1
SRC_BODY = 1
SRC_THERMAL = 2
SRC_PTENSOR = 4

OK = 0
EINVAL = -1
ENUMERIC = -4
EUNSUPPORTED = -5


def build(force=False):
    """Compile the oracle with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau_hat", ctypes.c_double),
        ("sources", ctypes.c_uint),
        ("isothermal", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("prandtl", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_T", ctypes.c_double),
        ("sc_G", ctypes.c_double),
        ("ptensor_k", ctypes.c_double),
        ("walls", ctypes.c_int),
        ("theta_wall", ctypes.c_double * 2),
        ("u_wall", (ctypes.c_double * 3) * 2),
        ("eos", ctypes.c_int),
        ("grad_lag", ctypes.c_int),
    ]


class _Lattice(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int), ("Q", ctypes.c_int),
        ("c", (ctypes.c_int * 3) * 39),
        ("w", ctypes.c_double * 39),
        ("c0sq", ctypes.c_double),
        ("opp", ctypes.c_int * 39),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d = ctypes.c_double
        dp = P(d)
        _lib.orc_lattice_get.argtypes = [ctypes.c_int, P(_Lattice)]
        _lib.orc_feq.argtypes = [ctypes.c_int, d, dp, d, dp]
        _lib.orc_src_force.argtypes = [ctypes.c_int, dp, dp, d, dp]
        _lib.orc_src_thermal.argtypes = [ctypes.c_int, d, d, d, dp, dp]
        _lib.orc_src_ptensor.argtypes = [ctypes.c_int, d, d, d, dp, d, dp]
        _lib.orc_vdw_pressure.argtypes = [d, d, d, d, dp]
        _lib.orc_psi.argtypes = [ctypes.c_int, d, d, d, d, d, dp]
        _lib.orc_cs_pressure.argtypes = [d, d, d, d, dp]
        _lib.orc_psi_eos.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d, d, dp]
        _lib.orc_sc_force_field.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            dp, d, dp]
        _lib.orc_create.argtypes = [P(_Config), P(ctypes.c_void_p)]
        _lib.orc_init.argtypes = [ctypes.c_void_p, dp, dp, dp]
        _lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        _lib.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        _lib.orc_reduce.argtypes = [ctypes.c_void_p, dp]
        _lib.orc_get_state.argtypes = [ctypes.c_void_p, dp]
        _lib.orc_set_state.argtypes = [ctypes.c_void_p, dp]
        _lib.orc_collide_only.argtypes = [ctypes.c_void_p, dp]
        _lib.orc_destroy.argtypes = [ctypes.c_void_p]
        _lib.orc_destroy.restype = None
        _lib.orc_num_threads.argtypes = []
        _lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib.orc_set_num_threads.restype = None
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("oracle %s failed with code %d" % (what, code))
        self.code = code


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


class Lattice:
    """Velocity set c[Q, 3] (int), weights w[Q], c0^2, opposite index."""

    def __init__(self, lattice):
        L = _Lattice()
        _check(lib().orc_lattice_get(lattice, ctypes.byref(L)), "lattice_get")
        self.D, self.Q = L.D, L.Q
        self.c = np.array([[L.c[i][a] for a in range(3)] for i in range(L.Q)], dtype=np.int64)
        self.w = np.array([L.w[i] for i in range(L.Q)])
        self.c0sq = L.c0sq
        self.opp = np.array([L.opp[i] for i in range(L.Q)], dtype=np.int64)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def feq(lattice, rho, u, theta):
    Q = 37 if lattice == D2Q37 else 39
    out = np.empty(Q)
    _check(lib().orc_feq(lattice, float(rho), _ptr(_f64(np.pad(np.asarray(u, float), (0, 3 - len(u))))),
                         float(theta), _ptr(out)), "feq")
    return out


def src_force(lattice, F, u, theta):
    Q = 37 if lattice == D2Q37 else 39
    out = np.empty(Q)
    pad = lambda v: _f64(np.pad(np.asarray(v, float), (0, 3 - len(v))))
    _check(lib().orc_src_force(lattice, _ptr(pad(F)), _ptr(pad(u)), float(theta), _ptr(out)), "src_force")
    return out


def src_thermal(lattice, rho, theta, prandtl, grad_theta):
    Q = 37 if lattice == D2Q37 else 39
    out = np.empty(Q)
    g = _f64(np.pad(np.asarray(grad_theta, float), (0, 3 - len(grad_theta))))
    _check(lib().orc_src_thermal(lattice, float(rho), float(theta), float(prandtl), _ptr(g), _ptr(out)),
           "src_thermal")
    return out


def src_ptensor(lattice, tau_hat, k, G, Fsc, psi):
    Q = 37 if lattice == D2Q37 else 39
    out = np.empty(Q)
    F = _f64(np.pad(np.asarray(Fsc, float), (0, 3 - len(Fsc))))
    _check(lib().orc_src_ptensor(lattice, float(tau_hat), float(k), float(G), _ptr(F), float(psi), _ptr(out)),
           "src_ptensor")
    return out


def vdw_pressure(a, b, T, rho):
    p = ctypes.c_double()
    _check(lib().orc_vdw_pressure(a, b, T, float(rho), ctypes.byref(p)), "vdw_pressure")
    return p.value


def cs_pressure(a, b, T, rho):
    p = ctypes.c_double()
    _check(lib().orc_cs_pressure(a, b, T, float(rho), ctypes.byref(p)), "cs_pressure")
    return p.value


def psi(lattice, a, b, T, G, rho, eos=EOS_VDW):
    p = ctypes.c_double()
    _check(lib().orc_psi_eos(lattice, eos, a, b, T, G, float(rho), ctypes.byref(p)), "psi")
    return p.value


def sc_force_field(lattice, psi_field, G):
    """F^SC of Eq. (3.8) for a periodic psi field of numpy shape (nz, ny, nx) or (ny, nx)."""
    shp = psi_field.shape
    nz, ny, nx = (1,) + shp if len(shp) == 2 else shp
    p = _f64(psi_field).ravel()
    out = np.empty(3 * p.size)
    _check(lib().orc_sc_force_field(lattice, nx, ny, nz, _ptr(p), float(G), _ptr(out)), "sc_force_field")
    return out.reshape((3,) + shp)


class Sim:
    """Whole-grid FP64 simulation.

    Keyword arguments mirror the GPU configuration: lattice, nx, ny, nz,
    tau_hat, sources, isothermal, g, prandtl, eos_a, eos_b, eos_T, sc_G,
    ptensor_k, walls, theta_wall (low, high), u_wall (low, high), eos, grad_lag.
    """

    def __init__(self, lattice, nx, ny, nz=1, tau_hat=0.8, sources=0, isothermal=0, g=(0, 0, 0),
                 prandtl=1.0, eos_a=0.0, eos_b=0.0, eos_T=0.0, sc_G=-1.0, ptensor_k=0.0, walls=0,
                 theta_wall=(1.0, 1.0), u_wall=((0, 0, 0), (0, 0, 0)), eos=EOS_VDW, grad_lag=0):
        c = _Config()
        c.lattice, c.nx, c.ny, c.nz = lattice, nx, ny, nz
        c.tau_hat, c.sources, c.isothermal = tau_hat, sources, int(isothermal)
        for a in range(3):
            c.g[a] = g[a] if a < len(g) else 0.0
        c.prandtl = prandtl
        c.eos_a, c.eos_b, c.eos_T, c.sc_G, c.ptensor_k = eos_a, eos_b, eos_T, sc_G, ptensor_k
        c.walls = int(walls)
        c.eos = int(eos)
        c.grad_lag = int(grad_lag)
        c.theta_wall[0], c.theta_wall[1] = theta_wall
        for w in range(2):
            for a in range(3):
                c.u_wall[w][a] = u_wall[w][a] if a < len(u_wall[w]) else 0.0
        self._cfg = c
        h = ctypes.c_void_p()
        _check(lib().orc_create(ctypes.byref(c), ctypes.byref(h)), "create")
        self._h = h
        self.lattice = lattice
        self.D = 2 if lattice == D2Q37 else 3
        self.Q = 37 if lattice == D2Q37 else 39
        self.shape = (ny, nx) if self.D == 2 else (nz, ny, nx)
        self.N = nx * ny * nz

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    def init(self, rho, u, theta):
        r = _f64(rho, self.N)
        uu = _f64(u, self.D * self.N)
        t = _f64(theta, self.N)
        _check(lib().orc_init(self._h, _ptr(r), _ptr(uu), _ptr(t)), "init")

    def step(self, n=1):
        _check(lib().orc_step(self._h, int(n)), "step")

    def fields(self):
        r = np.empty(self.N)
        u = np.empty(self.D * self.N)
        t = np.empty(self.N)
        _check(lib().orc_fields(self._h, _ptr(r), _ptr(u), _ptr(t)), "fields")
        return r.reshape(self.shape), u.reshape((self.D,) + self.shape), t.reshape(self.shape)

    def reduce(self):
        out = np.empty(5)
        _check(lib().orc_reduce(self._h, _ptr(out)), "reduce")
        return out

    def get_state(self):
        f = np.empty(self.Q * self.N)
        _check(lib().orc_get_state(self._h, _ptr(f)), "get_state")
        return f.reshape((self.Q,) + self.shape)

    def set_state(self, f):
        ff = _f64(f, self.Q * self.N)
        _check(lib().orc_set_state(self._h, _ptr(ff)), "set_state")

    def collide_only(self):
        f = np.empty(self.Q * self.N)
        _check(lib().orc_collide_only(self._h, _ptr(f)), "collide_only")
        return f.reshape((self.Q,) + self.shape)
