"""Helpers shared by the GPU parity tests: run a workload through the C ABI
and through the FP64 oracle on the same seeded inputs, and compare."""
import math
import sys

import numpy as np

from oracle import orc

C0SQ = {0: 0.6979533220196833, 1: 2.0 / 3.0}

# Tolerances on the relative L-infinity error of rho, u and theta against the
# FP64 oracle: 1e-5 for FP32 storage, 2e-3 for 16-bit deviation storage.
TOL = {0: 1e-5, 1: 2e-3, 2: 2e-3}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_sim(cfg, shape=None):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg.get("nz", 1)
    if shape is not None:
        if len(shape) == 2:
            ny, nx = shape
            nz = 1
        else:
            nz, ny, nx = shape
    return orc.Sim(cfg["lattice"], nx, ny, nz, tau_hat=cfg["tau_hat"], sources=cfg["sources"],
                   isothermal=cfg.get("isothermal", 0), g=tuple(cfg.get("g", (0, 0, 0))),
                   prandtl=cfg.get("prandtl", 1.0), eos_a=cfg.get("eos_a", 0.0), eos_b=cfg.get("eos_b", 0.0),
                   eos_T=cfg.get("eos_T", 0.0), sc_G=cfg.get("sc_G", -1.0), ptensor_k=cfg.get("ptensor_k", 0.0),
                   walls=cfg.get("walls", 0), theta_wall=tuple(cfg.get("theta_wall", (1.0, 1.0))),
                   u_wall=cfg.get("u_wall", ((0, 0, 0), (0, 0, 0))), eos=cfg.get("eos", 0),
                   grad_lag=cfg.get("grad_lag", 0))


def run_oracle(cfg, rho, u, theta, steps, shape=None):
    s = oracle_sim(cfg, shape)
    s.init(np.asarray(rho, np.float64), np.asarray(u, np.float64), np.asarray(theta, np.float64))
    s.step(steps)
    return s.fields()


def run_gpu(cfg, rho, u, theta, steps, storage=0, variant=None, tune=False):
    import torch
    from paper_2411_10751_amd import holb
    c = dict(cfg)
    c["storage"] = storage
    sim = holb.Sim(c)
    if variant is not None:
        sim.set_variant(variant)
    sim.init(rho, u, theta)
    if tune:
        sim.tune()
    sim.step(steps)
    r, uu, t = sim.fields()
    torch.cuda.synchronize()
    out = (r.cpu().numpy().astype(np.float64), uu.cpu().numpy().astype(np.float64),
           t.cpu().numpy().astype(np.float64))
    sim.close()
    return out


def rel_errors(gpu, ref, lattice):
    """(e_rho, e_u, e_theta): max|a - a_ref| / max|a_ref|; for u the denominator
    is max(max|u_ref|, 0.01 c0) so that near-zero velocity fields cannot blow
    the ratio up."""
    r, u, t = gpu
    ro, uo, to = ref
    c0 = math.sqrt(C0SQ[lattice])
    er = np.abs(r - ro).max() / np.abs(ro).max()
    eu = np.abs(u - uo).max() / max(np.abs(uo).max(), 1e-2 * c0)
    et = np.abs(t - to).max() / np.abs(to).max()
    return er, eu, et


def where_max(gpu, ref):
    """Index of the largest absolute error of each field (diagnostics)."""
    out = []
    for a, b in zip(gpu, ref):
        d = np.abs(a - b)
        out.append(np.unravel_index(int(np.argmax(d)), d.shape))
    return out


def assert_parity(gpu, ref, lattice, tol, what=""):
    e = rel_errors(gpu, ref, lattice)
    log("%s rel Linf errors rho %.3g u %.3g theta %.3g (tol %.1g) at %s" %
        (what, e[0], e[1], e[2], tol, where_max(gpu, ref)))
    assert max(e) <= tol, (what, e)
    return e


def wrap_window(a, starts, sizes, axes):
    """Periodic window of an array: a[..., s:s+n] with wrap on the given axes."""
    out = a
    for ax, s, n in zip(axes, starts, sizes):
        idx = np.arange(s, s + n) % a.shape[ax]
        out = np.take(out, idx, axis=ax)
    return out
