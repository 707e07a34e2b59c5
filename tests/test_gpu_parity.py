"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.

Tolerances (relative L-infinity of rho, u, theta): 1e-5 with FP32 storage,
2e-3 with 16-bit deviation storage.  Small cases span several blocks and a
ragged tail; the full-size workloads run a few steps in the launch
configuration the benchmark times and are compared on periodic windows the
oracle can compute on its own (the window interior is exact because the
dependency cone of n steps is bounded).
"""
import math

import numpy as np
import pytest

from _parity import TOL, assert_parity, log, rel_errors, run_gpu, run_oracle, wrap_window
from oracle import orc
from paper_2411_10751_amd import inputs

pytestmark = pytest.mark.gpu


def _both(w, steps=None, storage=0, **kw):
    steps = w["steps"] if steps is None else steps
    cfg = w["config"]
    log("case %s steps=%d storage=%d %s" % (w["name"], steps, storage, kw))
    g = run_gpu(cfg, w["rho"], w["u"], w["theta"], steps, storage=storage, **kw)
    o = run_oracle(cfg, w["rho"], w["u"], w["theta"], steps)
    return g, o


# ------------------------------------------------------------- small cases


def test_body_force_64_full_horizon():
    """The 64 x 64 body-force workload at its full 500-step horizon."""
    w = inputs.body_force_2d(n=64, steps=500)
    g, o = _both(w)
    assert_parity(g, o, 0, TOL[0], w["name"])


@pytest.mark.parametrize("frames", [0, 1])
def test_body_force_64_full_horizon_fp16(frames):
    """The same in FP16 deviation storage, with the frames AUTO takes there
    (one per plane) and with per-cell frames."""
    w = inputs.body_force_2d(n=64, steps=500)
    w = dict(w, config=dict(w["config"], frames=frames))
    g, o = _both(w, storage=1)
    assert_parity(g, o, 0, TOL[1], w["name"])


def test_body_force_invariants_on_gpu():
    """Mass constant and total momentum growing by M g per step (FP64 totals
    of the FP32 state)."""
    import torch
    from paper_2411_10751_amd import holb
    w = inputs.body_force_2d(n=64, steps=100)
    sim = holb.Sim(w["config"])
    sim.init(w["rho"], w["u"], w["theta"])
    r0 = sim.reduce()
    M = r0[0]
    g = w["config"]["g"][1]
    for k in range(1, 4):
        sim.step(25)
        r = sim.reduce()
        log("step %d mass %.15g momentum %.6g %.6g" % (25 * k, r[0], r[1], r[2]))
        assert abs(r[0] - M) < 2e-6 * M
        assert abs(r[2] - r0[2] - 25 * k * M * g) < 1e-4 * 25 * k * M * g + 1e-6
    torch.cuda.synchronize()


def test_thermal_small():
    w = inputs.thermal_2d(n=96, steps=300)
    g, o = _both(w)
    assert_parity(g, o, 0, TOL[0], w["name"])


def test_thermal_body_ragged():
    """A grid that is not a multiple of the block size, thermal + body force."""
    w = inputs.thermal_2d(n=64, steps=100)
    cfg = dict(w["config"], nx=67, ny=45, sources=inputs.SRC_BODY | inputs.SRC_THERMAL, g=(2e-5, -1e-5, 0))
    rng = np.random.default_rng(5)
    rho = (1 + 0.02 * rng.standard_normal((45, 67))).astype(np.float32)
    u = (0.05 * rng.standard_normal((2, 45, 67))).astype(np.float32)
    th = (1 + 0.03 * rng.standard_normal((45, 67))).astype(np.float32)
    w2 = dict(name="ragged_67x45", config=cfg, rho=rho, u=u, theta=th, steps=100)
    g, o = _both(w2)
    assert_parity(g, o, 0, TOL[0], w2["name"])


@pytest.mark.parametrize("shape", [(3, 5), (1, 40), (7, 1), (128, 1), (130, 2)])
def test_tiny_and_degenerate_grids(shape):
    """Grids smaller than the streaming reach (periodic wrap many times over),
    among them quasi-1D grids one and two cells wide in x and long in y, whose
    wavefronts lie away from the y edges (the pull's x-edge path)."""
    ny, nx = shape
    rng = np.random.default_rng(6)
    cfg = inputs.base_config(lattice=0, nx=nx, ny=ny, tau_hat=0.9,
                             sources=inputs.SRC_BODY | inputs.SRC_THERMAL, g=(1e-4, 2e-4, 0), prandtl=0.8)
    w = dict(name="tiny_%dx%d" % (ny, nx), config=cfg,
             rho=(1 + 0.02 * rng.standard_normal(shape)).astype(np.float32),
             u=(0.03 * rng.standard_normal((2,) + shape)).astype(np.float32),
             theta=(1 + 0.02 * rng.standard_normal(shape)).astype(np.float32), steps=50)
    g, o = _both(w)
    assert_parity(g, o, 0, TOL[0], w["name"])


@pytest.mark.parametrize("nx", [1, 2])
def test_thin_3d_slab(nx):
    """D3Q39 periodic slabs one and two cells wide in x (24 x 24 in y, z):
    every wavefront lies away from the y and z edges while x wraps many
    times over within the lattice reach."""
    n = 24
    rng = np.random.default_rng(21)
    shape = (n, n, nx)
    cfg = inputs.base_config(lattice=1, nx=nx, ny=n, nz=n, tau_hat=0.75,
                             sources=inputs.SRC_BODY | inputs.SRC_THERMAL, g=(1e-4, -2e-4, 1e-4), prandtl=0.8)
    w = dict(name="slab3d_%d" % nx, config=cfg,
             rho=(1 + 0.02 * rng.standard_normal(shape)).astype(np.float32),
             u=(0.03 * rng.standard_normal((3,) + shape)).astype(np.float32),
             theta=(1 + 0.02 * rng.standard_normal(shape)).astype(np.float32), steps=40)
    g, o = _both(w)
    assert_parity(g, o, 1, TOL[0], w["name"])


def _ptensor_small(n=160, steps=200):
    return inputs.ptensor_2d(n=n, steps=steps, ndrops=6, rmin=10.0, rmax=20.0, gap=8.0)


def test_ptensor_small_fp32():
    w = _ptensor_small()
    g, o = _both(w)
    assert_parity(g, o, 0, TOL[0], w["name"])


@pytest.mark.parametrize("storage,frames", [(1, 0), (1, 3), pytest.param(2, 0, marks=pytest.mark.xfail(
    reason="BF16 keeps 8 significand bits: u 7.3e-3 (rho 7.8e-4) at the interfaces, against the 2e-3 bound",
    strict=True)), pytest.param(2, 3, marks=pytest.mark.xfail(
        reason="BF16 with momentum frames: u 6.0e-3 (rho 6e-4), against the 2e-3 bound", strict=True))])
def test_ptensor_small_16bit(storage, frames):
    """16-bit storage on the droplet workload (160^2, six droplets, 200 steps),
    with the default frames and with momentum frames.  FP16 is the 16-bit form
    the droplet workload is quoted on; BF16 does not meet the bound on its
    interfaces with any frames."""
    w = _ptensor_small()
    w["config"] = dict(w["config"], frames=frames)
    g, o = _both(w, storage=storage)
    assert_parity(g, o, 0, TOL[storage], w["name"] + " st%d fr%d" % (storage, frames))


@pytest.mark.parametrize("storage", [0, 1])
def test_ptensor_cs_small(storage):
    """Carnahan-Starling droplets (Section 5.4, Eq. 5.9) at T = 0.8 Tc, density
    ratio 14, with the paper's optimum k, in FP32 and FP16 storage."""
    w = inputs.ptensor_cs_2d(n=128, steps=200, ndrops=4, rmin=10.0, rmax=20.0, gap=8.0)
    g, o = _both(w, storage=storage)
    assert_parity(g, o, 0, TOL[storage], w["name"] + " st%d" % storage)


@pytest.mark.parametrize("storage", [0, 1])
def test_ptensor_cs_3d(storage):
    """D3Q39 multiphase: two Carnahan-Starling droplets (r 10-13) on a 40^3
    periodic box, 60 steps of their acoustic start-up (|u| up to 0.15), FP32
    and FP16 storage."""
    w = inputs.ptensor_cs_3d(n=40, steps=60, ndrops=2, rmin=10.0, rmax=13.0, gap=4.0)
    g, o = _both(w, storage=storage)
    assert_parity(g, o, 1, TOL[storage], w["name"] + " st%d" % storage)


def _rb(n, nz, steps, **kw):
    """The Rayleigh-Benard recipe on a smaller box with the gravity of the
    256^3 workload (Ra scaled with H^3), so that the small case is as gentle
    as the full one."""
    ra = 1e5 * ((nz - 2) / 254.0) ** 3
    return inputs.rayleigh_benard_3d(n=n, nz=nz, steps=steps, ra=ra, **kw)


def _rb_small():
    return _rb(24, 20, 60)


@pytest.mark.parametrize("frames", [0, 1])
def test_rb3d_walls_fp32(frames):
    w = _rb_small()
    w["config"]["frames"] = frames
    g, o = _both(w)
    assert_parity(g, o, 1, TOL[0], w["name"] + " frames %d" % frames)


_RB_MID = {}


def _rb_mid_oracle():
    """32 x 32 x 64 box (wall distance 62) for 300 steps: the wall-normal
    gradients of the 256^3 workload scaled up four-fold, so that the
    non-equilibrium part of the populations -- what 16-bit storage rounds --
    is as large as at the 64^3 size of the workload recipe."""
    if not _RB_MID:
        w = _rb(32, 64, 300)
        _RB_MID["w"] = w
        _RB_MID["o"] = run_oracle(w["config"], w["rho"], w["u"], w["theta"], w["steps"])
    return _RB_MID["w"], _RB_MID["o"]


@pytest.mark.parametrize("storage,frames", [(0, 0), (1, 0), (1, 1), (2, 0), (2, 3)])
def test_rb3d_walls_mid(storage, frames):
    """FP32, FP16 and BF16 with their default frames (per plane, per plane,
    per cell), FP16 with per-cell frames, and BF16 with momentum frames.  BF16
    is the form closest to the bound: u 1.8e-3 with per-cell frames, 1.6e-3
    with momentum frames."""
    w, o = _rb_mid_oracle()
    log("case %s storage %d frames %d" % (w["name"], storage, frames))
    cfg = dict(w["config"], frames=frames)
    g = run_gpu(cfg, w["rho"], w["u"], w["theta"], w["steps"], storage=storage)
    assert_parity(g, o, 1, TOL[storage], w["name"] + " st%d fr%d" % (storage, frames))


@pytest.mark.parametrize("frames", [0, 1])
def test_rb3d_walls_16bit(frames):
    """FP16 on the small box, whose gradients are 14 times those of the 256^3
    workload, with its default (per-plane) and with per-cell frames (BF16
    keeps 8 bits and is checked on the larger box above)."""
    w = _rb_small()
    w["config"] = dict(w["config"], frames=frames)
    g, o = _both(w, storage=1)
    assert_parity(g, o, 1, TOL[1], w["name"] + " st1 fr%d" % frames)


def test_periodic_3d_thermal_body():
    """Periodic D3Q39 box started from the Rayleigh-Benard ramp, which jumps
    by 0.4 in theta across the periodic boundary, with per-cell frames (with
    the per-plane frames of FP32's default u reached 1.08e-5 here)."""
    w = _rb(20, 16, 50, walls=0)
    w["config"]["g"] = (1e-4, -2e-4, 3e-4)
    w["config"]["frames"] = 1
    g, o = _both(w)
    assert_parity(g, o, 1, TOL[0], "periodic 3D 20x20x16")


@pytest.mark.parametrize("frames", [0, 1])
def test_periodic_3d_smooth(frames):
    """Periodic D3Q39 box with a smooth periodic temperature profile (theta =
    1.2 + 0.2 sin(2 pi z / nz) + noise, rho = 1.2 / theta), thermal + body
    force; default (per-plane) and per-cell frames."""
    rng = np.random.default_rng(11)
    n, nz = 20, 24
    z = np.arange(nz)[:, None, None] * np.ones((1, n, n))
    th = 1.2 + 0.2 * np.sin(2 * np.pi * z / nz) + 1e-3 * rng.standard_normal((nz, n, n))
    cfg = inputs.base_config(lattice=1, nx=n, ny=n, nz=nz, tau_hat=0.56, sources=inputs.SRC_BODY | inputs.SRC_THERMAL,
                             g=(1e-4, -2e-4, 3e-4), prandtl=0.71, theta0=1.2, frames=frames)
    w = dict(name="periodic_smooth", config=cfg, rho=(1.2 / th).astype(np.float32),
             u=np.zeros((3, nz, n, n), np.float32), theta=th.astype(np.float32), steps=60)
    g, o = _both(w)
    assert_parity(g, o, 1, TOL[0], "periodic 3D smooth 20x20x24 frames %d" % frames)


def test_2d_walls_couette_like():
    """D2Q37 with TMS walls normal to y, a moving top wall and heated bottom."""
    n = 32
    rng = np.random.default_rng(9)
    cfg = inputs.base_config(lattice=0, nx=n, ny=24, tau_hat=0.75, sources=inputs.SRC_THERMAL, prandtl=0.71,
                             walls=1, theta_wall=(1.1, 0.9), u_wall=((0, 0, 0), (0.05, 0, 0)))
    shape = (24, n)
    w = dict(name="walls2d", config=cfg, rho=np.ones(shape, np.float32),
             u=np.zeros((2,) + shape, np.float32),
             theta=(1 + 0.01 * rng.standard_normal(shape)).astype(np.float32), steps=80)
    g, o = _both(w)
    assert_parity(g, o, 0, TOL[0], w["name"])


@pytest.mark.parametrize("isothermal,frames", [(1, 0), (0, 1), (0, 2)])
def test_3d_walls_moving(isothermal, frames):
    """D3Q39 between TMS walls normal to z, both walls moving tangentially in
    different directions (a 3D Couette start-up), with the body force along
    the walls; thermal runs also heat the bottom wall."""
    n, nz = 12, 20
    rng = np.random.default_rng(13)
    cfg = inputs.base_config(lattice=1, nx=n, ny=n, nz=nz, tau_hat=0.7,
                             sources=inputs.SRC_BODY | (0 if isothermal else inputs.SRC_THERMAL),
                             isothermal=isothermal, g=(2e-5, -1e-5, 0.0), prandtl=0.71, walls=1,
                             theta_wall=(1.0, 1.0) if isothermal else (1.05, 0.95),
                             u_wall=((-0.02, 0.01, 0.0), (0.04, -0.03, 0.0)), frames=frames)
    shape = (nz, n, n)
    w = dict(name="walls3d_moving", config=cfg,
             rho=(1 + 1e-3 * rng.standard_normal(shape)).astype(np.float32),
             u=np.zeros((3,) + shape, np.float32), theta=np.ones(shape, np.float32), steps=60)
    g, o = _both(w)
    assert_parity(g, o, 1, TOL[0], "%s iso %d frames %d" % (w["name"], isothermal, frames))


# ---------------------------------------------------- full-size workloads


def _window_check(w, gpu_fields, steps, radius_step, radius_fields, win, nwin, spatial_axes_last, seed):
    """Compare the full-size GPU fields on periodic windows recomputed by the
    oracle.  spatial_axes_last = number of trailing periodic axes to window."""
    rho, u, th = w["rho"], w["u"], w["theta"]
    cfg = w["config"]
    gr, gu, gt = gpu_fields
    m = steps * radius_step + radius_fields
    rng = np.random.default_rng(seed)
    worst = (0.0, 0.0, 0.0)
    nd = rho.ndim
    per_axes = list(range(nd - spatial_axes_last, nd))
    for k in range(nwin):
        starts = [int(rng.integers(0, rho.shape[a])) for a in per_axes]
        sizes = [win] * len(per_axes)
        wr = wrap_window(rho, starts, sizes, per_axes)
        wt = wrap_window(th, starts, sizes, per_axes)
        wu = wrap_window(u, starts, sizes, [a + 1 for a in per_axes])
        o = run_oracle(cfg, wr, wu, wt, steps, shape=wr.shape)
        sl = tuple(slice(None) if a not in per_axes else slice(m, win - m) for a in range(nd))
        slu = (slice(None),) + sl
        g_r = wrap_window(gr, starts, sizes, per_axes)[sl]
        g_t = wrap_window(gt, starts, sizes, per_axes)[sl]
        g_u = wrap_window(gu, starts, sizes, [a + 1 for a in per_axes])[slu]
        e = rel_errors((g_r, g_u, g_t), (o[0][sl], o[1][slu], o[2][sl]), cfg["lattice"])
        worst = tuple(max(a, b) for a, b in zip(worst, e))
        log("window %d at %s: rel errors %.3g %.3g %.3g" % (k, starts, *e))
    return worst


def test_full_rb3d_256_windows():
    """Rayleigh-Benard box 256^3 with walls, FP32, the tuned launch
    configuration, 2 steps, checked on oracle windows spanning the full height."""
    w = inputs.rayleigh_benard_3d(n=256, steps=2)
    log("case %s full size" % w["name"])
    g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], 2, tune=True)
    worst = _window_check(w, g, 2, 4, 0, win=28, nwin=3, spatial_axes_last=2, seed=41)
    assert max(worst) <= TOL[0], worst


def test_full_ptensor_2048_fp16_windows():
    """2048^2 droplets, FP16-deviation storage, 2 steps, oracle windows."""
    w = inputs.ptensor_2d(n=2048, steps=2)
    log("case %s full size fp16" % w["name"])
    g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], 2, storage=1, tune=True)
    # windows centred near droplet interfaces and in the bulk
    worst = _window_check(w, g, 2, 6, 3, win=64, nwin=4, spatial_axes_last=2, seed=43)
    assert max(worst) <= TOL[1], worst


def test_full_thermal_1024_windows():
    w = inputs.thermal_2d(n=1024, steps=3)
    log("case %s full size" % w["name"])
    g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], 3, tune=True)
    worst = _window_check(w, g, 3, 4, 0, win=48, nwin=3, spatial_axes_last=2, seed=44)
    assert max(worst) <= TOL[0], worst


@pytest.mark.parametrize("storage", [0, 1])
def test_full_body_2048_windows(storage):
    """2048^2 body-force workload in the launch configuration the benchmark
    times (block order 0; FP32 and FP16 storage, both with per-plane frames),
    3 steps, oracle windows."""
    w = inputs.body_force_2d(n=2048, steps=3)
    log("case %s full size storage %d" % (w["name"], storage))
    g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], 3, storage=storage, variant=0)
    worst = _window_check(w, g, 3, 3, 0, win=48, nwin=3, spatial_axes_last=2, seed=45)
    assert max(worst) <= TOL[storage], worst


@pytest.mark.parametrize("storage,frames", [(0, 0), (1, 0), pytest.param(1, 1, marks=pytest.mark.xfail(
    reason="FP16 with per-cell frames reaches u 3.7e-3 after 20,000 steps, against the 2e-3 bound", strict=True)),
    pytest.param(2, 3, marks=pytest.mark.xfail(
        reason="BF16 keeps 8 significand bits: even with momentum frames u reaches 4.6e-2 after 20,000 steps",
        strict=True))])
def test_full_thermal_1024_full_horizon(storage, frames):
    """The 1024^2 thermal workload over its whole 20,000-step horizon, in the
    launch configuration the benchmark times.  Its fields vary along x only,
    so every row of the exact solution is the same: the FP64 oracle runs one
    1024 x 1 row (periodic in y, the same scheme) and every GPU row is
    compared with it.  The workload is quoted on FP32 (u 7.8e-6 at 20,000
    steps); FP16 needs momentum frames over this horizon (u 1.8e-3, against
    3.7e-3 with per-cell frames), which its default frames are."""
    w = inputs.thermal_2d(n=1024, steps=20000)
    n, steps = 1024, w["steps"]
    log("case %s full size, full horizon, storage %d frames %d" % (w["name"], storage, frames))
    g = run_gpu(dict(w["config"], frames=frames), w["rho"], w["u"], w["theta"], steps, storage=storage, tune=True)
    row = dict(w["config"], ny=1)
    o = run_oracle(row, w["rho"][:1], w["u"][:, :1], w["theta"][:1], steps, shape=(1, n))
    ob = (np.broadcast_to(o[0], (n, n)), np.broadcast_to(o[1], (2, n, n)), np.broadcast_to(o[2], (n, n)))
    assert_parity(g, ob, 0, TOL[storage], w["name"] + " 20k steps st%d fr%d" % (storage, frames))


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_full_rb3d_256_column_horizon(storage):
    # default frames: per plane for FP32 and FP16 (walls), per cell for BF16
    """The 256^3 Rayleigh-Benard box over the benchmark's 200 steps, started
    without the noise so that the exact solution depends on z only: the FP64
    oracle runs one 1 x 1 x 256 column (periodic in x and y, the same walls
    and sources) and every GPU column is compared with it, in the storage
    forms and the launch configuration the benchmark times."""
    w = inputs.rayleigh_benard_3d(n=256, steps=200, noise=0.0)
    n, steps = 256, w["steps"]
    log("case %s no noise, full size, %d steps, storage %d" % (w["name"], steps, storage))
    g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], steps, storage=storage, tune=True)
    col = dict(w["config"], nx=1, ny=1)
    o = run_oracle(col, w["rho"][:, :1, :1], w["u"][:, :, :1, :1], w["theta"][:, :1, :1], steps, shape=(n, 1, 1))
    shp = (n, n, n)
    ob = (np.broadcast_to(o[0], shp), np.broadcast_to(o[1], (3,) + shp), np.broadcast_to(o[2], shp))
    assert_parity(g, ob, 1, TOL[storage], w["name"] + " column, %d steps st%d" % (steps, storage))


@pytest.mark.parametrize("storage,frames", [(0, 0), pytest.param(1, 0, marks=pytest.mark.xfail(
    reason="FP16: u reaches 2.5e-3 at the interfaces after 1000 steps (2e-5 in absolute terms, relative to the "
           "0.01 c0 floor of the velocity scale; 2.5e-3 with momentum frames too), against the 2e-3 bound; rho "
           "1.3e-3 passes.  The droplet-shaped case at the same horizon passes (u 1.4e-3)", strict=True))])
def test_full_ptensor_2048_slab_horizon(storage, frames):
    """The pressure-tensor workload's gas (van der Waals, 0.85 Tc, its k) on the
    full 2048^2 grid over its 1000-step horizon, as a flat liquid slab
    (Eq. 5.10) that depends on y only: every GPU column is compared with the
    FP64 oracle's 1 x 2048 column, in FP32 and in FP16 (the storage the
    droplet workload is quoted on)."""
    n, steps = 2048, 1000
    w = inputs.flat_interface_2d(ny=n, nx=n, eos=inputs.EOS_VDW, t_reduced=0.85, steps=steps)
    cfg = dict(w["config"], rho0=float((inputs.VDW_RHO_L_085 + inputs.VDW_RHO_G_085) / 2), frames=frames)
    rho = inputs.flat_profile(n, n, inputs.VDW_RHO_L_085, inputs.VDW_RHO_G_085, w["width"]).astype(np.float32)
    u = np.zeros((2, n, n), np.float32)
    th = np.ones((n, n), np.float32)
    log("case vdW slab %d^2, %d steps, storage %d frames %d" % (n, steps, storage, frames))
    g = run_gpu(cfg, rho, u, th, steps, storage=storage, tune=True)
    col = dict(cfg, nx=1)
    o = run_oracle(col, rho[:, :1], u[:, :, :1], th[:, :1], steps, shape=(n, 1))
    ob = (np.broadcast_to(o[0], (n, n)), np.broadcast_to(o[1], (2, n, n)), np.broadcast_to(o[2], (n, n)))
    assert_parity(g, ob, 0, TOL[storage], "vdW slab 2048^2, %d steps st%d fr%d" % (steps, storage, frames))


@pytest.mark.parametrize("case", ["rb_f32", "rb_f16", "thermal2d_f32", "thermal2d_f16"])
def test_grad_lag_parity(case):
    """The previous step's temperature gradient (grad_lag = 1): the one-pass
    thermal step against the oracle's same reading, on the walled
    Rayleigh-Benard box (24 x 24 x 20, 60 steps) and the periodic thermal
    workload on 128^2 (200 steps), in FP32 and FP16."""
    storage = 1 if case.endswith("f16") else 0
    w = _rb(24, 20, 60) if case.startswith("rb") else inputs.thermal_2d(n=128, steps=200)
    w["config"] = dict(w["config"], grad_lag=1)
    g, o = _both(w, storage=storage)
    lat = w["config"]["lattice"]
    assert_parity(g, o, lat, TOL[storage], w["name"] + " lagged st%d" % storage)
    # and it is a different scheme from the same-step one (by more than rounding)
    same = run_oracle(dict(w["config"], grad_lag=0), w["rho"], w["u"], w["theta"], w["steps"])
    assert max(rel_errors(o, same, lat)) > 1e-6


@pytest.mark.parametrize("case", ["rb_walls", "rb_walls_lag", "thermal2d_f16", "body2d"])
def test_graph_replay_matches_eager(case):
    """holb_step replays captured graphs of 16 steps: 37 steps in one call
    (two replays from alternating buffers after an odd eager start, and an
    eager remainder), repeated, against the same steps taken one call at a
    time, bitwise; with eager work and synchronisations between the calls."""
    import torch
    from paper_2411_10751_amd import holb
    storage = 1 if case.endswith("f16") else 0
    w = {"rb_walls": lambda: _rb(32, 24, 0), "rb_walls_lag": lambda: _rb(32, 24, 0),
         "thermal2d_f16": lambda: inputs.thermal_2d(n=96, steps=0),
         "body2d": lambda: inputs.body_force_2d(n=64, steps=0)}[case]()
    cfg = dict(w["config"], storage=storage, grad_lag=1 if case.endswith("lag") else 0)
    a = holb.Sim(cfg)
    a.init(w["rho"], w["u"], w["theta"])
    b = holb.Sim(cfg)
    b.init(w["rho"], w["u"], w["theta"])
    for rep in range(3):
        a.step(1)
        a.step(37)  # graphs from the other buffer, then 5 eager steps
        for _ in range(38):
            b.step(1)
        torch.cuda.synchronize()
        fa = [x.clone() for x in a.fields()]
        fb = b.fields()
        for x, y in zip(fa, fb):
            assert torch.equal(x, y), (case, rep)
        a.reduce()  # eager work between the replays
    a.close()
    b.close()


def test_grad_lag_resume_and_variants():
    """With the previous step's gradient, a run resumed from get_state
    continues bitwise, and every block order gives the same bits."""
    import torch
    from paper_2411_10751_amd import holb
    w = _rb(32, 24, 8)
    cfg = dict(w["config"], grad_lag=1)
    ref = run_gpu(cfg, w["rho"], w["u"], w["theta"], 8)
    sim = holb.Sim(cfg)
    sim.init(w["rho"], w["u"], w["theta"])
    sim.step(3)
    saved = sim.get_state().clone()
    sim.close()
    sim2 = holb.Sim(cfg)
    sim2.set_state(saved)
    sim2.step(5)
    got = [x.cpu().numpy().astype(np.float64) for x in sim2.fields()]
    sim2.close()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    for v in (1, 3):
        g = run_gpu(cfg, w["rho"], w["u"], w["theta"], 8, variant=v)
        for a, b in zip(g, ref):
            assert np.array_equal(a, b), v
    torch.cuda.synchronize()


# ------------------------------------------------ workloads at their horizons

_C3H = {}


def _c3_horizon():
    """The droplet recipe (van der Waals at 0.85 Tc, nu = 0.2, its k, profile of
    Eq. 5.11 between the Maxwell densities) on a reduced periodic 384^2 domain
    with 8 droplets of radius 20-40, over the workload's 1000 steps."""
    if not _C3H:
        w = inputs.ptensor_2d(n=384, steps=1000, ndrops=8, rmin=20.0, rmax=40.0, gap=10.0)
        _C3H["w"] = w
        _C3H["o"] = run_oracle(w["config"], w["rho"], w["u"], w["theta"], w["steps"])
    return _C3H["w"], _C3H["o"]


@pytest.mark.parametrize("storage,frames", [(0, 0), (1, 0), (1, 3), pytest.param(2, 3, marks=pytest.mark.xfail(
    reason="BF16 with momentum frames: u 1.05e-2 (rho 2.2e-3) after 1000 steps, against the 2e-3 bound",
    strict=True))])
def test_ptensor_droplets_1000_steps(storage, frames):
    w, o = _c3_horizon()
    log("case %s 1000 steps storage %d frames %d" % (w["name"], storage, frames))
    g = run_gpu(dict(w["config"], frames=frames), w["rho"], w["u"], w["theta"], w["steps"], storage=storage)
    assert_parity(g, o, 0, TOL[storage], w["name"] + " 1000 steps st%d fr%d" % (storage, frames))


_C4H = {}


def _c4_horizon():
    """The Rayleigh-Benard recipe at 64^3 (fluid height 62, the gravity of the
    256^3 box) with its seeded 1e-3 temperature noise, over 2000 steps."""
    if not _C4H:
        w = _rb(64, 64, 2000)
        _C4H["w"] = w
        _C4H["o"] = run_oracle(w["config"], w["rho"], w["u"], w["theta"], w["steps"])
    return _C4H["w"], _C4H["o"]


@pytest.mark.parametrize("storage,frames", [(0, 0), (1, 0), (1, 1), (2, 0), (2, 3)])
def test_rb3d_64_2000_steps(storage, frames):
    w, o = _c4_horizon()
    log("case %s 2000 steps storage %d frames %d" % (w["name"], storage, frames))
    g = run_gpu(dict(w["config"], frames=frames), w["rho"], w["u"], w["theta"], w["steps"], storage=storage)
    assert_parity(g, o, 1, TOL[storage], w["name"] + " 2000 steps st%d fr%d" % (storage, frames))


# --------------------------------------------------- reductions and state


def test_reduce_deterministic_and_matches_fields():
    import torch
    from paper_2411_10751_amd import holb
    w = inputs.thermal_2d(n=128, steps=20)
    log("case reduce %s" % w["name"])
    sim = holb.Sim(w["config"])
    sim.init(w["rho"], w["u"], w["theta"])
    sim.step(20)
    a = sim.reduce()
    b = sim.reduce()
    assert np.array_equal(a, b)  # bitwise repeatable
    r, u, t = [x.cpu().numpy().astype(np.float64) for x in sim.fields()]
    mass = math.fsum(r.ravel())
    # the fields are rounded to FP32 cell by cell: |sum fl(r) - sum r| <= 2^-24 sum r
    assert abs(a[0] - mass) <= 2.0 ** -24 * mass
    px = math.fsum((r * u[0]).ravel())
    assert abs(a[1] - px) <= 1e-6 * abs(px) + 1e-9
    # against the FP64 oracle's totals of the same run (Eq. 2.3 moments of the
    # fields of Eq. 4.5): mass, momentum and energy, each to the FP32 rounding
    # of the state (relative to its scale: total mass, sum rho |u|, energy)
    os_ = _oracle_sim_of(w)
    os_.step(20)
    ot = os_.reduce()
    ro, uo, to = os_.fields()
    pscale = float(np.sum(ro * np.sqrt(uo[0] ** 2 + uo[1] ** 2)))
    log("reduce vs oracle: mass %.3g momentum %.3g %.3g energy %.3g" % (
        abs(a[0] - ot[0]) / ot[0], abs(a[1] - ot[1]) / pscale, abs(a[2] - ot[2]) / pscale, abs(a[4] - ot[4]) / ot[4]))
    assert abs(a[0] - ot[0]) <= 1e-6 * ot[0]
    assert abs(a[1] - ot[1]) <= 1e-5 * pscale and abs(a[2] - ot[2]) <= 1e-5 * pscale and a[3] == 0.0
    assert abs(a[4] - ot[4]) <= 1e-6 * ot[4]
    torch.cuda.synchronize()


def _oracle_sim_of(w):
    from _parity import oracle_sim
    s = oracle_sim(w["config"])
    s.init(np.asarray(w["rho"], np.float64), np.asarray(w["u"], np.float64), np.asarray(w["theta"], np.float64))
    return s


def test_reduce_walls_matches_oracle():
    """FP64 totals on the walled Rayleigh-Benard box (mass, which the wall
    closure conserves, momentum and energy) against the oracle's."""
    import torch
    from paper_2411_10751_amd import holb
    w = _rb(24, 20, 60)
    sim = holb.Sim(w["config"])
    sim.init(w["rho"], w["u"], w["theta"])
    a0 = sim.reduce()
    sim.step(w["steps"])
    a = sim.reduce()
    os_ = _oracle_sim_of(w)
    o0 = os_.reduce()
    os_.step(w["steps"])
    ot = os_.reduce()
    ro, uo, _ = os_.fields()
    pscale = float(np.sum(ro * np.sqrt((uo ** 2).sum(axis=0))))
    log("walls reduce: mass drift gpu %.3g oracle %.3g; vs oracle mass %.3g momentum %.3g energy %.3g" % (
        a[0] / a0[0] - 1, ot[0] / o0[0] - 1, abs(a[0] - ot[0]) / ot[0], np.abs(a[1:4] - ot[1:4]).max() / pscale,
        abs(a[4] - ot[4]) / ot[4]))
    assert abs(a[0] / a0[0] - 1) < 1e-6
    assert abs(a[0] - ot[0]) <= 1e-6 * ot[0]
    assert np.abs(a[1:4] - ot[1:4]).max() <= 1e-5 * pscale
    assert abs(a[4] - ot[4]) <= 1e-6 * ot[4]
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_state_roundtrip_and_resume(storage):
    """get_state / set_state on a walled box: a fresh simulation that takes a
    saved state (populations, frames and wall targets) continues bitwise as
    the uninterrupted one, without any history of its own."""
    import torch
    from paper_2411_10751_amd import holb
    w = _rb(16, 12, 10)
    cfg = dict(w["config"], storage=storage)
    log("case state roundtrip storage %d" % storage)
    sim = holb.Sim(cfg)
    sim.init(w["rho"], w["u"], w["theta"])
    sim.step(5)
    saved = sim.get_state().clone()
    sim.step(5)
    r1 = [x.clone() for x in sim.fields()]
    sim2 = holb.Sim(cfg)
    sim2.set_state(saved)
    sim2.step(5)
    r2 = sim2.fields()
    torch.cuda.synchronize()
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)


@pytest.mark.parametrize("case", ["rb_f32", "rb_f16", "rb_bf16_mom", "thermal2d", "ptensor_f16", "periodic3d",
                                  "body2d_f16"])
def test_poisoned_workspace(case):
    """Every population slot a step should write is written, and nothing
    uninitialised reaches a result: with the whole workspace filled with NaN
    bytes before holb_init, the state after one and after two steps holds only
    finite populations, and the fields after six steps are bitwise equal to
    those of a run on a zeroed workspace."""
    import torch
    from paper_2411_10751_amd import holb
    if case.startswith("rb"):
        w = _rb(20, 16, 6)
        storage = {"rb_f32": 0, "rb_f16": 1, "rb_bf16_mom": 2}[case]
        cfg = dict(w["config"], storage=storage, frames=3 if case == "rb_bf16_mom" else 0)
    elif case == "thermal2d":
        w = inputs.thermal_2d(n=40, steps=6)
        cfg = dict(w["config"])
    elif case == "ptensor_f16":
        w = _ptensor_small(n=64, steps=6)
        cfg = dict(w["config"], storage=1)
    elif case == "body2d_f16":
        w = inputs.body_force_2d(n=40, steps=6)
        cfg = dict(w["config"], storage=1)
    else:
        w = _rb(16, 20, 6, walls=0)
        cfg = dict(w["config"])
    log("case poisoned workspace %s" % case)
    Q = 37 if cfg["lattice"] == 0 else 39
    N = int(np.prod(w["rho"].shape))
    elem = 4 if cfg.get("storage", 0) == 0 else 2
    pitch = -(-N // (256 // elem)) * (256 // elem)
    out = []
    for fill in (255, 0):
        sim = holb.Sim(cfg)
        sim.ws.fill_(fill)
        sim.init(w["rho"], w["u"], w["theta"])
        for k in range(2):
            sim.step(1)
            st = sim.get_state()
            pops = st[:Q * pitch * elem].view(torch.float32 if elem == 4 else torch.float16)
            if elem == 2 and cfg.get("storage") == 2:
                pops = st[:Q * pitch * elem].view(torch.bfloat16)
            pops = pops.view(Q, pitch)[:, :N]
            assert bool(torch.isfinite(pops).all()), (case, fill, k)
        sim.step(4)
        out.append([x.cpu().numpy() for x in sim.fields()])
        torch.cuda.synchronize()
        sim.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b), case


def test_error_flags_on_nonpositive_density():
    from paper_2411_10751_amd import holb
    w = inputs.body_force_2d(n=32, steps=1)
    rho = w["rho"].copy()
    rho[3, 4] = -1.0
    log("case negative density")
    sim = holb.Sim(w["config"])
    sim.init(rho, w["u"], w["theta"])
    with pytest.raises(holb.HolbError) as ei:
        sim.fields()
    assert ei.value.code == holb.ENUMERIC
    assert sim.error_flags() & 1


@pytest.mark.parametrize("storage,frames", [(1, 1), (2, 0), (1, 3), (2, 3)])
def test_codec_round_to_nearest_even(storage, frames):
    """The 16-bit state after init: every cell's frame is (rho, theta - 1)
    rounded to binary16, and slot i of cell y holds q_i = (f^eq_i(node y + c_i)
    - f^eq_i(rho_F, 0, theta_F)) / w_i - d_i in the frame F of y, rounded to
    nearest-even, with d_i = (f^eq_i(rho0, u0, theta0) - f^eq_i(rho0, 0,
    theta0)) / w_i; compared with torch's RNE conversion of the FP64 value,
    within the FP32 rounding of the value itself.  With momentum frames
    (frames 3) the cell also carries P = rho (u - u0) / c0^2 as 10-bit
    multiples of 2^-10, rounded to nearest, and q_i loses c_i . P."""
    import torch
    from paper_2411_10751_amd import holb
    n = 16
    rng = np.random.default_rng(3)
    shape = (n, n)
    rho = (1.2 + 0.3 * rng.standard_normal(shape)).astype(np.float32)
    u = (0.1 * rng.standard_normal((2,) + shape)).astype(np.float32)
    th = (1 + 0.1 * rng.standard_normal(shape)).astype(np.float32)
    r0, u0, t0 = 1.1, (0.02, -0.01), 1.05
    cfg = inputs.base_config(lattice=0, nx=n, ny=n, tau_hat=0.8, storage=storage, rho0=r0,
                             u0=(u0[0], u0[1], 0), theta0=t0, frames=frames)
    mom = frames == 3
    log("case codec storage %d frames %d" % (storage, frames))
    sim = holb.Sim(cfg)
    sim.init(rho, u, th)
    raw = sim.get_state().cpu()
    c, wts, c0sq = holb.lattice_info(0)
    words = raw.view(torch.int16)
    # Q planes of `pitch` binary16 codes, then one 32-bit frame word per cell
    # (n * n * 4 bytes is a multiple of 256: no padding), then with momentum a
    # plane of momentum words
    pitch = ((n * n + 127) // 128) * 128
    codes = words[:37 * pitch].view(37, pitch)[:, :n * n]
    f0 = 37 * pitch
    frames = words[f0:f0 + 2 * n * n].view(n * n, 2).view(torch.float16).double().numpy()
    # frames: binary16 RNE of (rho, theta - 1) of the cell
    want = np.stack([rho.ravel().astype(np.float64), th.ravel().astype(np.float64) - 1.0], axis=1)
    want16 = torch.tensor(want).to(torch.float16).double().numpy()
    assert np.array_equal(frames, want16)
    P = np.zeros((n * n, 2))
    if mom:
        w = words[f0 + 2 * n * n:f0 + 4 * n * n].contiguous().view(torch.int32).numpy().astype(np.int64) & 0xFFFFFFFF
        for a in range(2):
            qa = (w >> (10 * a)) & 0x3FF
            qa = np.where(qa >= 512, qa - 1024, qa)
            P[:, a] = qa / 1024.0
            exact = rho.ravel().astype(np.float64) * (u[a].ravel().astype(np.float64) - u0[a]) / c0sq
            # nearest multiple of 2^-10 (up to the FP32 evaluation of P),
            # saturating at +-511
            want = np.clip(exact, -511.0 / 1024, 511.0 / 1024)
            assert np.all(np.abs(P[:, a] - want) <= 0.5 / 1024 + 1e-6), np.abs(P[:, a] - want).max()
        assert np.all((w >> 20) & 0x3FF == 0)
    fb = orc.feq(0, r0, u0, t0)
    fb0 = orc.feq(0, r0, (0.0, 0.0), t0)
    L = orc.Lattice(0)
    idx = {tuple(v): k for k, v in enumerate(L.c.tolist())}
    dt = torch.float16 if storage == 1 else torch.bfloat16
    bad = 0
    for i in range(37):
        k = idx[tuple(c[i])]
        cx, cy = int(c[i][0]), int(c[i][1])
        d = (fb[k] - fb0[k]) / L.w[k]
        for y in range(n):
            for x in range(n):
                # slot (x, y) of direction i holds f^0_i of node (x + c_x, y + c_y)
                sx, sy = (x + cx) % n, (y + cy) % n
                fe = orc.feq(0, float(rho[sy, sx]), (float(u[0, sy, sx]), float(u[1, sy, sx])),
                             float(th[sy, sx]))[k]
                rf, tf = frames[y * n + x]
                fr = orc.feq(0, rf, (0.0, 0.0), 1.0 + tf)[k]
                q = (fe - fr) / L.w[k] - d - (cx * P[y * n + x, 0] + cy * P[y * n + x, 1])
                got = codes[i, y * n + x].view(dt).float().item()
                # the library evaluates f^eq and q in FP32: allow that rounding
                # (relative to the magnitudes that cancel in q) on either side
                slack = 4e-7 * (abs(fe) + abs(fr) + abs(fb[k])) / L.w[k]
                lo = torch.tensor(q - slack, dtype=torch.float64).to(dt).float().item()
                hi = torch.tensor(q + slack, dtype=torch.float64).to(dt).float().item()
                if not (min(lo, hi) <= got <= max(lo, hi)):
                    bad += 1
    assert bad == 0


# ----------------------------------------------------------------- batched


def test_batched_parity_and_self_consistency():
    """The batched workload's first 16 runs as drawn (sizes up to 256^2) over
    its 500-step horizon: each matches the oracle, and the first three are
    bitwise equal to the same run launched alone."""
    import torch
    from paper_2411_10751_amd import holb
    runs = inputs.batched_runs(nruns=16, steps=500)  # run r draws from seed 5 + r: the first 16 of the 512
    steps = runs[0]["steps"]
    log("case batched 16 runs, %d steps" % steps)
    b = holb.Batch([r["config"] for r in runs])
    b.init([r["rho"] for r in runs], [r["u"] for r in runs], [r["theta"] for r in runs])
    b.step(steps)
    for k, r in enumerate(runs):
        gf = [x.cpu().numpy().astype(np.float64) for x in b.fields(k)]
        o = run_oracle(r["config"], r["rho"], r["u"], r["theta"], steps)
        assert_parity(gf, o, 0, TOL[0], r["name"])
        if k < 3:
            # batched runs keep per-plane frames: the same run alone, same frames
            alone = run_gpu(dict(r["config"], frames=2), r["rho"], r["u"], r["theta"], steps)
            for a, bb in zip(gf, alone):
                assert np.array_equal(a, bb)
    torch.cuda.synchronize()


def test_batched_grad_lag():
    """The batched form with the previous step's temperature gradient (one
    launch per step): the first 8 runs of the workload over 300 steps match
    the oracle run with the same reading, and the first two are bitwise equal
    to the same run launched alone."""
    import torch
    from paper_2411_10751_amd import holb
    runs = inputs.batched_runs(nruns=8, steps=300)
    for r in runs:
        r["config"] = dict(r["config"], grad_lag=1)
    steps = runs[0]["steps"]
    log("case batched 8 runs with grad_lag, %d steps" % steps)
    b = holb.Batch([r["config"] for r in runs])
    b.init([r["rho"] for r in runs], [r["u"] for r in runs], [r["theta"] for r in runs])
    b.step(steps)
    for k, r in enumerate(runs):
        gf = [x.cpu().numpy().astype(np.float64) for x in b.fields(k)]
        o = run_oracle(r["config"], r["rho"], r["u"], r["theta"], steps)
        assert_parity(gf, o, 0, TOL[0], r["name"] + " lagged")
        if k < 2:
            alone = run_gpu(dict(r["config"], frames=2), r["rho"], r["u"], r["theta"], steps)
            for a, bb in zip(gf, alone):
                assert np.array_equal(a, bb)
    torch.cuda.synchronize()


def test_batched_graph_replay_matches_eager():
    """Odd and even step counts (graph replay + eager remainder) agree with
    single eager steps, replayed several times."""
    import torch
    from paper_2411_10751_amd import holb
    runs = inputs.batched_runs(nruns=6, nmin=32, nmax=48, steps=7)
    log("case batched graph replay")
    b1 = holb.Batch([r["config"] for r in runs])
    b1.init([r["rho"] for r in runs], [r["u"] for r in runs], [r["theta"] for r in runs])
    b2 = holb.Batch([r["config"] for r in runs])
    b2.init([r["rho"] for r in runs], [r["u"] for r in runs], [r["theta"] for r in runs])
    for rep in range(3):
        b1.step(7)
        for _ in range(7):
            b2.step(1)
        torch.cuda.synchronize()
        for k in range(len(runs)):
            assert torch.equal(b1.fields(k)[0], b2.fields(k)[0]), (rep, k)


def test_batched_launch_shapes_bitwise_identical():
    """Every batched launch shape (work items of 256 to 2048 cells, 2 to 8
    blocks per compute unit) gives bitwise identical fields, on runs that end
    in partial items; the tuner returns one of them; shapes outside the range
    are refused."""
    import torch
    from paper_2411_10751_amd import holb
    runs = inputs.batched_runs(nruns=7, nmin=33, nmax=97, steps=5)
    log("case batched launch shapes, sizes %s" % [r["config"]["nx"] * r["config"]["ny"] for r in runs])
    cfgs = [r["config"] for r in runs]
    fields = lambda r: ([x["rho"] for x in r], [x["u"] for x in r], [x["theta"] for x in r])
    ref = None
    for v in range(12):
        b = holb.Batch(cfgs)
        b.set_variant(v)
        b.init(*fields(runs))
        b.step(5)
        out = [b.fields(k) for k in range(len(runs))]
        torch.cuda.synchronize()
        if ref is None:
            ref = out
        else:
            for k in range(len(runs)):
                for a, c in zip(ref[k], out[k]):
                    assert torch.equal(a, c), (v, k)
        b.close()
    b = holb.Batch(cfgs)
    b.init(*fields(runs))
    assert 0 <= b.tune() < 12
    b.step(5)
    for k in range(len(runs)):
        for a, c in zip(ref[k], b.fields(k)):
            assert torch.equal(a, c), ("tuned", k)
    assert holb.holb_batch_set_variant(b._h, 12) == holb.EUNSUPPORTED
    assert holb.holb_batch_set_variant(b._h, -1) == holb.EUNSUPPORTED
    b.close()


# ----------------------------------------------------------------- variants


@pytest.mark.parametrize("wname", ["rb3d", "rb3d_tall", "periodic3d", "thermal2d", "body2d", "ptensor2d",
                                   "ptensor2d_256"])
def test_variants_bitwise_identical(wname):
    """Every kernel variant (block order) of a configuration gives bitwise
    identical fields, on boxes whose sizes leave partial blocks and on a
    256-wide grid whose blocks each lie in one row."""
    import torch
    from paper_2411_10751_amd import holb
    w = {"rb3d": lambda: _rb(40, 24, 6),
         "rb3d_tall": lambda: _rb(36, 150, 3),
         "periodic3d": lambda: _rb(36, 70, 3, walls=0),
         "thermal2d": lambda: inputs.thermal_2d(n=300, steps=6),
         "body2d": lambda: inputs.body_force_2d(n=130, steps=6),
         "ptensor2d": lambda: inputs.ptensor_2d(n=200, steps=6, ndrops=4, rmin=10, rmax=20),
         "ptensor2d_256": lambda: inputs.ptensor_2d(n=256, steps=6, ndrops=4, rmin=10, rmax=20)}[wname]()
    sim = holb.Sim(w["config"])
    nv = sim.num_variants()
    sim.close()
    log("case variants %s: %d variants" % (wname, nv))
    ref = None
    for v in range(nv):
        try:
            g = run_gpu(w["config"], w["rho"], w["u"], w["theta"], 6, variant=v)
        except holb.HolbError as e:
            assert e.code == holb.EUNSUPPORTED
            continue
        if ref is None:
            ref = g
        else:
            for a, b in zip(g, ref):
                assert np.array_equal(a, b), (wname, v)
    torch.cuda.synchronize()
