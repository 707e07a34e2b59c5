"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every declared entry point, its lattice tables agree with the oracle's own
derivation, and configuration/argument errors are reported."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import orc
from paper_2411_10751_amd import holb, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "holb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(holb_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(holb.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("lattice", [0, 1])
def test_lattice_tables_match_oracle(lattice):
    """The library's tables (solved by its own generator) equal the oracle's
    independently derived velocity set and weights."""
    c, w, c0sq = holb.lattice_info(lattice)
    L = orc.Lattice(lattice)
    assert c.shape[0] == L.Q
    lib = {tuple(v): x for v, x in zip(c.tolist(), w)}
    ref = {tuple(v): x for v, x in zip(L.c.tolist(), L.w)}
    assert lib.keys() == ref.keys()
    for k in ref:
        assert abs(lib[k] - ref[k]) < 1e-13 * ref[k] + 1e-16
    assert abs(c0sq - L.c0sq) < 1e-14
    # pairing convention: 0 is rest, then (+c, -c)
    assert np.all(c[0] == 0)
    assert np.all(c[1::2] == -c[2::2])


def _cfg(**kw):
    base = dict(lattice=0, nx=32, ny=32, nz=1, tau_hat=0.8, sources=1, g=(0, 1e-5, 0))
    base.update(kw)
    return base


@pytest.mark.parametrize("bad,code", [
    (dict(tau_hat=0.5), holb.EINVAL),
    (dict(tau_hat=float("nan")), holb.EINVAL),
    (dict(nx=0), holb.EINVAL),
    (dict(nz=4), holb.EINVAL),
    (dict(lattice=7), holb.EINVAL),
    (dict(sources=8), holb.EINVAL),
    (dict(sources=2, isothermal=1), holb.EUNSUPPORTED),
    (dict(sources=2, prandtl=0.0), holb.EINVAL),
    (dict(sources=4, isothermal=0, eos_a=0.1, eos_b=0.1, eos_T=0.5), holb.EUNSUPPORTED),
    (dict(sources=4, isothermal=1, eos_a=0.1, eos_b=0.0, eos_T=0.5), holb.EINVAL),
    (dict(sources=4, isothermal=1, eos_a=0.1, eos_b=0.1, eos_T=0.5, walls=1), holb.EUNSUPPORTED),
    (dict(sources=4, isothermal=1, eos_a=0.1, eos_b=0.1, eos_T=0.5, eos=2), holb.EINVAL),
    (dict(storage=5), holb.EINVAL),
    (dict(storage=1, rho0=0.0), holb.EINVAL),
    (dict(walls=1, ny=6), holb.EINVAL),
    (dict(g=(float("inf"), 0, 0)), holb.EINVAL),
    (dict(lattice=1, nx=1024, ny=1024, nz=1024), holb.ESIZE),
    (dict(frames=4), holb.EINVAL),
    (dict(storage=0, frames=3), holb.EUNSUPPORTED),
    (dict(sources=2, prandtl=0.7, grad_lag=2), holb.EINVAL),
    (dict(sources=1, grad_lag=1), holb.EINVAL),
])
def test_config_errors(bad, code):
    with pytest.raises(holb.HolbError) as ei:
        holb.workspace_size(_cfg(**bad))
    assert ei.value.code == code


def test_abi_version_checked():
    c = holb.make_config(_cfg())
    c.abi_version = 99
    n = ctypes.c_size_t()
    assert holb.holb_workspace_size(ctypes.byref(c), ctypes.byref(n)) == holb.EINVAL
    assert "abi_version" in holb.last_error()


def test_workspace_size_covers_populations():
    for lat, dims, st in [(0, (64, 48, 1), 0), (1, (16, 12, 10), 0), (1, (16, 12, 10), 2)]:
        cfg = _cfg(lattice=lat, nx=dims[0], ny=dims[1], nz=dims[2], storage=st)
        Q = 37 if lat == 0 else 39
        N = dims[0] * dims[1] * dims[2]
        assert holb.workspace_size(cfg) >= 2 * Q * N * (4 if st == 0 else 2)


def test_create_is_host_only_and_checks_workspace():
    """holb_create launches nothing: argument errors and a successful bind can
    be exercised without a GPU (the workspace address is never dereferenced)."""
    cfg = holb.make_config(_cfg(frames=1))
    need = ctypes.c_size_t()
    assert holb.holb_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == holb.OK
    h = ctypes.c_void_p()
    fake = 1 << 40  # 256-byte aligned, never touched
    assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(fake + 16), need.value, None,
                            ctypes.byref(h)) == holb.ESIZE
    assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(fake), need.value - 256, None,
                            ctypes.byref(h)) == holb.ESIZE
    assert holb.holb_create(ctypes.byref(cfg), None, need.value, None, ctypes.byref(h)) == holb.EINVAL
    assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(fake), need.value, None,
                            ctypes.byref(h)) == holb.OK
    assert holb.holb_step(h, 1) == holb.ESTATE  # not initialised: nothing launched
    assert holb.holb_step(h, -1) == holb.EINVAL
    n = ctypes.c_int32()
    assert holb.holb_num_variants(h, ctypes.byref(n)) == holb.OK and n.value >= 1
    assert holb.holb_set_variant(h, 10 ** 6) == holb.EUNSUPPORTED
    sb = ctypes.c_size_t()
    assert holb.holb_state_bytes(h, ctypes.byref(sb)) == holb.OK
    # Q planes + one frame (2 x binary16) per cell (per-cell frames)
    assert sb.value == 37 * 1024 * 4 + 1024 * 4
    assert holb.holb_get_state(h, ctypes.c_void_p(fake), sb.value - 4) == holb.ESIZE
    assert holb.holb_set_state(h, ctypes.c_void_p(fake), sb.value + 4) == holb.ESIZE
    assert holb.holb_timing_stop(h, None, None, None, None, 0) == holb.OK  # nothing timed: no event touched
    assert holb.holb_destroy(h) == holb.OK


@pytest.mark.parametrize("walls,storage,frames,per_cell", [
    (1, 0, 0, 0), (1, 0, 1, 4), (0, 0, 0, 0), (0, 0, 1, 4), (0, 0, 2, 0), (1, 1, 0, 0), (0, 1, 0, 8), (0, 2, 0, 4), (1, 2, 0, 4),
    (0, 1, 3, 8), (0, 2, 1, 4), (0, 2, 3, 8), (1, 1, 2, 0), (1, 2, 2, 0)])
def test_state_layout_by_frame_mode(walls, storage, frames, per_cell):
    """The raw state holds the Q planes, then per_cell bytes of frame words per
    cell (4 for per-cell frames, 8 with momentum, in two planes) or the per-plane table of
    2 + 7 NS floats per plane; with the body and thermal sources AUTO picks
    per-plane frames for FP32 and for FP16 with walls, momentum frames for
    periodic FP16 and per-cell frames for BF16."""
    nx, ny, nz = 24, 20, 15  # N = 7200: the frame planes need padding
    cfg = holb.make_config(dict(lattice=1, nx=nx, ny=ny, nz=nz, tau_hat=0.8, sources=3, prandtl=0.7,
                                g=(0, 0, -1e-5), walls=walls, storage=storage, frames=frames, rho0=1.0,
                                theta0=1.0))
    need = ctypes.c_size_t()
    assert holb.holb_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == holb.OK
    h = ctypes.c_void_p()
    assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 40), need.value, None, ctypes.byref(h)) == holb.OK
    sb = ctypes.c_size_t()
    assert holb.holb_state_bytes(h, ctypes.byref(sb)) == holb.OK
    N = nx * ny * nz
    elem = 4 if storage == 0 else 2
    pitch = -(-N // (256 // elem)) * (256 // elem)
    # frame plane (and momentum plane), each padded to 256 bytes
    extra = (-(-N * 4 // 256) * 256) * (per_cell // 4) if per_cell else (2 + 7 * 6) * nz * 4
    # walls: the next step's targets, (D + 2) doubles per cell of the 3 + 3 wall
    # layers, and the starting point (D + 2) and Jacobian factors (16) of the
    # two wall-node solves
    targets = (8 * 5 + 2 * 16) * nx * ny * 8 if walls else 0
    assert sb.value == 39 * pitch * elem + extra + targets
    assert holb.holb_destroy(h) == holb.OK


def test_batch_validation_host_only():
    runs = inputs.batched_runs(nruns=5, nmin=32, nmax=40)
    arr = (holb.holb_config * 5)(*[holb.make_config(r["config"]) for r in runs])
    n = ctypes.c_size_t()
    assert holb.holb_batch_workspace_size(arr, 5, ctypes.byref(n)) == holb.OK
    cells = sum(r["config"]["nx"] * r["config"]["ny"] for r in runs)
    assert n.value >= 2 * 37 * cells * 4
    bad = (holb.holb_config * 2)(holb.make_config(runs[0]["config"]),
                                 holb.make_config(dict(runs[1]["config"], lattice=1, nz=8)))
    assert holb.holb_batch_workspace_size(bad, 2, ctypes.byref(n)) == holb.EUNSUPPORTED
    mixed = (holb.holb_config * 2)(holb.make_config(runs[0]["config"]),
                                   holb.make_config(dict(runs[1]["config"], sources=1)))
    assert holb.holb_batch_workspace_size(mixed, 2, ctypes.byref(n)) == holb.EUNSUPPORTED
    assert holb.holb_batch_workspace_size(arr, 0, ctypes.byref(n)) == holb.EINVAL


def test_fastdiv_exact(tmp_path):
    """The division by a runtime constant used for cell coordinates equals
    integer division for every divisor up to 4096 and, for large divisors,
    on dividends spread over [0, 2^31)."""
    src = tmp_path / "fd.cpp"
    src.write_text(r'''
#include <cstdio>
#include "holb_params.h"
using namespace holb;
int main() {
    unsigned long long bad = 0;
    for (unsigned d = 1; d <= 4096; ++d) {
        const FastDiv f = make_fastdiv(d);
        for (unsigned n = 0; n < 300000; ++n) bad += fastdiv(n, f) != n / d;
        for (unsigned n = (1u << 31) - 70000; n < (1u << 31); ++n) bad += fastdiv(n, f) != n / d;
    }
    unsigned s = 12345u;
    for (int k = 0; k < 2000000; ++k) {
        s = s * 1664525u + 1013904223u;
        const unsigned d = (s >> 1) % ((1u << 30) - 1) + 1;
        s = s * 1664525u + 1013904223u;
        const unsigned n = s >> 1;
        bad += fastdiv(n, make_fastdiv(d)) != n / d;
    }
    printf("%llu\n", bad);
    return bad != 0;
}
''')
    exe = tmp_path / "fd"
    inc = os.path.join(ROOT, "paper_2411_10751_amd", "csrc")
    subprocess.run(["g++", "-O2", "-D__host__=", "-D__device__=", "-I" + inc, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout


def test_periodic_wrap_exact(tmp_path):
    """The periodic wrap of the stencils (one select each way, a loop only on
    axes shorter than the reach) equals the mathematical modulo for every
    offset the stencils use (up to 3 cells past either edge) on every axis
    length from 1 to 300, as does the loop form used on edge waves."""
    text = open(os.path.join(ROOT, "paper_2411_10751_amd", "csrc", "holb_device.h")).read()
    funcs = []
    for name in ("wrapc", "wrap_seq"):
        start = text.index("__device__ __forceinline__ int %s(int v, int n)" % name)
        end = text.index("\n}\n", start) + 3
        funcs.append(text[start:end])
    src = tmp_path / "wrap.cpp"
    src.write_text("#include <cstdio>\n#define __device__\n#define __forceinline__ inline\n" + "".join(funcs) + r'''
int main() {
    unsigned long long bad = 0, n_cases = 0;
    for (int n = 1; n <= 300; ++n)
        for (int x = 0; x < n; ++x)
            for (int c = -3; c <= 3; ++c) {
                const int v = x + c, m = ((v % n) + n) % n;
                bad += wrapc(v, n) != m;
                bad += wrap_seq(v, n) != m;
                ++n_cases;
            }
    printf("%llu %llu\n", bad, n_cases);
    return bad != 0;
}
''')
    exe = tmp_path / "wrap"
    subprocess.run(["g++", "-O2", str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.split()[0] == "0", r.stdout


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: asked for more it exits with status 2 and
    says so, before touching a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_bench_traffic_needs_matching_profile(tmp_path, monkeypatch):
    """bench.py reports the profiled HBM traffic only for the kernel, block
    order and kernel sources its counter summary records."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_2411_10751_amd.profile_summary import source_sha256
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_rb3d_f32.txt").write_text(
        "# HBM traffic per launch of the dominant kernel, test, variant 3\n"
        "kernel: k_step<D3Q39,0,1,false,1>\nsource_sha256: %s\nhbm_bytes_per_launch: 1234\n" % source_sha256())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("k_step<D3Q39,0,1,false,1>", "rb3d", 0, 3) == 1234.0
    assert bench.traffic_from_profile("k_step<D3Q39,0,1,false,1>", "rb3d", 0, 0) is None
    assert bench.traffic_from_profile("k_aux<D3Q39,0,1,false,1>", "rb3d", 0, 3) is None
    assert bench.traffic_from_profile("k_step<D3Q39,0,1,false,1>", "rb3d", 1, 3) is None
    (prof / "traffic_rb3d_f32.txt").write_text(
        "# title, variant 3\nkernel: k_step<D3Q39,0,1,false,1>\nsource_sha256: 0\nhbm_bytes_per_launch: 1\n")
    assert bench.traffic_from_profile("k_step<D3Q39,0,1,false,1>", "rb3d", 0, 3) is None


def test_profile_overlap_accounting():
    """Kernel summaries: the time each kernel ran with no other on the device
    and the device's busy time, from dispatch intervals (ns)."""
    from paper_2411_10751_amd.profile_summary import _overlap
    trace = [
        {"Kernel_Name": "void holb::k_aux<D3Q39, 0, 1, false, 1>(holb::KParams)", "Start_Timestamp": "0",
         "End_Timestamp": "100"},
        {"Kernel_Name": "void holb::k_wall_fluid<D3Q39, 0, 1>(holb::KParams)", "Start_Timestamp": "10",
         "End_Timestamp": "120"},
        {"Kernel_Name": "void holb::k_step<D3Q39, 0, 1, false, 1>(holb::KParams)", "Start_Timestamp": "200",
         "End_Timestamp": "300"},
    ]
    alone, busy = _overlap(trace)
    assert busy == 120 + 100
    assert alone["k_aux<D3Q39,0,1,false,1>"] == 10
    assert alone["k_wall_fluid<D3Q39,0,1>"] == 20
    assert alone["k_step<D3Q39,0,1,false,1>"] == 100


def test_profile_traffic_scaling(tmp_path):
    """Traffic summaries: each counter's mean per dispatch of the kernel,
    scaled by what the same counter reads for the calibration dispatch of
    1 GiB in and 1 GiB out, compared with the algorithmic bytes."""
    import sys
    from paper_2411_10751_amd import profile_summary as ps

    def run(d, counter, rows):
        (tmp_path / d).mkdir()
        lines = ["Kernel_Name,Counter_Name,Counter_Value"] + ["\"%s\",%s,%s" % (k, counter, v) for k, v in rows]
        (tmp_path / d / "p_counter_collection.csv").write_text("\n".join(lines) + "\n")

    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>(int)"
    kern = "void holb::k_step<D3Q39, 0, 1, false, 1>(holb::KParams)"
    # FETCH_SIZE reads half the calibration bytes, WRITE_SIZE all of them
    run("fetch", "FETCH_SIZE", [(neg, 524288.0), (kern, 1000.0), (kern, 1200.0)])
    run("write", "WRITE_SIZE", [(neg, 1048576.0), (kern, 2000.0)])
    out = tmp_path / "traffic.txt"
    argv = sys.argv
    sys.argv = ["x", "traffic", str(tmp_path / "fetch"), str(tmp_path / "write"), str(out),
                "--kernel", "k_step<D3Q39,0,1,false,1>", "--cells", "100", "--bytes-per-cell", "312",
                "--cmd", "a", "--cmd", "b", "--title", "test, variant 0"]
    try:
        ps.main()
    finally:
        sys.argv = argv
    vals = dict(l.split(": ", 1) for l in out.read_text().splitlines() if not l.startswith("#"))
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    hbm = 1100.0 * 1024 * 2.0 + 2000.0 * 1024
    assert float(vals["hbm_bytes_per_launch"]) == pytest.approx(hbm, abs=0.5)
    assert int(vals["algorithmic_bytes_per_launch"]) == 31200
    assert vals["source_sha256"] == ps.source_sha256()


def test_grad_lag_state_and_batches_host_only():
    """With the previous step's gradient the state carries the theta field the
    next step reads (N floats more); a batch takes the option when all its
    runs share it (its workspace holds a second theta field) and refuses a
    mix."""
    base = _cfg(sources=3, prandtl=0.7)
    sizes = []
    for lag in (0, 1):
        cfg = holb.make_config(dict(base, grad_lag=lag))
        need = ctypes.c_size_t()
        assert holb.holb_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == holb.OK
        h = ctypes.c_void_p()
        assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 40), need.value, None,
                                ctypes.byref(h)) == holb.OK
        sb = ctypes.c_size_t()
        assert holb.holb_state_bytes(h, ctypes.byref(sb)) == holb.OK
        sizes.append(sb.value)
        assert holb.holb_destroy(h) == holb.OK
    assert sizes[1] - sizes[0] == 32 * 32 * 4
    nb = []
    for lag in (0, 1):
        arr = (holb.holb_config * 2)(*[holb.make_config(dict(base, grad_lag=lag))] * 2)
        n = ctypes.c_size_t()
        assert holb.holb_batch_workspace_size(arr, 2, ctypes.byref(n)) == holb.OK
        nb.append(n.value)
    assert nb[1] - nb[0] >= 2 * 32 * 32 * 4
    mixed = (holb.holb_config * 2)(holb.make_config(dict(base, grad_lag=0)), holb.make_config(dict(base, grad_lag=1)))
    n = ctypes.c_size_t()
    assert holb.holb_batch_workspace_size(mixed, 2, ctypes.byref(n)) == holb.EUNSUPPORTED


@pytest.mark.parametrize("storage,sources,per_cell", [(0, 4, 4), (0, 1, 0), (1, 4, 4), (1, 1, 0), (1, 2, 8),
                                                      (2, 1, 4), (2, 4, 4)])
def test_auto_frames_periodic_by_source(storage, sources, per_cell):
    """AUTO on a periodic domain: FP32 and FP16 keep one frame per plane (no
    frame words) except with the pressure-tensor source, whose liquid and
    vapour share planes (per-cell frames, 4 bytes per cell), and FP16 with the
    thermal source (momentum frames, 8 bytes per cell); BF16 keeps per-cell
    frames."""
    nx, ny, nz = 16, 16, 12
    iso = 1 if sources & 4 else 0
    cfg = holb.make_config(dict(lattice=1, nx=nx, ny=ny, nz=nz, tau_hat=0.8, sources=sources, isothermal=iso,
                                g=(0, 0, -1e-5), eos_a=9.0 / 49.0, eos_b=2.0 / 21.0, eos_T=0.05, sc_G=-1.0,
                                ptensor_k=0.5, storage=storage, frames=0, rho0=1.0, theta0=1.0))
    need = ctypes.c_size_t()
    assert holb.holb_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == holb.OK, holb.last_error()
    h = ctypes.c_void_p()
    assert holb.holb_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 40), need.value, None, ctypes.byref(h)) == holb.OK
    sb = ctypes.c_size_t()
    assert holb.holb_state_bytes(h, ctypes.byref(sb)) == holb.OK
    N = nx * ny * nz
    elem = 4 if storage == 0 else 2
    pitch = -(-N // (256 // elem)) * (256 // elem)
    extra = (-(-N * 4 // 256) * 256) * (per_cell // 4) if per_cell else (2 + 7 * 6) * nz * 4
    assert sb.value == 39 * pitch * elem + extra
    assert holb.holb_destroy(h) == holb.OK
