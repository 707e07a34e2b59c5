"""Build step of the HIP library: compiles csrc/*.hip for gfx950 with hipcc
into paper_2411_10751_amd/libholb.so (in-tree, so that it travels with the
source tree).  Usage: python -m paper_2411_10751_amd.build

    python -m paper_2411_10751_amd.build --resource-usage [REGEX]

compiles the kernel units once more with the compiler's resource-usage
remarks and prints, per kernel whose name matches REGEX, its vector
registers, accumulation registers, scratch bytes per lane and the waves per
SIMD they allow (nothing is linked).
"""
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libholb.so")
SOURCES = ["holb_inst_d3_f32.hip", "holb_inst_d3_16.hip", "holb_inst_d2_f32.hip", "holb_inst_d2_16.hip",
           "holb_kernels.hip", "holb_capi.hip", "holb_batch.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # code-object v5 loads on the HIP runtime bundled with PyTorch as well
    "-mcode-object-version=5",
    # reproducible arithmetic: no implicit contraction (fmaf() is explicit)
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def build(verbose=False, jobs=7):
    """Compile every source and link the shared library; always rebuilds."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc()] + HIPCC_FLAGS + ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if verbose and err:
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-mcode-object-version=5", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


PROBE_SRC = os.path.join(HERE, "ceiling_probe.hip")
PROBE = os.path.join(HERE, "ceiling_probe")


def build_probe():
    """Compile the memory-ceiling probe (a stand-alone measurement program)."""
    cmd = [hipcc(), "-O3", "-std=c++17", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", PROBE_SRC, "-o", PROBE + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (PROBE_SRC, r.stderr))
    os.replace(PROBE + ".tmp", PROBE)
    return PROBE


def resource_usage(pattern=".", jobs=4):
    """[(kernel, VGPRs, AGPRs, scratch bytes per lane, waves per SIMD)] of the
    kernels whose demangled name matches `pattern`."""
    objdir = os.path.join(HERE, "_build", "ru")
    os.makedirs(objdir, exist_ok=True)

    def one(src):
        cmd = [hipcc()] + HIPCC_FLAGS + ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o",
                                         os.path.join(objdir, src.replace(".hip", ".o")),
                                         "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr))
        found, name = {}, None
        for line in r.stderr.splitlines():
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                found[name] = {}
                continue
            m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
            if m and name:
                found[name][m.group(1).split()[0]] = int(m.group(2))
        return found

    units = [s for s in SOURCES if s.startswith("holb_inst_") or s == "holb_batch.hip"]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        merged = {}
        for d in ex.map(one, units):
            merged.update(d)
    names = list(merged)
    dem = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True).stdout.split("\n")
    out = []
    for n, dm in zip(names, dem):
        short = dm.split("(")[0].replace("void ", "").replace("holb::", "").replace(" ", "")
        if re.search(pattern, short):
            v = merged[n]
            out.append((short, v.get("VGPRs"), v.get("AGPRs"), v.get("ScratchSize"), v.get("Occupancy")))
    return sorted(out)


if __name__ == "__main__":
    if "--resource-usage" in sys.argv:
        rest = sys.argv[sys.argv.index("--resource-usage") + 1:]
        print("| kernel | VGPRs | AGPRs | scratch B/lane | waves/SIMD |")
        print("|---|---|---|---|---|")
        for row in resource_usage(rest[0] if rest else "."):
            print("| `%s` | %s | %s | %s | %s |" % row)
    else:
        print(build(verbose="-v" in sys.argv))
        print(build_probe())
