"""Build of the HIP library liberi_hip.so (gfx950).

Steps: generate the Boys table and the class kernels into _build/gen, compile
every translation unit with hipcc in parallel, link the shared library into
the package directory (where the Python binding loads it).
"""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
GEN = os.path.join(BUILD, "gen")
OBJ = os.path.join(BUILD, "obj")
LIB = os.path.join(PKG, "liberi_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CXXFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + GEN,
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def _digest(paths, extra=""):
    h = hashlib.sha1(extra.encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _compile(src, obj, deps):
    stamp = obj + ".sha"
    dig = _digest([src] + deps, " ".join(CXXFLAGS))
    if os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == dig:
        return obj, 0.0, False
    t0 = time.time()
    cmd = [HIPCC] + CXXFLAGS + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    os.replace(obj + ".tmp", obj)
    with open(stamp, "w") as f:
        f.write(dig)
    return obj, time.time() - t0, True


def build(jobs=None, verbose=True, precisions=("fp64", "mixed", "rys", "rys32"), classes=None):
    sys.path.insert(0, CSRC)
    import codegen  # noqa: E402
    import gen_boys_table  # noqa: E402
    import gen_rys_table  # noqa: E402
    sys.path.pop(0)
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    bt = os.path.join(GEN, "boys_table.h")
    if not os.path.exists(bt):
        gen_boys_table.write(bt)
    # the Rys rule's tables (about 30 s of 40-digit arithmetic): rewritten when
    # their generator changes
    rt = os.path.join(GEN, "rys_table.h")
    rstamp = rt + ".sha"
    rdig = _digest([os.path.join(CSRC, "gen_rys_table.py")])
    if ("rys" in precisions or "rys32" in precisions) and not (os.path.exists(rt) and os.path.exists(rstamp) and open(rstamp).read() == rdig):
        err = gen_rys_table.write(rt)
        with open(rstamp, "w") as f:
            f.write(rdig)
        if verbose:
            print("  Rys rule tables: max relative error %.2e" % err, flush=True)
    files, _ = codegen.generate(GEN, precisions=precisions, classes=classes)
    # generated kernel TUs see the device headers only; the host TUs also the
    # plan internals and the C ABI header
    kdeps = [os.path.join(CSRC, f) for f in ("eri_device.h", "eri_plan_types.h", "eri_dispatch.h")] + [bt]
    hdeps = kdeps + [os.path.join(CSRC, "eri_internal.h"), os.path.join(ROOT, "include", "eri.h")]
    host = [os.path.join(CSRC, "eri_lib.hip"), os.path.join(CSRC, "eri_backward.hip")]
    srcs = files + host
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = []
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {}
        rdeps = kdeps + [os.path.join(CSRC, "eri_rys.h"), os.path.join(GEN, "rys_table.h")]
        for s in srcs:
            obj = os.path.join(OBJ, os.path.basename(s) + ".o")
            deps = hdeps if s in host else (rdeps if os.path.basename(s).startswith("eri_rys") else kdeps)
            futs[ex.submit(_compile, s, obj, deps)] = s
        for fu in cf.as_completed(futs):
            obj, dt, did = fu.result()
            objs.append(obj)
            if verbose and did:
                print("  compiled %-40s %6.1fs" % (os.path.basename(futs[fu]), dt), flush=True)
    objs.sort()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-6000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


if __name__ == "__main__":
    build()
