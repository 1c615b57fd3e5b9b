"""Build libstencil.so (gfx950 only) in-tree with hipcc.

Every .hip file under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_2406_08923_amd/libstencil.so. Always recompiles: the
build step doubles as the "does it build" check.

The compiler's per-kernel resource report (-Rpass-analysis=kernel-resource-
usage) is collected into _build/kernel_resources.json. A kernel that uses
scratch memory (register spills or private arrays) must be listed in
scratch_kernels.txt beside this file together with the GPU tests that check
it element by element (against the oracle, or bitwise against launches of a
kernel that does not spill); an unlisted one fails the build.
"""
import concurrent.futures as cf
import json
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libstencil.so")
SCRATCH_LIST = os.path.join(HERE, "scratch_kernels.txt")
RESOURCES = os.path.join(OUT_DIR, "kernel_resources.json")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed FP32 instructions (some forms have misbehaved on these parts)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-Rpass-analysis=kernel-resource-usage",
    "-I" + os.path.join(ROOT, "include"),
]

_FN = re.compile(r"remark: Function Name: (\S+)")
_KV = re.compile(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis=kernel-resource-usage\]")


def parse_resources(text):
    """{mangled kernel name: {field: value}} from hipcc's resource remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = _FN.search(line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = _KV.search(line)
        if m and cur is not None:
            out[cur][m.group(1).strip()] = m.group(2)
    return out


def demangle(names):
    names = list(names)
    tool = shutil.which("llvm-cxxfilt", path="/opt/rocm/llvm/bin") or shutil.which("c++filt")
    if not tool or not names:
        return {n: n for n in names}
    r = subprocess.run([tool], input="\n".join(names), capture_output=True, text=True)
    dem = r.stdout.splitlines()
    return dict(zip(names, dem)) if len(dem) == len(names) else {n: n for n in names}


def read_scratch_list(path=SCRATCH_LIST):
    """{demangled kernel: [test ids]} from the scratch allowance list: one
    kernel per line, then ' | ' and the space-separated pytest ids that check
    it; '#' starts a comment."""
    allowed = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            kernel, _, tests = line.partition(" | ")
            allowed[kernel.strip()] = tests.split()
    return allowed


def _compile(src):
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    text = r.stdout + r.stderr
    msgs = "\n".join(l for l in text.splitlines()
                     if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, msgs))
    return obj, msgs, parse_resources(text)


def check_scratch(resources):
    """Raise if a kernel uses scratch memory without a listed test."""
    names = demangle(resources)
    allowed = read_scratch_list()
    bad = []
    for mangled, fields in resources.items():
        if int(fields.get("ScratchSize [bytes/lane]", "0")) > 0:
            d = names[mangled]
            if not allowed.get(d):
                bad.append("%s (%s B/lane)" % (d, fields["ScratchSize [bytes/lane]"]))
    if bad:
        raise RuntimeError("kernels use scratch memory without a listed element-wise test "
                           "(add them to %s):\n  %s" % (SCRATCH_LIST, "\n  ".join(bad)))


def build(verbose=False, jobs=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, srcs))
    resources = {}
    for obj, msgs, res in results:
        if verbose and msgs.strip():
            print(msgs, file=sys.stderr)
        resources.update(res)
    names = demangle(resources)
    with open(RESOURCES, "w") as fh:
        json.dump({names[k]: v for k, v in sorted(resources.items())}, fh, indent=0)
    check_scratch(resources)
    objs = [o for o, _, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    # a kernel whose device code the host pass rejects without a message
    # leaves its launch stub undefined: refuse such a library
    r = subprocess.run(["nm", "-C", "--undefined-only", tmp], capture_output=True, text=True)
    stubs = sorted({l.split("U", 1)[1].strip() for l in r.stdout.splitlines()
                    if "__device_stub__" in l})
    if r.returncode != 0 or stubs:
        raise RuntimeError("kernels without a host launch stub (the host pass dropped them):\n  "
                           + "\n  ".join(stubs or [r.stderr]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
