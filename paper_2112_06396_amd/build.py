"""Build libhks.so (HIP for gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(the key-switch path has no floating-point arithmetic and the encoder's is
fp64; the flag keeps the compiler from forming packed FP32 ops anywhere).
"""
import hashlib
import re
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhks.so")
SOURCES = ["ntt.hip", "ntt_cols.hip", "ntt_rows_fwd.hip", "ntt_rows_inv.hip", "ksk.hip", "kernels.hip", "tables.cpp",
           "abi.cpp", "ks32.hip", "ctx32.cpp"]
# the files that define the 64-bit kernels and their launch shapes (host
# orchestration excluded): counter summaries are valid for one hash of them
KERNEL_SOURCES = ["ntt_device.h", "pass_shapes.h", "ntt.hip", "ntt_cols.hip", "ntt_rows_fwd.hip", "ntt_rows_inv.hip",
                  "ksk.hip", "kernels.hip", "modarith.h", "device_util.h", "hks_internal.h"]


def _code_only(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed
    (no kernel source holds a string literal containing comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash() -> str:
    """Hash of the code (comments and layout excluded) of KERNEL_SOURCES."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
            h.update(b"\0")
    return h.hexdigest()[:16]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str = LIB, src_dir: str = CSRC, extra_flags=()) -> str:
    """Compile SOURCES from src_dir into the shared library `out`."""
    bdir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build", os.path.basename(out) + ".d")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC, *FLAGS, *extra_flags, *lang, "-c", os.path.join(src_dir, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        log, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n{log}\n")
        elif verbose and log.strip():
            sys.stderr.write(log)
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
