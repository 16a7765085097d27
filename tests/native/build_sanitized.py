"""Builds tests/native/host_checks.cpp against the library sources with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (device code as in the library build) into
_build/host_checks, reusing the library's device objects' compiler flags.

    python tests/native/build_sanitized.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_1507_05925_amd import build as lib_build  # noqa: E402

# every -fsanitize= goes to the host pass only (the device code is not instrumented)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
HOST_SOURCES = ("capi.cpp", "gmres.cpp", "batch.cpp", "server.cpp", "checks.cpp", "autotune.cpp",
                "profile.cpp")


def build(jobs=8):
    out = os.path.join(ROOT, "_build", "host_checks")
    os.makedirs(out, exist_ok=True)
    procs, objs = [], []
    paths = [os.path.join(lib_build.CSRC, src) for src in lib_build.SOURCES]
    for path in paths + [os.path.join(HERE, "host_checks.cpp")]:
        obj = os.path.join(out, os.path.basename(path) + ".o")
        objs.append(obj)
        host = os.path.basename(path) in HOST_SOURCES or path.endswith("host_checks.cpp")
        lang = ["-x", "hip"] if path.endswith(".cpp") else []
        cmd = [lib_build.hipcc(), *lib_build.HIP_FLAGS, *(SAN if host else []), *lang, "-c", path,
               "-o", obj]
        procs.append((path, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = [(p, pr.communicate()[0].decode()) for p, pr in procs]
    failed = [(p, t) for (p, t), (_, pr) in zip(failed, procs) if pr.returncode != 0]
    if failed:
        raise RuntimeError("\n".join(f"--- {p}\n{t}" for p, t in failed))
    exe = os.path.join(out, "host_checks")
    subprocess.check_call([lib_build.hipcc(), "--offload-arch=gfx950", *SAN, *objs, "-o", exe,
                           "-lpthread"])
    return exe


if __name__ == "__main__":
    print(build())
