"""Build libbhfwi.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("bhfwi_host.hip", "bhfwi_semblance.hip")]
OUT = os.path.join(HERE, "libbhfwi.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
]


def source_files():
    """Every file the library is compiled from: the HIP sources and headers
    under csrc/ and the C-ABI header."""
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                   glob.glob(os.path.join(HERE, "csrc", "*.h")))
    return files + [os.path.join(ROOT, "include", "bhfwi.h")]


def source_id() -> str:
    """SHA-256 (hex) over the names and contents of source_files(); compiled
    into the library as its build id (bhfwi_build_id)."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = (["hipcc"] + HIPCC_FLAGS + ['-DBHFWI_BUILD_ID="%s"' % source_id(), "-o", tmp] +
           SRCS)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libbhfwi.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
