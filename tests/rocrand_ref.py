"""rocRAND's host implementation of Philox4x32-10, an independent reference
for the oracle's generator.

A small host program (no device code) built with hipcc against the rocRAND
header: for each (counter, key) it seeds the engine with the key, skips to
the counter's high half as the subsequence and to its low half as the
block offset, and prints the block.  ``blocks()`` returns None when the
compiler or the header is missing.
"""
import atexit
import os
import shutil
import subprocess
import tempfile

import numpy as np

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned c[4], k[2];
    while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        const unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        const unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
        rocrand_device::philox4x32_10_engine e(seed, sub, 0ull);
        unsigned long long a = ((unsigned long long)c[1] << 32) | c[0];
        while (a) {
            const unsigned long long s = a < (1ull << 61) ? a : (1ull << 61);
            e.discard(4ull * s);
            a -= s;
        }
        const uint4 v = e.next4();
        printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
"""

_exe = None


def _build():
    global _exe
    if _exe is not None:
        return _exe or None
    _exe = ""
    if not (os.path.exists(HIPCC) and os.path.exists(HEADER)):
        return None
    d = tempfile.mkdtemp(prefix="rocrand_ref_")
    atexit.register(shutil.rmtree, d, True)
    src = os.path.join(d, "philox_ref.cpp")
    exe = os.path.join(d, "philox_ref")
    with open(src, "w") as f:
        f.write(SRC)
    r = subprocess.run([HIPCC, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        shutil.rmtree(d, ignore_errors=True)
        return None
    _exe = exe
    return exe


def blocks(counters, keys):
    """Philox4x32-10 blocks [n][4] (uint32) for counters [n][4] and keys [n][2]."""
    exe = _build()
    if exe is None:
        return None
    lines = "".join("%08x %08x %08x %08x %08x %08x\n" % (tuple(int(v) for v in c) + tuple(int(v) for v in k))
                    for c, k in zip(counters, keys))
    out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w, 16) for w in l.split()] for l in out.strip().splitlines()], dtype=np.uint32)
