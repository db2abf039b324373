"""The lattice pass's 1-D kernel weights (delta_weights in csrc/lbib_device.h), compiled for
the host, against the kernels' closed forms in FP64: the cosine kernel's (sine and cosine
from Taylor series in the device code) and Peskin's 4-point kernel's, over 20001 offsets
s in [0, 1). Bars: every weight within 2e-7 of the closed form (a few FP32 roundings of
values below 1/2), and the even and odd sums equal to 1/2 within the same."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_06726_amd", "csrc")

SRC = r"""
#include "lbib_device.h"
#include <cstdio>
int main() {
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i <= 20000; ++i) {
            const float s = (float)i / 20001.0f;
            float w[4];
            lbib::delta_weights(k, s, w);
            std::printf("%d %.9g %.9g %.9g %.9g %.9g\n", k, s, w[0], w[1], w[2], w[3]);
        }
    return 0;
}
"""


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def closed_form(kernel, s):
    if kernel == 0:      # cosine kernel, phi(r) = (1 + cos(pi r / 2)) / 4 for |r| <= 2
        r = np.stack([s + 1, s, s - 1, s - 2])
        return 0.25 * (1 + np.cos(np.pi * r / 2))
    q = np.sqrt(1 + 4 * s - 4 * s * s)
    return np.stack([(3 - 2 * s - q) / 8, (3 - 2 * s + q) / 8, (1 + 2 * s + q) / 8, (1 + 2 * s - q) / 8])


@pytest.mark.skipif(_hipcc() is None, reason="hipcc is needed to compile the device header for the host")
def test_kernel_weights_match_closed_forms():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "weights.cpp")
        exe = os.path.join(d, "weights")
        with open(src, "w") as f:
            f.write(SRC)
        subprocess.run([_hipcc(), "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    a = np.array([[float(v) for v in line.split()] for line in out.splitlines()])
    for k in (0, 1):
        rows = a[a[:, 0] == k]
        s, w = rows[:, 1], rows[:, 2:].T
        ref = closed_form(k, s)
        assert np.max(np.abs(w - ref)) <= 2e-7, (k, np.max(np.abs(w - ref)))
        assert np.max(np.abs(w[0] + w[2] - 0.5)) <= 2e-7
        assert np.max(np.abs(w[1] + w[3] - 0.5)) <= 2e-7
