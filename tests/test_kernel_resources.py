"""Register budgets of the traversal kernels, checked at compile time (no
GPU): the persistent kernels must keep the occupancy they are tuned for
(mixed: 3 waves per SIMD, <= 168 VGPRs; FP64: 4 waves, <= 128; the transport
kernels of both modes: 3 waves), since a few extra registers cut the rays in
flight by a third or a half."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1310_1854_amd import build_lib

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")

WANT = {
    "_ZN12_GLOBAL__N_118k_trace_persistentILi1ELb1ELb0EEEvNS_9TraceArgsE": 3,   # mixed, segments
    "_ZN12_GLOBAL__N_118k_trace_persistentILi0ELb1ELb0EEEvNS_9TraceArgsE": 4,   # FP64, segments
    "_ZN12_GLOBAL__N_118k_trace_persistentILi1ELb1ELb1EEEvNS_9TraceArgsE": 3,   # mixed, transport
    "_ZN12_GLOBAL__N_118k_trace_persistentILi0ELb1ELb1EEEvNS_9TraceArgsE": 3,   # FP64, transport
}


def test_persistent_kernels_keep_their_occupancy(tmp_path):
    src = os.path.join(build_lib.CSRC, "trace.hip")
    flags = [f for f in build_lib.FLAGS if f != "-shared"]
    r = subprocess.run(["hipcc", "-c"] + flags + ["--cuda-device-only", src, "-o", str(tmp_path / "t.o"),
                        "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    occ = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"Occupancy \[waves/SIMD\]: (\d+)", line)
        if m and name:
            occ[name] = int(m.group(1))
    for k, want in WANT.items():
        assert k in occ, f"{k} not compiled"
        assert occ[k] >= want, f"{k}: occupancy {occ[k]} < {want} waves per SIMD"
