"""No kernel of the library calls a device function.

The compiler may keep a large device function out of line and reach it by a
call whose return address sits in s[30:31].  In a callee tens of kilobytes
long it has been seen expanding an out-of-range branch through that same
register pair (s_getpc_b64 / s_setpc_b64 s[30:31]) with no save of the
return address, so the callee's return jumps to a wrong address.  Every
helper on the hot path is therefore inlined; this test compiles each source
to gfx950 assembly on the host and checks that no kernel contains a call.
"""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2508_03180_amd import build as hipbuild


def _asm(src, out):
    subprocess.check_call([hipbuild.HIPCC, *hipbuild.FLAGS, "--cuda-device-only", "-S", src, "-o", out],
                          stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


@pytest.mark.skipif(not os.path.exists(hipbuild.HIPCC), reason="needs hipcc")
def test_no_device_function_calls():
    srcs = sorted(os.path.join(hipbuild.CSRC, f) for f in os.listdir(hipbuild.CSRC) if f.endswith(".hip"))
    tmp = tempfile.mkdtemp()
    try:
        with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            asms = list(ex.map(lambda s: _asm(s, os.path.join(tmp, os.path.basename(s) + ".s")), srcs))
    finally:
        shutil.rmtree(tmp)
    for src, asm in zip(srcs, asms):
        assert "s_swappc_b64" not in asm, f"{os.path.basename(src)} calls a device function"
        # a kernel returns by s_endpgm; s_setpc is only the long-branch form
        for line in asm.splitlines():
            if "s_setpc_b64" in line:
                assert "s[30:31]" not in line, f"{os.path.basename(src)}: return through s[30:31]"
