"""Release sequences of the built gfx950 code: the L2 write-back completes
before the atomic that publishes.

A workgroup of the persistent solve publishes a job's results with an
agent-scope release: its XCD's L2 is written back (buffer_wbl2), then an
atomic raises the job's counter, which other XCDs poll.  The atomic may only
be issued once the write-back has completed (s_waitcnt vmcnt(0) in between);
otherwise a consumer that is already polling sees the counter before the data
reaches memory and reads the state from before the write.  The compiler's own
wait after the write-back can be deleted by its wait-count pass, so the
library issues an explicit one.  This test disassembles the device code of
the built library (our own build) and checks every write-back in it.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1303_6615_amd.build import LIB_PATH

OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
ATOMIC = re.compile(r"^\s*(global|flat|buffer)_atomic_\w+")
WAIT_VM0 = re.compile(r"^\s*s_waitcnt\b.*\bvmcnt\(0\)")


def _device_code(tmp_path):
    if not os.path.exists(LIB_PATH):
        pytest.fail("libaparareal.so not built (run python -m paper_1303_6615_amd.build)")
    if not os.path.exists(OBJDUMP):
        pytest.skip("llvm-objdump not available")
    lib = tmp_path / "lib.so"
    shutil.copy(LIB_PATH, lib)
    # extracts each offload bundle next to its input
    subprocess.run([OBJDUMP, "--offloading", str(lib)], check=True, capture_output=True, cwd=tmp_path)
    objs = sorted(p for p in tmp_path.iterdir() if p.name.endswith("gfx950"))
    assert objs, "no gfx950 code object in the library"
    return [subprocess.run([OBJDUMP, "-d", str(p)], check=True, capture_output=True, text=True).stdout
            for p in objs]


def unwaited_releases(asm: str):
    """Write-backs followed by an atomic (or the end of the kernel) with no
    s_waitcnt vmcnt(0) in between; returns their line numbers."""
    lines = asm.splitlines()
    bad = []
    for i, ln in enumerate(lines):
        if "buffer_wbl2" not in ln:
            continue
        for nxt in lines[i + 1:]:
            if WAIT_VM0.search(nxt):
                break
            if ATOMIC.search(nxt) or "s_endpgm" in nxt or "buffer_wbl2" in nxt:
                bad.append(i + 1)
                break
    return bad


def test_checker_flags_an_atomic_right_after_the_write_back():
    assert unwaited_releases("\tbuffer_wbl2 sc1\n\tflat_atomic_add v[0:1], v2\n") == [1]
    assert unwaited_releases("\tbuffer_wbl2 sc1\n\ts_waitcnt vmcnt(0)\n\tflat_atomic_add v[0:1], v2\n") == []
    assert unwaited_releases("\tbuffer_wbl2 sc1\n\ts_waitcnt vmcnt(0) lgkmcnt(0)\n"
                             "\tglobal_atomic_add v1, v0, s[2:3]\n") == []
    assert unwaited_releases("\tbuffer_wbl2 sc1\n\ts_waitcnt vmcnt(1)\n\tglobal_atomic_add v1, v0, s[2:3]\n") == [1]


def test_every_write_back_completes_before_the_publishing_atomic(tmp_path):
    codes = _device_code(tmp_path)
    total = 0
    for asm in codes:
        total += asm.count("buffer_wbl2")
        assert unwaited_releases(asm) == []
    assert total > 0          # the pipeline kernels publish with write-backs
