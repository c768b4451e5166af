"""Structure of the compiled RANSAC kernels (gfx950 assembly, CPU only).

The persistent kernels exchange nothing between workgroups but atomics that
the finish kernel reads after the launch boundary, so they need no cache
write-back or invalidate instructions. Their workgroup barriers must sit in
the persistent loop itself (loop depth 1): a barrier inside a loop nested
within it can be executed a different number of times by different waves,
which is how a missing end-of-item barrier once hung the batched launch."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2402_18008_amd import build

SRC = os.path.join(build.CSRC, "ransac.hip")


def compile_asm(tmp_path):
    try:
        hipcc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    out = tmp_path / "ransac.s"
    cmd = [hipcc, *flags, "--cuda-device-only", "-S", "-I", os.path.join(build.ROOT, "include"),
           "-I", build.CSRC, "-o", str(out), SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def functions(asm):
    names = set(re.findall(r"^\s*\.type\s+(_ZN2hg\S+),@function", asm, re.M))
    for m in re.finditer(r"^(_ZN2hg\S+):", asm, re.M):
        if m.group(1) not in names:        # a device variable, not a function
            continue
        body = asm[m.end():]
        body = body[:body.index(".Lfunc_end")]
        yield m.group(1), body


def barrier_depths(body):
    depth, out = 0, []
    for line in body.splitlines():
        if re.match(r"^\.LBB\d+_\d+:", line):
            d = re.search(r"Depth=(\d+)", line)
            depth = int(d.group(1)) if d else 0
        if "s_barrier" in line:
            out.append(depth)
    return out


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_ransac_kernels_barriers_and_fences(tmp_path):
    asm = compile_asm(tmp_path)
    seen = set()
    for name, body in functions(asm):
        if "ransac_kernel" in name and "Lb1E" in name:          # persistent forms
            seen.add("persistent")
            d = barrier_depths(body)
            assert d and max(d) <= 1, (name, d)
        if "ransac_kernel" in name or "ransac_finish_kernel" in name:
            seen.add("any")
            assert "buffer_wbl2" not in body and "buffer_inv" not in body, name
    assert seen == {"persistent", "any"}
