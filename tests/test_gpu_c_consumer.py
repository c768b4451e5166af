"""The library driven by a host program with no Python or torch in it: a
C++ program (host code only, built with g++ against the HIP runtime) allocates device memory with
hipMalloc, solves 4096 quadruples with hg_solve4 (ACA and SKS) and writes H
and the flags back; the results match the float64 oracle within the solver's
bar (parity test, GPU)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from paper_2402_18008_amd import build
from tests.gpu_util import announce, require_gpu
from tests.test_gpu_solve import check

pytestmark = pytest.mark.gpu

PROGRAM = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "homog.h"

#define CHECK(x) do { if ((x) != hipSuccess) { std::fprintf(stderr, "HIP error %s\n", #x); return 2; } } while (0)

int main(int argc, char **argv) {
  if (argc != 5) return 3;
  const int method = std::atoi(argv[1]);
  const long n = std::atol(argv[2]);
  std::vector<float> src(8 * n), dst(8 * n), H(9 * n);
  std::vector<unsigned char> flags(n);
  FILE *f = std::fopen(argv[3], "rb");
  if (!f || std::fread(src.data(), 4, 8 * n, f) != size_t(8 * n) ||
      std::fread(dst.data(), 4, 8 * n, f) != size_t(8 * n)) return 4;
  std::fclose(f);
  float *d_src, *d_dst, *d_H;
  unsigned char *d_flags;
  CHECK(hipMalloc(&d_src, 32 * n));
  CHECK(hipMalloc(&d_dst, 32 * n));
  CHECK(hipMalloc(&d_H, 36 * n));
  CHECK(hipMalloc(&d_flags, n));
  CHECK(hipMemcpy(d_src, src.data(), 32 * n, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_dst, dst.data(), 32 * n, hipMemcpyHostToDevice));
  const int st = hg_solve4(method, d_src, d_dst, n, n, d_H, d_flags, nullptr);
  if (st != HG_OK) { std::fprintf(stderr, "hg_solve4: %s\n", hg_last_error()); return 5; }
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemcpy(H.data(), d_H, 36 * n, hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(flags.data(), d_flags, n, hipMemcpyDeviceToHost));
  f = std::fopen(argv[4], "wb");
  if (!f) return 6;
  std::fwrite(H.data(), 4, 9 * n, f);
  std::fwrite(flags.data(), 1, n, f);
  std::fclose(f);
  CHECK(hipFree(d_src));
  CHECK(hipFree(d_dst));
  CHECK(hipFree(d_H));
  CHECK(hipFree(d_flags));
  return 0;
}
"""


@pytest.mark.parametrize("method", ["aca", "sks"])
def test_c_program_solves_against_oracle(method, tmp_path):
    require_gpu()
    gxx = shutil.which("g++")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if gxx is None or not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP runtime headers are not available")
    libdir = os.path.join(build.ROOT, "paper_2402_18008_amd")
    src_file = tmp_path / "consumer.cpp"
    src_file.write_text(PROGRAM)
    exe = tmp_path / "consumer"
    r = subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                        "-I", os.path.join(build.ROOT, "include"), str(src_file), "-o", str(exe),
                        f"-L{os.path.join(rocm, 'lib')}", "-lamdhip64", f"-L{libdir}", "-l:libhomog.so",
                        f"-Wl,-rpath,{os.path.join(rocm, 'lib')}", f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    src, dst, _ = synth.config0()
    n = src.shape[1]
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.ascontiguousarray(src, np.float32).tobytes())
        f.write(np.ascontiguousarray(dst, np.float32).tobytes())
    announce(f"C++ consumer hg_solve4 {method} n={n}")
    r = subprocess.run([str(exe), "0" if method == "aca" else "1", str(n), str(inp), str(out)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    raw = np.fromfile(out, np.uint8)
    Hg = raw[:36 * n].view(np.float32).reshape(9, n).T.reshape(n, 3, 3)
    fg = raw[36 * n:]
    st = check(src, dst, method, Hg, fg, "C++ consumer")
    print(method, st)
