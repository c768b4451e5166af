"""The refit kernel's moment shift, run on the host: the count and moments summed
about a reference point (the pair's first point) and shifted to the centroids
by the library's own center_moments must equal the moments summed about the
centroids directly, on 200 random point sets whose origins lie up to 500 px
from the reference and whose spreads range from 1 to 300 px (bar: 1e-11 of
the sum of the terms' magnitudes; observed ~1e-13). The program includes the
kernel source, is built with hipcc and calls only host code."""
import os
import subprocess

import pytest

from paper_2402_18008_amd import build

PROGRAM = r"""
#include "refit.hip"
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

int main() {
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double worst = 0.0;
  for (int trial = 0; trial < 200; ++trial) {
    const int n = 5 + trial * 7;
    std::vector<double> X(n), Y(n), Uu(n), V(n);
    const double ox = 500 * U(g), oy = 500 * U(g), ou = 500 * U(g), ov = 500 * U(g);
    const double sp = 1.0 + 300.0 * (0.5 + 0.5 * U(g));
    for (int i = 0; i < n; ++i) {
      X[i] = ox + sp * U(g); Y[i] = oy + sp * U(g); Uu[i] = ou + sp * U(g); V[i] = ov + sp * U(g);
    }
    const double rx = X[0], ry = Y[0], ru = Uu[0], rv = V[0];
    double r[hg::kRaw] = {0};
    for (int i = 0; i < n; ++i) {
      const double x = X[i] - rx, y = Y[i] - ry, u = Uu[i] - ru, v = V[i] - rv;
      const double mono[6] = {x * x, x * y, x, y * y, y, 1.0};
      for (int k = 0; k < 6; ++k) {
        r[k] += mono[k]; r[6 + k] += u * mono[k]; r[12 + k] += u * u * mono[k];
        r[18 + k] += v * mono[k]; r[24 + k] += v * v * mono[k];
      }
    }
    double m[hg::kMoments], a, b, c, d;
    hg::center_moments(r, m, a, b, c, d);
    // direct
    double cx = 0, cy = 0, cu = 0, cv = 0;
    for (int i = 0; i < n; ++i) { cx += X[i]; cy += Y[i]; cu += Uu[i]; cv += V[i]; }
    cx /= n; cy /= n; cu /= n; cv /= n;
    double md[hg::kMoments] = {0};
    for (int i = 0; i < n; ++i) {
      const double x = X[i] - cx, y = Y[i] - cy, u = Uu[i] - cu, v = V[i] - cv;
      const double mono[6] = {x * x, x * y, x, y * y, y, 1.0};
      for (int k = 0; k < 5; ++k) md[k] += mono[k];
      for (int k = 0; k < 6; ++k) {
        md[5 + k] += u * mono[k]; md[11 + k] += u * u * mono[k];
        md[17 + k] += v * mono[k]; md[23 + k] += v * v * mono[k];
      }
    }
    // scale of each moment: the sum of the absolute values of its terms
    double sc[hg::kMoments] = {0};
    for (int i = 0; i < n; ++i) {
      const double x = fabs(X[i] - cx), y = fabs(Y[i] - cy), u = fabs(Uu[i] - cu), v = fabs(V[i] - cv);
      const double mono[6] = {x * x, x * y, x, y * y, y, 1.0};
      for (int k = 0; k < 5; ++k) sc[k] += mono[k];
      for (int k = 0; k < 6; ++k) {
        sc[5 + k] += u * mono[k]; sc[11 + k] += u * u * mono[k];
        sc[17 + k] += v * mono[k]; sc[23 + k] += v * v * mono[k];
      }
    }
    for (int k = 0; k < hg::kMoments; ++k) {
      const double e = fabs(m[k] - md[k]) / sc[k];
      if (e > worst) worst = e;
    }
    if (fabs(rx + a - cx) > 1e-9 * (fabs(cx) + sp) || fabs(rv + d - cv) > 1e-9 * (fabs(cv) + sp)) {
      printf("centroid mismatch trial %d\n", trial);
      return 1;
    }
  }
  printf("worst relative (to the sum of |terms|) moment error %.3g\n", worst);
  return worst < 1e-11 ? 0 : 1;
}
"""


def test_center_moments_matches_direct_sums(tmp_path):
    try:
        hipcc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    csrc = os.path.join(build.ROOT, "paper_2402_18008_amd", "csrc")
    src = tmp_path / "center_check.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "center_check"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I",
                        os.path.join(build.ROOT, "include"), "-I", csrc, str(src),
                        os.path.join(csrc, "status.hip"), "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout, r.stderr)
