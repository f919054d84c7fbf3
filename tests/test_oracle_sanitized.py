"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, gcc) and run on small inputs of every shape class: no sanitizer
report, and the three entry points agree with each other."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_xmac(const uint8_t *in, int n, int f, int t, int layout, int64_t *out);
int oracle_xmac_full(const uint8_t *in, int n, int f, int t, int layout, int64_t *out);
int oracle_incoherent_beam(const uint8_t *in, int n, int f, int t, int layout, int64_t *out);
void oracle_set_threads(int n);

int main(void) {
  const int shapes[][3] = {{1, 1, 1}, {2, 3, 5}, {7, 2, 33}, {16, 4, 9}, {33, 1, 70}, {64, 2, 17}};
  uint32_t seed = 12345;
  oracle_set_threads(2);
  for (unsigned s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
    for (int layout = 0; layout < 2; ++layout) {
      const int n = shapes[s][0], f = shapes[s][1], t = shapes[s][2];
      const size_t nb = (size_t)n * (n + 1) / 2;
      uint8_t *in = malloc((size_t)n * f * t);
      int64_t *tri = malloc(sizeof(int64_t) * f * nb * 2);
      int64_t *full = malloc(sizeof(int64_t) * f * n * n * 2);
      int64_t *beam = malloc(sizeof(int64_t) * f * t);
      for (size_t k = 0; k < (size_t)n * f * t; ++k) {
        seed = seed * 1664525u + 1013904223u;
        in[k] = (uint8_t)(seed >> 24);  /* all 256 codes, invalid ones included */
      }
      if (oracle_xmac(in, n, f, t, layout, tri) || oracle_xmac_full(in, n, f, t, layout, full) ||
          oracle_incoherent_beam(in, n, f, t, layout, beam)) return 2;
      for (int c = 0; c < f; ++c) {
        int64_t autos = 0, beams = 0;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j <= i; ++j) {
            const int64_t *a = tri + ((size_t)c * nb + (size_t)i * (i + 1) / 2 + j) * 2;
            const int64_t *b = full + (((size_t)c * n + i) * n + j) * 2;
            const int64_t *m = full + (((size_t)c * n + j) * n + i) * 2;
            if (a[0] != b[0] || a[1] != b[1] || m[0] != b[0] || m[1] != -b[1]) return 3;
            if (i == j) {
              if (a[1] != 0 || a[0] < 0) return 4;
              autos += a[0];
            }
          }
        for (int k = 0; k < t; ++k) beams += beam[(size_t)c * t + k];
        if (autos != beams) return 5;
      }
      free(in); free(tri); free(full); free(beam);
    }
  puts("ok");
  return 0;
}
"""


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_asan"
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", str(drv), os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr[-2000:])
