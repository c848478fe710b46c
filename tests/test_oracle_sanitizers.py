"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only): a small driver calls every exported routine on a ragged block
with padded leading dimensions, every buffer allocated at its exact size, so
an out-of-bounds access, a leak or undefined arithmetic ends the run with a
report and a non-zero status."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int or_gram_q(int64_t, int, const double*, int64_t, int, const double*, int64_t, double*, double*);
int or_gram_w_q(int64_t, int, const double*, int64_t, int, const double*, int64_t, const double*,
                double*, double*);
int or_chol_q(int, const double*, const double*, double*, double*);
int or_trinv_q(int, const double*, const double*, double*, double*);
int or_update_q(int64_t, int, const double*, int64_t, int, const double*, int64_t, const double*,
                const double*, const double*, double*, int64_t);
int or_qr_q(int64_t, int, const double*, int64_t, int, const double*, int64_t, double*, int64_t,
            double*, double*, double*, double*);
int or_svqb_q(int, const double*, const double*, double*, double*);
int or_gram_dot2(int64_t, int, const double*, int64_t, int, const double*, int64_t, double*, double*);
int or_gram_f64(int64_t, int, const double*, int64_t, int, const double*, int64_t, double*);
int or_cholqr_steps(int64_t, int, const double*, int64_t, int, const double*, int64_t, int, int, int,
                    int, double*, int64_t, double*, double*, double*, double*);
int or_metrics(int64_t, int, const double*, int64_t, const double*, int64_t, int, const double*,
               int64_t, const double*, const double*, double*, double*);
int or_gram_split_bf16(int64_t, int, const float*, int64_t, int64_t, double*);
int or_iterate(int64_t, int, const double*, int64_t, int, const double*, int64_t, int, int, int,
               double, int, double*, int64_t, double*, double*, double*, double*, double*);

static uint64_t st = 88172645463325252ull;
static double rnd(void) {
  st ^= st << 13; st ^= st >> 7; st ^= st << 17;
  return (double)(st >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}
static double* mat(int64_t rows, int64_t ld) {
  double* p = (double*)malloc(sizeof(double) * (size_t)(rows * ld));
  for (int64_t i = 0; i < rows * ld; ++i) p[i] = rnd();
  return p;
}
int main(void) {
  const int64_t m = 1001;
  const int k = 5, ky = 3, W = ky + k;
  const int64_t ldx = 7, ldy = 4, ldq = 6;
  double* X = mat(m, ldx);
  double* Y = mat(m, ldy);
  double* w = mat(m, 1);
  for (int64_t i = 0; i < m; ++i) w[i] = 1.5 + w[i];
  double *ghi = mat(W, W), *glo = mat(W, W);
  int rc = 0;
  rc |= or_gram_q(m, ky, Y, ldy, k, X, ldx, ghi, glo);
  rc |= or_gram_w_q(m, ky, Y, ldy, k, X, ldx, w, ghi, glo);
  rc |= or_gram_dot2(m, ky, Y, ldy, k, X, ldx, ghi, glo);
  rc |= or_gram_f64(m, ky, Y, ldy, k, X, ldx, ghi);
  double *g = mat(k, k), *gl = mat(k, k), *rhi = mat(k, k), *rlo = mat(k, k);
  rc |= or_gram_q(m, k, X, ldx, k, X, ldx, g, gl);  /* X^T X */
  rc |= or_chol_q(k, g, gl, rhi, rlo);
  double *zhi = mat(k, k), *zlo = mat(k, k), *lam = mat(k, 1);
  rc |= or_trinv_q(k, rhi, rlo, zhi, zlo);
  rc |= or_svqb_q(k, g, gl, zhi, lam);
  double *chi = mat(ky, k), *clo = mat(ky, k), *Q = mat(m, ldq), *R = mat(k, k), *C = mat(ky, k);
  rc |= or_update_q(m, k, X, ldx, ky, Y, ldy, chi, clo, zhi, Q, ldq);
  rc |= or_qr_q(m, k, X, ldx, ky, Y, ldy, Q, ldq, R, C, ghi, glo);
  rc |= or_cholqr_steps(m, k, X, ldx, ky, Y, ldy, 1, 1, 2, 1, Q, ldq, rhi, rlo, chi, clo);
  rc |= or_cholqr_steps(m, k, X, ldx, 0, NULL, 0, 0, 0, 1, 1, Q, ldq, rhi, rlo, NULL, NULL);
  double out[4];
  for (int dd = 0; dd < 2; ++dd)
    for (int fact = 0; fact < 2; ++fact)
      for (int fused = 0; fused < 2; ++fused)
        rc |= or_iterate(m, k, X, ldx, ky, Y, ldy, dd, fact, fused, 1e-10, 3, Q, ldq, rhi, rlo, chi,
                         clo, out);
  rc |= or_metrics(m, k, Q, ldq, X, ldx, ky, Y, ldy, R, C, out, NULL);
  float* Xf = (float*)malloc(sizeof(float) * (size_t)(m * ldx));
  for (int64_t i = 0; i < m * ldx; ++i) Xf[i] = (float)X[i];
  rc |= or_gram_split_bf16(m, k, Xf, ldx, 256, g);
  printf("rc=%d omega=%.3e rho=%.3e\n", rc, out[0], out[1]);
  free(X); free(Y); free(w); free(ghi); free(glo); free(g); free(gl); free(rhi); free(rlo);
  free(zhi); free(zlo); free(lam); free(chi); free(clo); free(Q); free(R); free(C); free(Xf);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", str(exe), str(drv), str(ROOT / "oracle" / "oracle.c"), "-lquadmath", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                            "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "rc=0 " in r.stdout and "runtime error" not in r.stderr, (r.stdout, r.stderr[-3000:])
