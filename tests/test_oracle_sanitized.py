"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only), driven through its entry points on small instances with ragged
shapes (H != T, lags past the day, a short last minibatch, paths of different
lengths, FIFO-violating speeds): any out-of-bounds access, use of freed memory
or undefined arithmetic aborts the driver.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "dode_oracle.c")

DRIVER = r'''
#include <stdio.h>
#include <stdlib.h>
#include "dode_oracle.c"

static unsigned long long rs = 88172645463325252ULL;
static double rnd(void) {   /* xorshift64, uniform in [0, 1) */
  rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
  return (double)(rs >> 11) / 9007199254740992.0;
}
static double* arr(size_t n) {
  double* a = (double*)malloc(sizeof(double) * (n ? n : 1));
  for (size_t i = 0; i < n; ++i) a[i] = rnd();
  return a;
}

int main(void) {
  /* band problem: P=5 ODs, L=7 links, T=9, H=11, K=4, 3 days in 2 clusters */
  orc_dims dm = {5, 7, 9, 11, 4};
  int32_t row_ptr[8], col[35];
  int32_t nnz = 0;
  for (int a = 0; a < dm.L; ++a) {
    row_ptr[a] = nnz;
    for (int p = 0; p < dm.P; ++p) if ((a + 2 * p) % 3 != 0) col[nnz++] = p;
  }
  row_ptr[dm.L] = nnz;
  const int64_t nw = (int64_t)dm.K * dm.T * nnz, nq = (int64_t)dm.T * dm.P, nx = (int64_t)dm.H * dm.L;
  double* W[2] = {arr(nw), arr(nw)};
  int32_t dc[3] = {0, 1, 1};
  double* X = arr(3 * nx);
  double* Q = (double*)calloc(3 * nq, sizeof(double));
  double* A = (double*)calloc(3 * nq, sizeof(double));
  const int E = 3;
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * E * 2 * dm.H);
  for (int e = 0; e < E; ++e)
    for (int c = 0; c < 2; ++c)
      for (int h = 0; h < dm.H; ++h) perm[(e * 2 + c) * dm.H + h] = (h * 5 + e + c) % dm.H;
  double hist[9];
  if (orc_spgd(&dm, 3, dc, row_ptr, col, (const double* const*)W, X, Q, A, perm, 2 * dm.H, dm.H,
               E, 4, 0, 0, 0.5, 1e-10, hist, 1)) return 2;
  double loss[3], kkt[3], r2[3];
  orc_metrics(&dm, 3, dc, row_ptr, col, (const double* const*)W, X, Q, loss, kkt, r2, 1);
  double* xh = arr(nx);
  double* g = arr(nq);
  orc_apply(&dm, row_ptr, col, W[0], Q, xh);
  orc_adjoint(&dm, row_ptr, col, W[0], X, g);
  double* dW = arr(nw);
  double* dQ = arr(2 * nq);
  orc_loss_backward(&dm, row_ptr, col, W[1], 2, X, Q, dW, dQ);

  /* routes: 3 paths of lengths 2, 3, 1 over the pattern above */
  int32_t path_od[3] = {0, 1, 3};
  int32_t pair_ptr[4] = {0, 2, 5, 6};
  int32_t pair_link[6];
  int m = 0;
  for (int k = 0; k < 3; ++k)
    for (int a = 0, got = 0; a < dm.L && got < pair_ptr[k + 1] - pair_ptr[k]; ++a)
      for (int j = row_ptr[a]; j < row_ptr[a + 1]; ++j)
        if (col[j] == path_od[k]) { pair_link[m++] = a; ++got; break; }
  if (m != 6) return 3;
  double* Rr = arr((size_t)dm.K * dm.T * 6);
  double z[3] = {0.3, -1.0, 2.0}, dz[3];
  double* Wr = arr(nw);
  if (orc_rho_from_logits(&dm, 3, path_od, pair_ptr, pair_link, Rr, z, row_ptr, col, Wr)) return 4;
  if (orc_logits_backward(&dm, 3, path_od, pair_ptr, pair_link, Rr, z, row_ptr, col, dW, dz)) return 5;

  /* speeds: 2 days, 7 links, 6 speed intervals (shorter than H), a slow-then-fast link */
  double len[7], *speed = arr(2 * 7 * 6);
  for (int a = 0; a < 7; ++a) len[a] = 0.5 + rnd();
  for (int i = 0; i < 2 * 7 * 6; ++i) speed[i] = 0.05 + speed[i];
  speed[0] = 0.01; speed[1] = 5.0;   /* overtaking on link 0 of day 0 */
  double* Rs = arr((size_t)dm.K * dm.H * 6);
  if (orc_dar_from_speeds(3, pair_ptr, pair_link, 7, len, speed, 2, 6, 5.0, dm.H, dm.K, 1, Rs)) return 6;
  if (orc_dar_from_speeds(3, pair_ptr, pair_link, 7, len, speed, 2, 6, 5.0, dm.H, dm.K, 0, Rs)) return 6;
  double* cost = arr((size_t)dm.T * 3);
  double* port = arr((size_t)dm.T * 3);
  if (orc_path_costs(3, pair_ptr, pair_link, 7, len, speed, 2, 6, 5.0, dm.T, 1, cost)) return 7;
  if (orc_path_costs(3, pair_ptr, pair_link, 7, len, speed, 2, 6, 5.0, dm.T, 0, cost)) return 7;
  orc_logit_portions(dm.P, 3, path_od, dm.T, 0.6, cost, port);
  if (orc_rho_from_portions(&dm, 3, path_od, pair_ptr, pair_link, Rs, port, row_ptr, col, Wr)) return 8;

  /* dense: 13 x 6, minibatches of 5 (short tail) */
  double* B = arr(13 * 6);
  double* y = arr(13);
  double qd[6] = {0}, Ad[6] = {0}, dh[2];
  int32_t dp[26];
  for (int e = 0; e < 2; ++e)
    for (int i = 0; i < 13; ++i) dp[e * 13 + i] = (i * 4 + e) % 13;
  if (orc_dense_spgd(13, 6, B, y, qd, Ad, dp, 2, 5, 0, 0.1, 1e-10, dh)) return 9;
  printf("ok %.6g %.6g %.6g\n", hist[0], loss[0], dh[1]);
  free(W[0]); free(W[1]); free(X); free(Q); free(A); free(perm); free(xh); free(g); free(dW); free(dQ);
  free(Rr); free(Wr); free(speed); free(Rs); free(cost); free(port); free(B); free(y);
  return 0;
}
'''


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I",
                           os.path.dirname(SRC), str(drv), "-o", str(exe), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
