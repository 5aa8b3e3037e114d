/*
 * dode_oracle.c -- plain FP64 CPU reference for the per-day dynamic OD
 * estimation problem of Ma & Qian (arXiv 1901.09266) and its SPGD solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source, header, table or helper
 * with the HIP library and must never be linked into it.
 *
 * Everything is written as plain loops in the order the paper states the
 * computation; there is no blocking, fusion or reordering beyond that.
 *
 * Data layout (Table "DODE framework variable vectorization"; the paper's
 * interval-major vectors, one day at a time):
 *   q[t][p]      OD demand of OD p departing in interval t      (T x P)
 *   x[h][a]      observed count of link a in interval h          (H x L)
 *   rho          assignment matrix, entry ((t+l)*L + a, t*P + p) = W[l][t][nz]
 *                where nz runs over the incidence pattern in CSR form
 *                (row_ptr[L+1], col[nnz]: the ODs whose routes cross link a).
 *                W is [K][T][nnz]; a block with t+l >= H does not exist.
 *
 * Parity: pinned by the tests listed in the module docstring of oracle.py
 * (brute-force active sets, scipy's Lawson-Hanson NNLS, planted recovery, KKT,
 * adjoint identity, finite differences, closed forms, torch's Adagrad).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t P, L, T, H, K;
} orc_dims;

#define IDX2(i, j, n) ((int64_t)(i) * (int64_t)(n) + (int64_t)(j))

static const double* block_of(const orc_dims* dm, const double* W, int64_t nnz, int l, int t) {
  return W + ((int64_t)l * dm->T + t) * nnz;
}

/* Eq. "finalobj" / eq. "assign": estimated link count of link a in interval h
 *   xhat[h][a] = sum_{l=0}^{K-1} sum_{p} rho_{(t=h-l)}[l][a][p] * q[h-l][p]. */
static double row_value(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col,
                        const double* W, const double* q, int h, int a) {
  const int64_t nnz = row_ptr[dm->L];
  double s = 0.0;
  for (int l = 0; l < dm->K; ++l) {
    const int t = h - l;
    if (t < 0 || t >= dm->T) continue;
    const double* w = block_of(dm, W, nnz, l, t);
    for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) s += w[j] * q[IDX2(t, col[j], dm->P)];
  }
  return s;
}

/* O1: xhat = rho q for one day. */
void orc_apply(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
               const double* q, double* xhat) {
  for (int h = 0; h < dm->H; ++h)
    for (int a = 0; a < dm->L; ++a) xhat[IDX2(h, a, dm->L)] = row_value(dm, row_ptr, col, W, q, h, a);
}

/* O3 helper: g += rho^T r restricted to one row (h, a) of rho, i.e.
 *   g[h-l][p] += rho[l][h-l][a][p] * r  for every l and p. */
static void add_row_transpose(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col,
                              const double* W, int h, int a, double r, double* g) {
  const int64_t nnz = row_ptr[dm->L];
  for (int l = 0; l < dm->K; ++l) {
    const int t = h - l;
    if (t < 0 || t >= dm->T) continue;
    const double* w = block_of(dm, W, nnz, l, t);
    for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) g[IDX2(t, col[j], dm->P)] += w[j] * r;
  }
}

/* O3: g = rho^T r for a full residual r[h][a] of one day. */
void orc_adjoint(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
                 const double* r, double* g) {
  memset(g, 0, sizeof(double) * (size_t)dm->T * dm->P);
  for (int h = 0; h < dm->H; ++h)
    for (int a = 0; a < dm->L; ++a)
      add_row_transpose(dm, row_ptr, col, W, h, a, r[IDX2(h, a, dm->L)], g);
}

/* O2 (eq. "nnls"): loss = || rho q - x ||_2^2 for one day (no 1/2, no mean). */
double orc_loss(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
                const double* q, const double* x) {
  double s = 0.0;
  for (int h = 0; h < dm->H; ++h)
    for (int a = 0; a < dm->L; ++a) {
      const double r = row_value(dm, row_ptr, col, W, q, h, a) - x[IDX2(h, a, dm->L)];
      s += r * r;
    }
  return s;
}

/* Full gradient of Algorithm 1's form: g = rho^T (rho q - x)  (= half the
 * gradient of the loss). */
void orc_grad(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
              const double* q, const double* x, double* g) {
  memset(g, 0, sizeof(double) * (size_t)dm->T * dm->P);
  for (int h = 0; h < dm->H; ++h)
    for (int a = 0; a < dm->L; ++a) {
      const double r = row_value(dm, row_ptr, col, W, q, h, a) - x[IDX2(h, a, dm->L)];
      add_row_transpose(dm, row_ptr, col, W, h, a, r, g);
    }
}

/* KKT natural residual of the NNLS: max_k | min(q_k, g_k) |. */
double orc_kkt(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
               const double* q, const double* x) {
  const int64_t n = (int64_t)dm->T * dm->P;
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  orc_grad(dm, row_ptr, col, W, q, x, g);
  double k = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double m = fabs(q[i] < g[i] ? q[i] : g[i]);
    if (m > k) k = m;
  }
  free(g);
  return k;
}

/* Step 6 quality check: R^2 between observed and estimated link counts,
 * 1 - sum (x - xhat)^2 / sum (x - mean x)^2 over all (h, a) of the day. */
double orc_r2(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
              const double* q, const double* x) {
  const int64_t n = (int64_t)dm->H * dm->L;
  double mean = 0.0;
  for (int64_t i = 0; i < n; ++i) mean += x[i];
  mean /= (double)n;
  double sst = 0.0;
  for (int64_t i = 0; i < n; ++i) sst += (x[i] - mean) * (x[i] - mean);
  const double sse = orc_loss(dm, row_ptr, col, W, q, x);
  return 1.0 - sse / sst;
}

/* One minibatch of Algorithm 1 on the rows `rows` (flat ids h*L + a):
 *   rho_o = rho[rows, :];  g = rho_o^T (rho_o q - x_o);
 *   q = Adagrad(q, g, eta) (or a fixed step);  q = max(q, 0).
 * The residual of every row in the minibatch is taken with q before the step.
 * The step and the projection apply to every coordinate. */
static void spgd_minibatch(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col,
                           const double* W, const double* x, double* q, double* A,
                           const int64_t* rows, int64_t nrows, int optimizer, double eta,
                           double eps, double* r, double* g) {
  const int64_t n = (int64_t)dm->T * dm->P;
  for (int64_t i = 0; i < nrows; ++i) {
    const int h = (int)(rows[i] / dm->L), a = (int)(rows[i] % dm->L);
    r[i] = row_value(dm, row_ptr, col, W, q, h, a) - x[rows[i]];
  }
  memset(g, 0, sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < nrows; ++i) {
    const int h = (int)(rows[i] / dm->L), a = (int)(rows[i] % dm->L);
    add_row_transpose(dm, row_ptr, col, W, h, a, r[i], g);
  }
  for (int64_t k = 0; k < n; ++k) {
    if (optimizer == 0) {
      /* Adagrad (Duchi et al. 2011) as PyTorch defines it: accumulator from 0,
       * eps added after the square root, no decay. */
      A[k] += g[k] * g[k];
      q[k] -= eta * g[k] / (sqrt(A[k]) + eps);
    } else {
      q[k] -= eta * g[k];
    }
    if (!(q[k] > 0.0)) q[k] = 0.0;
  }
}

/* One minibatch of Algorithm 1 on the rows of the n_h observation intervals
 * hblocks[] (all L rows of each, in the order given). */
int orc_spgd_step(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
                  const double* x, double* q, double* A, const int32_t* hblocks, int32_t n_h,
                  int32_t optimizer, double eta, double eps) {
  const int64_t nrows = (int64_t)n_h * dm->L;
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)nrows);
  double* r = (double*)malloc(sizeof(double) * (size_t)nrows);
  double* g = (double*)malloc(sizeof(double) * (size_t)dm->T * dm->P);
  if (!rows || !r || !g) {
    free(rows); free(r); free(g);
    return 2;
  }
  int64_t k = 0;
  for (int32_t i = 0; i < n_h; ++i)
    for (int a = 0; a < dm->L; ++a) rows[k++] = (int64_t)hblocks[i] * dm->L + a;
  spgd_minibatch(dm, row_ptr, col, W, x, q, A, rows, nrows, optimizer, eta, eps, r, g);
  free(rows); free(r); free(g);
  return 0;
}

/*
 * O4: Algorithm 1 for one day.
 *   granularity 0: the permuted units are interval blocks (all L rows of an
 *                  observation interval h); perm_e lists the H blocks of epoch e
 *                  and each minibatch holds `chunk` consecutive blocks.
 *   granularity 1: the permuted units are single rows (h*L + a), as printed;
 *                  perm_e lists the H*L rows and each minibatch holds `chunk` rows.
 * The last minibatch of an epoch may be shorter.  perm for epoch e starts at
 * perm + e * perm_stride.  loss_hist[e] (if not NULL) is the full loss after
 * epoch e.  optimizer 0 = Adagrad, 1 = fixed step.  Returns 0 on success.
 */
int orc_spgd_day(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col, const double* W,
                 const double* x, double* q, double* A, const int32_t* perm, int64_t perm_stride,
                 int32_t E, int32_t chunk, int32_t granularity, int32_t optimizer, double eta,
                 double eps, double* loss_hist) {
  const int64_t n_units = granularity == 0 ? (int64_t)dm->H : (int64_t)dm->H * dm->L;
  const int64_t max_rows = granularity == 0 ? (int64_t)chunk * dm->L : (int64_t)chunk;
  if (chunk <= 0) return 1;
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)max_rows);
  double* r = (double*)malloc(sizeof(double) * (size_t)max_rows);
  double* g = (double*)malloc(sizeof(double) * (size_t)dm->T * dm->P);
  if (!rows || !r || !g) {
    free(rows); free(r); free(g);
    return 2;
  }
  for (int32_t e = 0; e < E; ++e) {
    const int32_t* pe = perm + (int64_t)e * perm_stride;
    for (int64_t s = 0; s < n_units; s += chunk) {
      const int64_t s1 = s + chunk < n_units ? s + chunk : n_units;
      int64_t nrows = 0;
      for (int64_t u = s; u < s1; ++u) {
        if (granularity == 0) {
          for (int a = 0; a < dm->L; ++a) rows[nrows++] = (int64_t)pe[u] * dm->L + a;
        } else {
          rows[nrows++] = pe[u];
        }
      }
      spgd_minibatch(dm, row_ptr, col, W, x, q, A, rows, nrows, optimizer, eta, eps, r, g);
    }
    if (loss_hist) loss_hist[e] = orc_loss(dm, row_ptr, col, W, q, x);
  }
  free(rows); free(r); free(g);
  return 0;
}

/*
 * Many days at once (days are independent subproblems, section "Estimate the
 * dynamic OD demand").  Day d belongs to cluster day_cluster[d] and uses
 * W[day_cluster[d]]; its permutation for epoch e is
 *   perm + e * perm_epoch_stride + day_cluster[d] * perm_cluster_stride.
 * X is [D][H][L], Q and A are [D][T][P] (updated in place), loss_hist is
 * [D][E] or NULL.  Days run in parallel over `nthreads` OpenMP threads.
 */
int orc_spgd(const orc_dims* dm, int32_t D, const int32_t* day_cluster, const int32_t* row_ptr,
             const int32_t* col, const double* const* W, const double* X, double* Q, double* A,
             const int32_t* perm, int64_t perm_epoch_stride, int64_t perm_cluster_stride,
             int32_t E, int32_t chunk, int32_t granularity, int32_t optimizer, double eta,
             double eps, double* loss_hist, int32_t nthreads) {
  int fail = 0;
  const int64_t nx = (int64_t)dm->H * dm->L, nq = (int64_t)dm->T * dm->P;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : fail)
  for (int32_t d = 0; d < D; ++d) {
    const int32_t c = day_cluster[d];
    fail |= orc_spgd_day(dm, row_ptr, col, W[c], X + d * nx, Q + d * nq, A + d * nq,
                         perm + c * perm_cluster_stride, perm_epoch_stride, E, chunk,
                         granularity, optimizer, eta, eps,
                         loss_hist ? loss_hist + (int64_t)d * E : NULL);
  }
  return fail;
}

/* Per-day end-of-solve figures for many days: loss, KKT residual, R^2. */
void orc_metrics(const orc_dims* dm, int32_t D, const int32_t* day_cluster, const int32_t* row_ptr,
                 const int32_t* col, const double* const* W, const double* X, const double* Q,
                 double* loss, double* kkt, double* r2, int32_t nthreads) {
  const int64_t nx = (int64_t)dm->H * dm->L, nq = (int64_t)dm->T * dm->P;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int32_t d = 0; d < D; ++d) {
    const double* w = W[day_cluster[d]];
    if (loss) loss[d] = orc_loss(dm, row_ptr, col, w, Q + d * nq, X + d * nx);
    if (kkt) kkt[d] = orc_kkt(dm, row_ptr, col, w, Q + d * nq, X + d * nx);
    if (r2) r2[d] = orc_r2(dm, row_ptr, col, w, Q + d * nq, X + d * nx);
  }
}

/* ---------------------------------------------------------------------------
 * O6: route-choice parameterisation (eqs. "logit", "flow", "assign").
 * Path k serves OD path_od[k]; its links are pair_link[pair_ptr[k] .. pair_ptr[k+1]);
 * Rr[l][t][m] is the lag ratio of path-link pair m.  Route proportions are a
 * softmax of the logits z over the paths of each OD (time-invariant), and
 *   rho[l][t][a][p] = sum_{k serving p, a on k} Rr[l][t][(k,a)] * pi_k.
 * ------------------------------------------------------------------------- */
static int32_t find_nz(const int32_t* row_ptr, const int32_t* col, int32_t a, int32_t p) {
  for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j)
    if (col[j] == p) return j;
  return -1;
}

/* pi = softmax of z within each OD's path set. */
void orc_route_softmax(int32_t P, int32_t n_paths, const int32_t* path_od, const double* z, double* pi) {
  for (int32_t p = 0; p < P; ++p) {
    double zmax = -INFINITY;
    for (int32_t k = 0; k < n_paths; ++k)
      if (path_od[k] == p && z[k] > zmax) zmax = z[k];
    double s = 0.0;
    for (int32_t k = 0; k < n_paths; ++k)
      if (path_od[k] == p) s += exp(z[k] - zmax);
    for (int32_t k = 0; k < n_paths; ++k)
      if (path_od[k] == p) pi[k] = exp(z[k] - zmax) / s;
  }
}

/* W_out[l][t][nz] = sum over path-link pairs feeding nz of Rr * pi. */
int orc_rho_from_logits(const orc_dims* dm, int32_t n_paths, const int32_t* path_od,
                        const int32_t* pair_ptr, const int32_t* pair_link, const double* Rr,
                        const double* z, const int32_t* row_ptr, const int32_t* col, double* W_out) {
  const int64_t nnz = row_ptr[dm->L], npairs = pair_ptr[n_paths];
  double* pi = (double*)malloc(sizeof(double) * (size_t)n_paths);
  orc_route_softmax(dm->P, n_paths, path_od, z, pi);
  memset(W_out, 0, sizeof(double) * (size_t)(dm->K * dm->T * nnz));
  for (int32_t k = 0; k < n_paths; ++k)
    for (int32_t m = pair_ptr[k]; m < pair_ptr[k + 1]; ++m) {
      const int32_t j = find_nz(row_ptr, col, pair_link[m], path_od[k]);
      if (j < 0) { free(pi); return 1; }
      for (int l = 0; l < dm->K; ++l)
        for (int t = 0; t < dm->T; ++t)
          W_out[((int64_t)l * dm->T + t) * nnz + j] += Rr[((int64_t)l * dm->T + t) * npairs + m] * pi[k];
    }
  free(pi);
  return 0;
}

/* Derivatives of the summed loss sum_d ||rho q_d - x_d||^2 over n days:
 *   dW[l][t][nz=(a,p)] = 2 sum_d r_d[t+l][a] q_d[t][p]   (only blocks with t+l < H)
 *   dQ_d               = 2 rho^T r_d
 * with r_d = rho q_d - x_d.  Either output may be NULL. */
void orc_loss_backward(const orc_dims* dm, const int32_t* row_ptr, const int32_t* col,
                       const double* W, int32_t n, const double* X, const double* Q, double* dW,
                       double* dQ) {
  const int64_t nnz = row_ptr[dm->L], nx = (int64_t)dm->H * dm->L, nq = (int64_t)dm->T * dm->P;
  double* r = (double*)malloc(sizeof(double) * (size_t)nx);
  if (dW) memset(dW, 0, sizeof(double) * (size_t)(dm->K * dm->T * nnz));
  for (int32_t d = 0; d < n; ++d) {
    const double* q = Q + d * nq;
    for (int h = 0; h < dm->H; ++h)
      for (int a = 0; a < dm->L; ++a)
        r[IDX2(h, a, dm->L)] = row_value(dm, row_ptr, col, W, q, h, a) - X[d * nx + IDX2(h, a, dm->L)];
    if (dQ) {
      orc_adjoint(dm, row_ptr, col, W, r, dQ + d * nq);
      for (int64_t i = 0; i < nq; ++i) dQ[d * nq + i] *= 2.0;
    }
    if (dW) {
      for (int l = 0; l < dm->K; ++l)
        for (int t = 0; t < dm->T; ++t) {
          if (t + l >= dm->H) continue;
          for (int a = 0; a < dm->L; ++a)
            for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j)
              dW[((int64_t)l * dm->T + t) * nnz + j] += 2.0 * r[IDX2(t + l, a, dm->L)] * q[IDX2(t, col[j], dm->P)];
        }
    }
  }
  free(r);
}

/* Chain rule from dW to the logits:
 *   dpi_k = sum_{l,t, a on k} Rr[l][t][(k,a)] * dW[l][t][nz(a, od(k))]
 *   dz_k  = pi_k * (dpi_k - sum_{k' serving od(k)} pi_k' dpi_k'). */
int orc_logits_backward(const orc_dims* dm, int32_t n_paths, const int32_t* path_od,
                        const int32_t* pair_ptr, const int32_t* pair_link, const double* Rr,
                        const double* z, const int32_t* row_ptr, const int32_t* col,
                        const double* dW, double* dz) {
  const int64_t nnz = row_ptr[dm->L], npairs = pair_ptr[n_paths];
  double* pi = (double*)malloc(sizeof(double) * (size_t)n_paths);
  double* dpi = (double*)calloc((size_t)n_paths, sizeof(double));
  orc_route_softmax(dm->P, n_paths, path_od, z, pi);
  for (int32_t k = 0; k < n_paths; ++k)
    for (int32_t m = pair_ptr[k]; m < pair_ptr[k + 1]; ++m) {
      const int32_t j = find_nz(row_ptr, col, pair_link[m], path_od[k]);
      if (j < 0) { free(pi); free(dpi); return 1; }
      for (int l = 0; l < dm->K; ++l)
        for (int t = 0; t < dm->T; ++t)
          dpi[k] += Rr[((int64_t)l * dm->T + t) * npairs + m] * dW[((int64_t)l * dm->T + t) * nnz + j];
    }
  for (int32_t k = 0; k < n_paths; ++k) {
    double s = 0.0;
    for (int32_t k2 = 0; k2 < n_paths; ++k2)
      if (path_od[k2] == path_od[k]) s += pi[k2] * dpi[k2];
    dz[k] = pi[k] * (dpi[k] - s);
  }
  free(pi); free(dpi);
  return 0;
}

/* ------------------------------------------------------------------------
 * Dynamic assignment ratios from link speeds (section "Dynamic assignment
 * ratio", eqs. "dar2"/"dar", Example "DAR matrix computation"; section
 * "Link/path travel time", eq. "cost").
 *
 * Time is in minutes, observation intervals are [h*dt, (h+1)*dt).  Link a
 * entered at time t is crossed in c_a(t) = len[a] / speed[a][floor(t/dt)]
 * minutes (speed per link and interval, length/speed in consistent units;
 * the last interval's speed holds after the end of the day).  A vehicle of
 * path k departing at t enters the i-th link of the path at tau_i(t), with
 * tau_0(t) = t and tau_{i+1}(t) = tau_i(t) + c_{alpha(i)}(tau_i(t)) (eq.
 * "cost").  Departure interval h maps onto the arrival window
 * [tau_i(h*dt), tau_i((h+1)*dt)] at link alpha(i), and the ratio of
 * observation interval h2 is the share of the window that lies in it (eq.
 * "dar", as the worked example computes it from the two boundary
 * trajectories).  A window of zero length puts all its mass in the interval
 * of its start; reversed end points (a FIFO violation) are swapped.  Shares
 * in intervals h2 >= H (after the day) or with h2 - h >= K are dropped.
 *
 * Paths: path_ptr[n_paths+1], path_link[] the links of each path in the order
 * they are traversed; pair m = path_ptr[k] + i is the i-th link of path k.
 * Output Rr[K][H][n_pairs] = the mean over the n_days days of each day's
 * ratios (one averaged ratio set per traffic pattern).
 *
 * walk_f32 = 1 takes the walk's interval decisions (which speed a link is
 * crossed at) in binary32, the precision of a single-precision GPU run, so
 * that both sides pick the same speeds: the departure time t0 = h*dt, the
 * travel time so far r and each link time len/speed are binary32 values, and
 * a link is entered at the binary32 sum t0 + r (tau_i(t0) = t0 + r_i, the same
 * recursion as eq. "cost" with the departure time taken out).  The windows,
 * shares and day means stay in binary64.  walk_f32 = 0 is the binary64 walk.
 * ---------------------------------------------------------------------- */
static double link_time(const double* len, const double* speed_day, int32_t H_speed, double dt,
                        int32_t a, double t) {
  int64_t h = (int64_t)floor(t / dt);
  if (h < 0) h = 0;
  if (h >= H_speed) h = H_speed - 1;
  return len[a] / speed_day[IDX2(a, h, H_speed)];
}

/* the link time of link_time with every operation in binary32 */
static float link_time_f32(const double* len, const double* speed_day, int32_t H_speed, float dt,
                           int32_t a, float t) {
  int64_t h = (int64_t)floorf(t / dt);
  if (h < 0) h = 0;
  if (h >= H_speed) h = H_speed - 1;
  return (float)len[a] / (float)speed_day[IDX2(a, h, H_speed)];
}

/* overlap length of [lo, hi] with [h2*dt, (h2+1)*dt) */
static double overlap(double lo, double hi, int64_t h2, double dt) {
  const double a = fmax(lo, (double)h2 * dt), b = fmin(hi, (double)(h2 + 1) * dt);
  return b > a ? b - a : 0.0;
}

int orc_dar_from_speeds(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                        int32_t L, const double* len, const double* speed, int32_t n_days,
                        int32_t H_speed, double dt, int32_t H, int32_t K, int32_t walk_f32,
                        double* Rr) {
  const int64_t n_pairs = path_ptr[n_paths];
  const float dt32 = (float)dt;
  memset(Rr, 0, sizeof(double) * (size_t)K * H * n_pairs);
  if (n_days < 1) return 0;
  for (int32_t d = 0; d < n_days; ++d) {
    const double* sp = speed + (int64_t)d * L * H_speed;
    for (int32_t k = 0; k < n_paths; ++k)
      for (int32_t h = 0; h < H; ++h) {
        /* the two boundary trajectories of departure interval h */
        double s = h * dt, e = (h + 1) * dt;
        const float s0 = (float)h * dt32, e0 = (float)(h + 1) * dt32;
        float rs = 0.0f, re = 0.0f; /* binary32 travel times so far */
        for (int32_t m = path_ptr[k]; m < path_ptr[k + 1]; ++m) {
          const int32_t a = path_link[m];
          if (walk_f32) {
            s = (double)s0 + (double)rs;
            e = (double)e0 + (double)re;
          }
          double lo = s, hi = e;
          if (hi < lo) { const double tmp = lo; lo = hi; hi = tmp; }
          const double w = hi - lo;
          if (w <= 0.0) {
            const int64_t h2 = (int64_t)floor(lo / dt);
            if (h2 < H && h2 - h < K && h2 >= h) Rr[IDX2(IDX2(h2 - h, h, H), m, n_pairs)] += 1.0 / n_days;
          } else {
            const int64_t h2a = (int64_t)floor(lo / dt), h2b = (int64_t)floor(hi / dt);
            for (int64_t h2 = h2a; h2 <= h2b; ++h2) {
              if (h2 >= H || h2 - h >= K || h2 < h) continue;
              Rr[IDX2(IDX2(h2 - h, h, H), m, n_pairs)] += overlap(lo, hi, h2, dt) / w / n_days;
            }
          }
          if (walk_f32) {
            rs += link_time_f32(len, sp, H_speed, dt32, a, s0 + rs);
            re += link_time_f32(len, sp, H_speed, dt32, a, e0 + re);
          } else {
            s += link_time(len, sp, H_speed, dt, a, s);
            e += link_time(len, sp, H_speed, dt, a, e);
          }
        }
      }
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Route choice portions from mean path travel times (section "Route choice
 * portions", eqs. "logit" and "rt"; section "Link/path travel time",
 * eq. "cost") and the assignment matrix they give (eq. "assign").
 *
 * Path cost: c_k(t1) is the time a vehicle departing at t1 needs to cross
 * every link of path k in order, each link timed at the speed of the interval
 * in which the vehicle enters it (the link time of orc_dar_from_speeds).  The
 * portions of interval t use the departure at the interval's start, t1 = t*dt
 * (eq. "rt" holds them constant over the interval), and c~ is the mean of the
 * n_days days' costs.  Output cost[T][n_paths].  walk_f32 as for
 * orc_dar_from_speeds: the day's travel time is walked in binary32 (departure
 * time, travel time so far and link times binary32, links entered at their
 * binary32 sum) and summed over the days in binary64.
 * ---------------------------------------------------------------------- */
int orc_path_costs(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link, int32_t L,
                   const double* len, const double* speed, int32_t n_days, int32_t H_speed,
                   double dt, int32_t T, int32_t walk_f32, double* cost) {
  const float dt32 = (float)dt;
  memset(cost, 0, sizeof(double) * (size_t)T * n_paths);
  if (n_days < 1) return 0;
  for (int32_t t = 0; t < T; ++t)
    for (int32_t k = 0; k < n_paths; ++k) {
      double sum = 0.0;
      for (int32_t d = 0; d < n_days; ++d) {
        const double* sp = speed + (int64_t)d * L * H_speed;
        if (walk_f32) {
          const float t0 = (float)t * dt32;
          float r = 0.0f; /* travel time so far */
          for (int32_t m = path_ptr[k]; m < path_ptr[k + 1]; ++m)
            r += link_time_f32(len, sp, H_speed, dt32, path_link[m], t0 + r);
          sum += (double)r;
          continue;
        }
        const double t1 = t * dt;
        double tau = t1; /* entry time of the current link */
        for (int32_t m = path_ptr[k]; m < path_ptr[k + 1]; ++m)
          tau += link_time(len, sp, H_speed, dt, path_link[m], tau);
        sum += tau - t1;
      }
      cost[IDX2(t, k, n_paths)] = sum / n_days;
    }
  return 0;
}

/* p[t][k] = exp(-theta c[t][k]) / sum over the paths k' of od(k) of
 * exp(-theta c[t][k']) (eq. "logit", interval-wise per eq. "rt"). */
void orc_logit_portions(int32_t P, int32_t n_paths, const int32_t* path_od, int32_t T, double theta,
                        const double* cost, double* p) {
  double* z = (double*)malloc(sizeof(double) * (size_t)n_paths);
  for (int32_t t = 0; t < T; ++t) {
    for (int32_t k = 0; k < n_paths; ++k) z[k] = -theta * cost[IDX2(t, k, n_paths)];
    orc_route_softmax(P, n_paths, path_od, z, p + (int64_t)t * n_paths);
  }
  free(z);
}

/* B of eq. "assign" with time-dependent portions: W[l][t][nz=(a,p)] = sum
 * over the paths k of OD p that cross link a of Rr[l][t][pair (k,a)] *
 * p[t][k]; the pair's delta is 1 by construction.  Rr [K][T][n_pairs],
 * p [T][n_paths]. */
int orc_rho_from_portions(const orc_dims* dm, int32_t n_paths, const int32_t* path_od,
                          const int32_t* pair_ptr, const int32_t* pair_link, const double* Rr,
                          const double* p, const int32_t* row_ptr, const int32_t* col,
                          double* W_out) {
  const int64_t nnz = row_ptr[dm->L], npairs = pair_ptr[n_paths];
  memset(W_out, 0, sizeof(double) * (size_t)(dm->K * dm->T * nnz));
  for (int32_t k = 0; k < n_paths; ++k)
    for (int32_t m = pair_ptr[k]; m < pair_ptr[k + 1]; ++m) {
      const int32_t j = find_nz(row_ptr, col, pair_link[m], path_od[k]);
      if (j < 0) return 1;
      for (int l = 0; l < dm->K; ++l)
        for (int t = 0; t < dm->T; ++t)
          W_out[((int64_t)l * dm->T + t) * nnz + j] +=
              Rr[((int64_t)l * dm->T + t) * npairs + m] * p[IDX2(t, k, n_paths)];
    }
  return 0;
}

/* ------------------------------------------------------------------------
 * Dense NNLS by Algorithm 1 (section "Solution algorithm"), the workload of
 * the efficiency experiment (section "Algorithm efficiency"): a random dense
 * B [m][n] (row-major), y [m], min over q >= 0 of ||B q - y||^2.  Each epoch
 * takes the rows in the order perm[e][0..m), in minibatches of `chunk` rows
 * (the last one shorter); a minibatch computes r = B_o q - y_o, g = B_o^T r,
 * the Adagrad (optimizer 0, PyTorch's form) or fixed step (optimizer 1), then
 * q = max(q, 0).  q, A [n] are updated in place; loss_hist [E] (or NULL)
 * receives ||B q - y||^2 after each epoch.
 * ---------------------------------------------------------------------- */
double orc_dense_loss(int32_t m, int32_t n, const double* B, const double* y, const double* q) {
  double s = 0.0;
  for (int32_t i = 0; i < m; ++i) {
    double v = 0.0;
    for (int32_t j = 0; j < n; ++j) v += B[IDX2(i, j, n)] * q[j];
    v -= y[i];
    s += v * v;
  }
  return s;
}

int orc_dense_spgd(int32_t m, int32_t n, const double* B, const double* y, double* q, double* A,
                   const int32_t* perm, int32_t E, int32_t chunk, int32_t optimizer, double eta,
                   double eps, double* loss_hist) {
  if (chunk <= 0 || m < 0 || n < 0) return 1;
  double* r = (double*)malloc(sizeof(double) * (size_t)(chunk > 0 ? chunk : 1));
  double* g = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!r || !g) {
    free(r); free(g);
    return 2;
  }
  for (int32_t e = 0; e < E; ++e) {
    const int32_t* pe = perm + (int64_t)e * m;
    for (int32_t s0 = 0; s0 < m; s0 += chunk) {
      const int32_t nr = s0 + chunk < m ? chunk : m - s0;
      for (int32_t i = 0; i < nr; ++i) {
        const double* row = B + (int64_t)pe[s0 + i] * n;
        double v = 0.0;
        for (int32_t j = 0; j < n; ++j) v += row[j] * q[j];
        r[i] = v - y[pe[s0 + i]];
      }
      for (int32_t j = 0; j < n; ++j) g[j] = 0.0;
      for (int32_t i = 0; i < nr; ++i) {
        const double* row = B + (int64_t)pe[s0 + i] * n;
        for (int32_t j = 0; j < n; ++j) g[j] += row[j] * r[i];
      }
      for (int32_t j = 0; j < n; ++j) {
        if (optimizer == 0) {
          A[j] += g[j] * g[j];
          q[j] -= eta * g[j] / (sqrt(A[j]) + eps);
        } else {
          q[j] -= eta * g[j];
        }
        if (!(q[j] > 0.0)) q[j] = 0.0;
      }
    }
    if (loss_hist) loss_hist[e] = orc_dense_loss(m, n, B, y, q);
  }
  free(r); free(g);
  return 0;
}
