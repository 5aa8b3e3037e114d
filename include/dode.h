/*
 * dode.h -- C ABI of the MI355X library for the per-day dynamic OD estimation
 * problem of Ma & Qian, "Estimating multi-year 24/7 origin-destination demand
 * using high-granular multi-source traffic data" (arXiv 1901.09266).
 *
 * The library solves, for every day d of traffic-pattern cluster c,
 *     min_{q_d >= 0} || rho_c q_d - x_d ||_2^2          (eq. "nnls")
 * with the stochastic projected gradient descent of Algorithm 1 ("SPGD"),
 * batched over days (days are independent subproblems, section "Estimate the
 * dynamic OD demand").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Dimensions: P OD pairs, L observed links, T departure intervals, H
 *    observation intervals, K lag band (rho_c has a nonzero block for
 *    departure interval t and observation interval h only if 0 <= h-t < K).
 *  - Per-day vectors are interval-major (Table "DODE framework variable
 *    vectorization"): demand q[t][p] (T*P values), counts x[h][a] (H*L values).
 *    A batch of n days is day-major: Q[n][T][P], X[n][H][L].
 *  - rho_c is given by a static incidence pattern shared by all clusters (CSR
 *    over links: row_ptr[L+1], col_idx[nnz] = the ODs whose route crosses link
 *    a, strictly increasing within a row) and per-cluster values W_c[K][T][nnz]:
 *        rho_c[(t+l)*L + a, t*P + p] = W_c[l][t][nz(a,p)]     (eq. "assign")
 *    Values of blocks with t+l >= H are ignored (spill-over past the last
 *    interval is dropped).
 *  - State type: a handle created with storage DODE_F64 works on double
 *    Q, X, A, G, Xhat buffers; every other storage works on float buffers.
 *  - Device buffers (Q, X, A, G, Xhat, loss outputs marked "dev") are owned by
 *    the caller and are never freed by the library.  Host buffers are read or
 *    written before the call returns unless stated otherwise.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *    on it and return; calls that return host results synchronise it.
 *  - Argument and shape errors are detected before any launch and returned as
 *    a status; HIP failures return DODE_ERR_HIP.  dode_last_error() gives the
 *    message of the last failing call of the calling thread.  No C++
 *    exception crosses this interface.
 *  - A handle is immutable after creation except through dar_set_values;
 *    concurrent calls that only read one handle are safe.
 */
#ifndef DODE_H
#define DODE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DODE_OK = 0,
  DODE_ERR_ARG = 1,         /* NULL pointer, bad enum or parameter value */
  DODE_ERR_SHAPE = 2,       /* inconsistent dimensions or pattern */
  DODE_ERR_DTYPE = 3,       /* storage type not usable for this call */
  DODE_ERR_NONFINITE = 4,   /* NaN or Inf in the observations or values */
  DODE_ERR_OOM = 5,         /* device allocation failed */
  DODE_ERR_HIP = 6,         /* a HIP runtime call failed */
  DODE_ERR_UNSUPPORTED = 7  /* valid request the library does not implement */
} dode_status;

typedef enum {
  DODE_F64 = 0,       /* values and state in double */
  DODE_F32 = 1,       /* values and state in float */
  DODE_BF16 = 2,      /* values bfloat16 (round to nearest even), state float */
  DODE_FP8_E4M3 = 3   /* values OCP E4M3FN with one float scale per (cluster, l, t,
                         64-OD column tile); state float */
} dode_dtype;

typedef struct {
  int32_t P, L, T, H, K;
} dode_dims;

typedef struct dode_dar dode_dar;   /* opaque, library-owned */

typedef struct {
  int32_t epochs;      /* E, number of passes over the rows (paper: 300) */
  int32_t batch_rows;  /* b, rows per minibatch (paper: 8192); rounded down to
                          whole observation intervals: b_h = max(1, b / L) */
  double eta;          /* learning rate (paper: 5) */
  double eps;          /* Adagrad denominator offset, added after the square root */
  int32_t optimizer;   /* 0 = Adagrad (Algorithm 1), 1 = fixed step q -= eta g */
  int32_t check_finite;/* nonzero: scan X for NaN/Inf before solving */
  int32_t kernel_path; /* 0 = fastest available for the storage type (matrix-core
                          tiles for BF16 / FP8 when a cluster has more than 2
                          days or refine_steps > 0, a forward and an adjoint
                          launch per minibatch, else the sparse kernels),
                          1 = sparse pattern kernels, 2 = matrix-core tiles
                          with one launch per minibatch, one workgroup per
                          independent part of it, 3 = matrix-core tiles with
                          one cooperative launch per epoch whose resident
                          workgroups meet at a grid barrier between the
                          forward and adjoint phases of every minibatch (needs
                          a given day_tile and one day slab; the chunked
                          adjoint only with day_tile 16; refinement steps run
                          as separate launches after it; spgd_run then waits
                          for the stream once per call to check the barrier).
                          2 and 3 give the same bits as 0 and are slower on
                          the benchmark workloads */
  int32_t use_graph;   /* nonzero: spgd_run replays one captured hipGraph per epoch
                          (the epoch index lives in a device counter) */
  int32_t day_tile;    /* days of one cluster handled together by a matrix-core
                          wave (the GEMM N dimension): 16, 32 or 64; 0 = let
                          spgd_plan_load choose the matrix-core schedule (day
                          tile, adjoint order, day slabs) by timing an epoch of
                          every candidate,
                          or reuse the choice made earlier in this process for
                          the same shapes, storage and GPU, or recorded for
                          them in the file named by the environment variable
                          DODE_SCHEDULE_CACHE (each new choice is appended
                          there as "<key> TAB <day tile> <adj_order> <slabs>
                          <ms>"; unreadable or invalid lines are skipped);
                          results are the same bits for every choice */
  int32_t refine_steps;/* full-batch refinement steps after the minibatches of
                          every epoch: each is one step of Algorithm 1 with all
                          H intervals as its minibatch, computed with the
                          corrected values of an FP8 assignment (needs a dar
                          built with DODE_DAR_CORRECTION); 0 = none */
  int32_t adj_order;   /* order of the matrix-core adjoint's work items when
                          day_tile != 0: 0 = by reached interval, OD tiles
                          fastest; 1 = by OD tile, reached intervals fastest
                          (neighbouring waves share residual rows); 2 = one
                          wave per run of up to 6 consecutive reached
                          intervals, which loads each residual row once for
                          the run; by run, then OD tile, day groups fastest
                          (neighbouring waves share the run's tiles; also
                          used by the refinement steps; not with day_tile 64,
                          an argument error); same bits */
  int32_t slabs;       /* day slabs of a matrix-core epoch when day_tile != 0:
                          the day groups split into `slabs` parts of about
                          D/slabs days, each with its own launches of every
                          minibatch, run at the same time on streams of their
                          own (forked from and joined to the run's stream in
                          every epoch, also inside the epoch graph), so one
                          part's launches fill the others' ramp and tail;
                          0 or 1 = all days together; same bits */
} dode_spgd_params;

/* Message of the last failing call on this thread ("" if none). */
const char* dode_last_error(void);

/* Fill p with the defaults: epochs 300, batch_rows 8192, eta 5, eps 1e-10,
 * Adagrad, check_finite 1, kernel_path 0, use_graph 1, day_tile 32,
 * refine_steps 0, adj_order 1, slabs 1 (section "Goodness of fit" gives E, b
 * and eta). */
void dode_spgd_defaults(dode_spgd_params* p);

/*
 * Build a device copy of the assignment matrices rho_c of n_clusters clusters
 * (eq. "assign"; the COO sparse layout of section "Tensor representation" is
 * replaced by the band form described above).
 *   dims            P, L, T, H, K (all >= 1)
 *   row_ptr, col_idx  host CSR incidence pattern (see conventions)
 *   values          host array of n_clusters pointers, each to FP64 [K][T][nnz]
 *   storage         value type kept on the device
 *   out             receives the handle; release it with dar_destroy
 * Errors: DODE_ERR_SHAPE for a malformed pattern, DODE_ERR_NONFINITE for
 * non-finite values, DODE_ERR_OOM, DODE_ERR_HIP.  Synchronises `stream`.
 */
dode_status dar_create(const dode_dims* dims, int32_t n_clusters, const int32_t* row_ptr,
                       const int32_t* col_idx, const double* const* values, dode_dtype storage,
                       void* stream, dode_dar** out);

/*
 * dar_create with options.  flags is 0 or DODE_DAR_CORRECTION: for FP8
 * storage, also keep bfloat16 correction tiles c = bf16(w - h), where
 * h = bf16(scale * e4m3(w / scale)) is the FP8 value as the kernels expand it,
 * so that h + c matches w to about 2^-13 relative; refinement steps
 * (dode_spgd_params.refine_steps) multiply with h + c.  dar_set_values is not
 * supported on such a handle (DODE_ERR_UNSUPPORTED).  DODE_ERR_ARG for a flag
 * that does not apply to the storage type.
 */
#define DODE_DAR_CORRECTION 1
dode_status dar_create_ex(const dode_dims* dims, int32_t n_clusters, const int32_t* row_ptr,
                          const int32_t* col_idx, const double* const* values,
                          dode_dtype storage, int32_t flags, void* stream, dode_dar** out);

/* Free a handle (NULL is a no-op).  The caller must have finished every call
 * that uses it. */
dode_status dar_destroy(dode_dar* dar);

/* Shape, cluster count, pattern size, storage type and device bytes of a handle.
 * Any output pointer may be NULL. */
dode_status dar_info(const dode_dar* dar, dode_dims* dims, int32_t* n_clusters, int64_t* nnz,
                     dode_dtype* storage, int64_t* device_bytes);

/* Replace cluster c's values with the device array W_dev (state type,
 * [K][T][nnz]) -- used when rho_c is a learned function of route logits.
 * For reduced storage the values are rounded (and FP8 scales recomputed) on
 * the device.  Asynchronous on `stream`. */
dode_status dar_set_values(dode_dar* dar, int32_t cluster, const void* W_dev, void* stream);

/* Xhat = rho_c Q for n_days days of cluster c (eq. "finalobj").
 *   Q dev [n][T][P], Xhat dev [n][H][L], state type. */
dode_status dode_apply(const dode_dar* dar, int32_t cluster, const void* Q, int32_t n_days,
                       void* Xhat, void* stream);

/* loss[d] = || rho_c q_d - x_d ||^2 per day (eq. "nnls"), accumulated in FP64
 * in a fixed order (bitwise reproducible).  loss dev double [n]. */
dode_status dode_loss(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                      int32_t n_days, double* loss, void* stream);

/*
 * dode_loss for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (the same bits) as dode_loss; it calls no
 * allocator.  Its per-row partials live in one fixed 4 MiB device array per
 * GPU, so n_days * H * 8 bytes must fit in 4 MiB (1820 days at H = 288):
 * larger calls return DODE_ERR_ARG before any launch.  The current device
 * must be the dar's (DODE_ERR_ARG otherwise).  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (concurrent streams, or threads)
 * race and may return wrong losses; serialise them, as one stream does.
 */
dode_status dode_loss_noalloc(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                              int32_t n_days, double* loss, void* stream);

/* G = rho_c^T (rho_c Q - X), Algorithm 1's gradient (half the gradient of the
 * loss).  G dev [n][T][P], state type. */
dode_status dode_grad(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                      int32_t n_days, void* G, void* stream);

/* End-of-solve figures per day (Step 6 "Quality check"), all FP64 dev [n],
 * each may be NULL:  loss as dode_loss;  kkt = max_i |min(q_i, g_i)| with the
 * full gradient g;  r2 = 1 - sum (x - xhat)^2 / sum (x - mean x)^2. */
dode_status dode_metrics(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                         int32_t n_days, double* loss, double* kkt, double* r2, void* stream);

/*
 * One minibatch of Algorithm 1 for n_days days of cluster c, on the rows of
 * the n_h observation intervals chunk_h (host, distinct, each in [0, H)):
 *   g = rho_o^T (rho_o q - x_o)  with rho_o the chunk's rows,
 *   Adagrad (A += g*g; q -= eta g / (sqrt(A) + eps)) or fixed step, q = max(q, 0).
 * Only the coordinates (t, p) that the chunk reaches (h - K < t <= h) are
 * written; the others have g = 0 and keep their value (the same as the
 * algorithm when Q >= 0 on entry).  X dev, Q and A dev (in/out), state type.
 */
dode_status spgd_step(const dode_dar* dar, int32_t cluster, const int32_t* chunk_h, int32_t n_h,
                      const void* X, void* Q, void* A, int32_t n_days,
                      const dode_spgd_params* params, void* stream);

/*
 * Algorithm 1 for D days of any clusters in one call (all clusters advance
 * together, one minibatch at a time).
 *   day_cluster  host [D], cluster of each day
 *   X dev [D][H][L]; Q, A dev [D][T][P] (in/out; pass A = 0 and the starting
 *                Q, e.g. 0, to start fresh; Q is projected onto Q >= 0 first)
 *   perm         host [E][C][H]: the permutation of the H observation
 *                intervals of each (epoch, cluster); NULL = drawn by the library
 *                from `seed`: one SplitMix64 stream (Steele, Lea and Flood
 *                2014) started at `seed`, and for each (epoch, cluster) in
 *                order a Fisher-Yates shuffle of 0..H-1 from the top, element
 *                i swapping with element (next draw mod (i + 1)), i = H-1..1
 *   loss_hist    host [D][E] or NULL: full loss of each day after each epoch
 *                (costs one extra forward pass per epoch; synchronises stream)
 * The minibatches of epoch e and cluster c are consecutive slices of b_h
 * intervals of perm[e][c]; the last may be shorter.
 */
dode_status spgd_solve(const dode_dar* dar, const int32_t* day_cluster, int32_t D, const void* X,
                       void* Q, void* A, const dode_spgd_params* params, const int32_t* perm,
                       uint64_t seed, double* loss_hist, void* stream);

/*
 * Gradients of the summed loss f = grad_out * sum_d ||rho_c q_d - x_d||^2 over
 * n_days days of cluster c (eq. "nnls"), for learning rho_c or the route
 * parameters behind it.  The residual r_d = rho_c q_d - x_d is recomputed,
 * not stored.
 *   dQ  dev [n][T][P], state type, or NULL:  dQ_d = 2 grad_out rho_c^T r_d
 *   dW  dev [K][T][nnz], state type, or NULL:
 *         dW[l][t][nz(a,p)] = 2 grad_out sum_d r_d[t+l][a] q_d[t][p]
 *       (entries of blocks with t+l >= H are set to 0)
 */
dode_status dode_loss_bwd(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                          int32_t n_days, double grad_out, void* dQ, void* dW, void* stream);

/*
 * Route-choice parameterisation of rho_c (eqs. "logit", "flow", "assign"):
 * path k serves OD path_od[k] and crosses the links
 * pair_link[pair_ptr[k] .. pair_ptr[k+1]); pair m feeds pattern entry
 * pair_nz[m] (the (link, OD) entry of the incidence pattern).  With
 * per-pair lag ratios Rr[l][t][m] and logits z,
 *   pi_k = softmax of z over the paths of OD path_od[k]   (time invariant)
 *   W[l][t][nz] = sum over pairs m feeding nz of Rr[l][t][m] * pi_{path(m)}
 * All host arrays are copied; the handle is immutable.  n_pairs = pair_ptr[n_paths].
 */
typedef struct dode_routes dode_routes;

dode_status dode_routes_create(const dode_dims* dims, int64_t nnz, int32_t n_paths,
                               const int32_t* path_od, const int32_t* pair_ptr,
                               const int32_t* pair_link, const int32_t* pair_nz, void* stream,
                               dode_routes** out);

dode_status dode_routes_destroy(dode_routes* routes);

/* W = rho(z) as above.  Rr dev [K][T][n_pairs], z dev [n_paths], W dev
 * [K][T][nnz]; `f64` selects double (else float) for all three.  The result
 * can be installed with dar_set_values. */
dode_status dar_from_logits(const dode_routes* routes, int32_t f64, const void* Rr, const void* z,
                            void* W, void* stream);

/* Chain rule from dW (dev [K][T][nnz]) to the logits (eq. "logit"):
 *   dpi_k = sum_{l,t, pairs m of k} Rr[l][t][m] dW[l][t][pair_nz[m]]
 *   dz_k  = pi_k (dpi_k - sum_{k' serving od(k)} pi_k' dpi_k')
 * dz dev [n_paths]; sums are taken in FP64 in a fixed order. */
dode_status dar_logits_bwd(const dode_routes* routes, int32_t f64, const void* Rr, const void* z,
                           const void* dW, void* dz, void* stream);

/*
 * Dynamic assignment ratios of paths from link speeds (section "Dynamic
 * assignment ratio", eqs. "dar2"/"dar" and Example "DAR matrix computation";
 * section "Link/path travel time", eq. "cost").  All arrays are device memory.
 *   path_ptr [n_paths+1], path_link [n_pairs]: the links of each path in the
 *       order they are traversed; pair m = path_ptr[k] + i is the i-th link
 *       of path k (the pair order of dode_routes_create)
 *   link_len [L], speed [n_days][L][H_speed]: positive and finite, in
 *       consistent units (e.g. miles and miles per minute); dt is the interval
 *       length in the time unit of len/speed
 *   Rr [K][H][n_pairs] (output): for departure interval t and lag l, the
 *       share of the vehicles of path k departing in t that enter link i in
 *       interval t+l, averaged over the n_days days (one ratio set per traffic
 *       pattern).  Link a entered at time x is crossed in
 *       len[a] / speed[a][floor(x/dt)] (the last interval's speed after the
 *       day); an interval maps onto the window between the entry times of its
 *       two boundary departures, and the ratios are the window's shares of the
 *       observation intervals.  Shares past interval H-1 or at lags >= K are
 *       dropped.
 *   f64: nonzero for double arrays, else float.  K <= 16.
 * Errors: DODE_ERR_SHAPE for malformed path tables, DODE_ERR_ARG for
 * non-positive or non-finite lengths or speeds.  Synchronises `stream` (the
 * path tables and the checks are read back); uses a scratch buffer of at
 * most 4 GiB (the trajectories of a chunk of days), or of the byte count in
 * the environment variable DODE_DAR_SCRATCH_BYTES (smaller values process
 * fewer days at a time; a value that is not a positive integer is
 * DODE_ERR_ARG).  The results do not depend on the chunking beyond the
 * rounding of the running day sums.
 */
dode_status dode_dar_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                 const int32_t* path_link, int64_t n_pairs, int32_t L,
                                 const void* link_len, const void* speed, int32_t n_days,
                                 int32_t H_speed, double dt, int32_t H, int32_t K, int32_t f64,
                                 void* Rr, void* stream);

/*
 * dode_dar_from_speeds and, from the same trajectories, the mean path costs
 * of dode_path_costs for the H departure intervals (section "Route choice
 * portions", eqs. "logit" and "rt"; eq. "cost").  Arguments, checks, errors
 * and synchronisation as for dode_dar_from_speeds, plus
 *   cost [H][n_paths] (output, device, may be NULL): for departure interval t,
 *       the mean over the n_days days of the time to cross the whole path when
 *       leaving at t*dt (days summed in FP64).
 * The scratch grows by n_paths*(H+1) values per day of a chunk and an FP64
 * array of n_paths*H.
 */
dode_status dode_dar_costs_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                       const int32_t* path_link, int64_t n_pairs, int32_t L,
                                       const void* link_len, const void* speed, int32_t n_days,
                                       int32_t H_speed, double dt, int32_t H, int32_t K,
                                       int32_t f64, void* Rr, void* cost, void* stream);

/*
 * The ratios of several traffic patterns in one call, and optionally their
 * mean path costs (sections "Dynamic assignment ratio" and "Route choice
 * portions"; eqs. "dar2"/"dar", "cost", "logit"): pattern q averages days
 * pattern_ptr[q] .. pattern_ptr[q+1]-1 of speed [D][L][H_speed].
 *   pattern_ptr host [n_patterns+1], from 0 to D, every pattern non-empty
 *   Rr dev [n_patterns][K][H][n_pairs]; cost dev [n_patterns][H][n_paths] or NULL
 * Each pattern's results are the bits of dode_dar_costs_from_speeds on its
 * days.  The path tables and all D days' speeds are checked once for the job
 * (one read-back, one synchronisation), the scratch is allocated once; errors
 * as for dode_dar_from_speeds (DODE_ERR_SHAPE also for a malformed pattern_ptr).
 */
dode_status dode_dar_patterns_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                          const int32_t* path_link, int64_t n_pairs, int32_t L,
                                          const void* link_len, const void* speed,
                                          int32_t n_patterns, const int32_t* pattern_ptr,
                                          int32_t H_speed, double dt, int32_t H, int32_t K,
                                          int32_t f64, void* Rr, void* cost, void* stream);

/*
 * Mean path travel times of a traffic pattern (section "Route choice
 * portions", eqs. "logit" and "rt"; section "Link/path travel time",
 * eq. "cost").  Path tables, lengths and speeds as for dode_dar_from_speeds
 * (device memory, same checks and errors).
 *   cost [T][n_paths] (output, device): for departure interval t, the mean
 *       over the n_days days of the time a vehicle leaving at t*dt needs to
 *       cross every link of path k, each link at the speed of the interval in
 *       which it is entered (the last interval's speed after the day).  The
 *       start of the interval stands for the whole interval (eq. "rt").
 *   f64: nonzero for double arrays, else float; days are summed in FP64.
 * Synchronises `stream` (the path tables and checks are read back); uses a
 * scratch buffer of at most 256 MiB.
 */
dode_status dode_path_costs(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                            int64_t n_pairs, int32_t L, const void* link_len, const void* speed,
                            int32_t n_days, int32_t H_speed, double dt, int32_t T, int32_t f64,
                            void* cost, void* stream);

/*
 * Assignment matrix from path costs (eqs. "logit", "rt", "flow", "assign"):
 *   p[t][k] = exp(-theta cost[t][k]) / sum over the paths k' of OD(k) of
 *             exp(-theta cost[t][k'])                       (FP64 softmax)
 *   W[l][t][nz] = sum over the pairs m feeding nz of Rr[l][t][m] p[t][path(m)]
 * routes from dode_routes_create; Rr dev [K][T][n_pairs] (e.g. the output of
 * dode_dar_from_speeds when T = H, or its first T intervals), cost dev
 * [T][n_paths] (finite, in the time unit theta is the inverse of: 0.01 per
 * second is 0.6 per minute), W dev [K][T][nnz] (output), portions dev
 * [T][n_paths] (output, may be NULL).  `f64` selects double (else float) for
 * every array.  Asynchronous on `stream`; W can be installed with
 * dar_set_values.
 */
dode_status dar_from_costs(const dode_routes* routes, int32_t f64, const void* Rr, const void* cost,
                           double theta, void* portions, void* W, void* stream);

/*
 * Dense NNLS by Algorithm 1 (section "Solution algorithm"), the random dense
 * workload of the efficiency experiment (section "Algorithm efficiency"):
 * min over q >= 0 of ||B q - y||^2.
 *   B dev [m][n] row-major, y dev [m]; q, A dev [n] (in/out: the iterate and
 *       the Adagrad accumulator, usually zeros at the start)
 *   perms dev [E][m]: epoch e takes the rows in the order perms[e], in
 *       minibatches of `chunk` rows (the last one shorter); each minibatch
 *       computes r = B_o q - y_o, g = B_o^T r, then Adagrad (optimizer 0:
 *       A += g^2, q -= eta g / (sqrt(A) + eps)) or a fixed step (optimizer 1:
 *       q -= eta g), then q = max(q, 0)
 *   loss_hist host [E] or NULL: ||B q - y||^2 after each epoch (FP64 sum in
 *       a fixed order; costs one more pass over B per epoch)
 *   prec: 0 for float arrays, 1 for double arrays, 2 for B as bfloat16 bits
 *       (uint16, the upper half of the float) with y, q, A and all
 *       arithmetic in float.
 * Errors: DODE_ERR_ARG if a perms row is not a permutation of 0..m-1 (checked
 * on the host), for a non-positive eta or chunk, a negative eps or another
 * prec.
 * Synchronises `stream` (the permutations are read back first, and the loss
 * history after the run); scratch of m + ceil(min(chunk, m)/128)*n values.
 */
dode_status dense_spgd_run(int32_t m, int32_t n, int32_t prec, const void* B, const void* y, void* q,
                           void* A, const int32_t* perms, int32_t E, int32_t chunk,
                           int32_t optimizer, double eta, double eps, double* loss_hist,
                           void* stream);

/*
 * Reusable form of spgd_solve for repeated or timed runs.  A plan holds
 *  - the minibatch schedule of every epoch (permutations, their inverses and
 *    the departure intervals each minibatch reaches),
 *  - its own copy of the solver state of the D days -- X, Q and A -- in an
 *    interval-major layout ([rows][days][cols], days grouped by cluster) so
 *    that the rows one minibatch touches are contiguous across days,
 *  - the residual scratch of one minibatch,
 * all on the device of `dar`.  Arguments as for spgd_solve; `params->epochs`
 * is the number of epochs the schedule covers.  The plan keeps a pointer to
 * `dar`, which must outlive it.  The state starts at X = 0, Q = 0, A = 0;
 * fill it with spgd_plan_load.  Synchronises `stream`.
 */
typedef struct dode_plan dode_plan;

dode_status spgd_plan_create(const dode_dar* dar, const int32_t* day_cluster, int32_t D,
                             const dode_spgd_params* params, const int32_t* perm, uint64_t seed,
                             void* stream, dode_plan** out);

dode_status spgd_plan_destroy(dode_plan* plan);

/* Copy the caller's X (dev [D][H][L]), Q and A (dev [D][T][P], state type; A
 * may be NULL for zeros) into the plan, projecting Q onto Q >= 0 (day d is
 * day d of the plan's day_cluster).  With params->check_finite, X is scanned
 * for NaN/Inf first (DODE_ERR_NONFINITE; synchronises `stream`).  With
 * params->day_tile == 0 the first load of a matrix-core plan also times a few
 * minibatches at each day tile on this state, keeps the fastest, and loads Q
 * and A again (synchronises `stream`). */
dode_status spgd_plan_load(dode_plan* plan, const void* X, const void* Q, const void* A,
                           void* stream);

/* Copy the plan's Q (and A unless NULL) back to the caller (dev [D][T][P]). */
dode_status spgd_plan_store(const dode_plan* plan, void* Q, void* A, void* stream);

/*
 * Epochs epoch_begin .. epoch_begin+n_epochs-1 of the plan's schedule on the
 * plan's state.  loss_dev (dev double [n_epochs][D], caller's day order)
 * receives the full loss of each day after each epoch, or pass NULL to skip
 * that extra forward pass.  Asynchronous on `stream`; calls on one plan must
 * not overlap (they share its state and scratch).
 */
dode_status spgd_run(dode_plan* plan, int32_t epoch_begin, int32_t n_epochs, double* loss_dev,
                     void* stream);

/*
 * Kernel timing of a plan.  enable != 0 makes later spgd_run calls record a
 * HIP event pair around every kernel launch on the run's stream (day slabs
 * then run one after another on that stream, each launch alone); the summed
 * durations in milliseconds (host [3]: forward-residual launches, adjoint-step
 * launches or whole-minibatch launches of the one-launch path, loss kernels)
 * and the launch counts (host [3]) are returned and reset by the next call
 * (which synchronises the last run's stream).
 */
dode_status spgd_plan_timing(dode_plan* plan, int32_t enable, double* ms, int64_t* launches);

/* Shape of a plan's schedule (any pointer may be NULL): the day tile in use
 * (0 for the sparse pattern kernels), minibatches per epoch, intervals per
 * minibatch (b_h) and day groups. */
dode_status spgd_plan_info(const dode_plan* plan, int32_t* day_tile, int32_t* n_minibatches,
                           int32_t* minibatch_intervals, int32_t* n_day_groups);

/* Matrix-core schedule of a plan (any pointer may be NULL): the day tile,
 * adjoint item order and day slabs in use, the number of candidates timed at
 * load (0 when given by the caller, or taken from this process's earlier
 * choice or the DODE_SCHEDULE_CACHE file for the same P, L, T, H, K, b_h,
 * storage, refinement steps, cluster sizes and GPU architecture), and the time
 * in milliseconds of the chosen candidate's trial epoch (0 if none ran).  A
 * sparse-kernel plan reports day tile 0. */
dode_status spgd_plan_schedule(const dode_plan* plan, int32_t* day_tile, int32_t* adj_order,
                               int32_t* n_slabs, int32_t* n_timed, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* DODE_H */
