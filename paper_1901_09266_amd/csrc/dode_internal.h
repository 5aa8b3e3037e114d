// Internal declarations shared by the host API and the kernel files of libdode.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dode.h"

// Device view of the incidence pattern (CSR by link and CSC by OD).
struct DevPat {
  int32_t P, L, T, H, K;
  int64_t nnz;
  const int32_t* row_ptr;   // [L+1]
  const int32_t* col;       // [nnz]  OD of CSR entry j
  const int32_t* col_ptr;   // [P+1]
  const int32_t* row;       // [nnz]  link of CSC entry jj
};

// Device view of the value arrays of all clusters.
//   W : CSR order  [C][K][T][nnz]
//   WT: CSC order  [C][K][T][nnz]
//   scale (FP8 only): [C][K][T][n_ptile], one float per 64-OD column tile
struct DevVals {
  const void* W;
  const void* WT;
  const float* scale;
  int64_t cstride;       // K*T*nnz
  int32_t n_ptile;       // ceil(P/64)
};

// Dense MFMA tiles of the assignment blocks (BF16 / FP8 storage).
//   forward:  link tile i (16 links) x OD hull [f_plo[i], f_plo[i] + 32*f_ks[i])
//   adjoint:  OD tile j (16 ODs) x link hull [g_alo[j], g_alo[j] + 32*g_ks[j])
// Values of block (c, l, t) are stored per 16x32 k-step in MFMA operand order
// (lane-major, 8 consecutive k per lane): Fv[c][l][t][kf_total][64 lanes][8].
// FP8 storage keeps one float scale per 16-row tile and k-step range:
//   Fsc[c][l][t][kf_total], Gsc[c][l][t][kg_total].
struct DevTiles {
  int32_t nLT = 0, nPT = 0, kf_total = 0, kg_total = 0;
  const int32_t* f_plo = nullptr;
  const int32_t* f_ks = nullptr;
  const int32_t* f_koff = nullptr;
  const int32_t* g_alo = nullptr;
  const int32_t* g_ks = nullptr;
  const int32_t* g_koff = nullptr;
  const void* Fv = nullptr;
  const void* Gv = nullptr;
  const float* Fsc = nullptr;
  const float* Gsc = nullptr;
};

struct dode_dar {
  dode_dims dims{};
  int32_t C = 0;
  int64_t nnz = 0;
  dode_dtype storage = DODE_F32;
  int device = 0;
  int32_t* d_row_ptr = nullptr;
  int32_t* d_col = nullptr;
  int32_t* d_col_ptr = nullptr;
  int32_t* d_row = nullptr;
  int32_t* d_csc2csr = nullptr;   // CSC slot -> CSR slot
  int32_t* d_row_of_nz = nullptr; // link of CSR slot j
  void* d_W = nullptr;
  void* d_WT = nullptr;
  float* d_scale = nullptr;
  int64_t device_bytes = 0;
  std::vector<int32_t> h_row_ptr, h_col, h_col_ptr, h_row, h_csc2csr;
  // MFMA tile layout (BF16 / FP8 storage only)
  bool has_tiles = false;
  DevTiles tiles;
  int32_t* d_tile_meta = nullptr;   // f_plo | f_ks | f_koff | g_alo | g_ks | g_koff
  int32_t* d_posf = nullptr;        // [nnz] element offset of CSR slot j in a forward block
  int32_t* d_posg = nullptr;        // [nnz] element offset of CSC slot jj in an adjoint block
  void* d_Fv = nullptr;
  void* d_Gv = nullptr;
  float* d_Fsc = nullptr;
  float* d_Gsc = nullptr;

  DevPat pat() const {
    return DevPat{dims.P, dims.L, dims.T, dims.H, dims.K, nnz, d_row_ptr, d_col, d_col_ptr, d_row};
  }
  DevVals vals() const {
    return DevVals{d_W, d_WT, d_scale, (int64_t)dims.K * dims.T * nnz, (dims.P + 63) / 64};
  }
};

// Device view of a route-choice structure (see dode_routes_create).
struct DevRoutes {
  int32_t P, L, T, H, K, n_paths;
  int64_t nnz, n_pairs;
  const int32_t* path_od;     // [n_paths]
  const int32_t* pair_ptr;    // [n_paths+1]
  const int32_t* pair_nz;     // [n_pairs]
  const int32_t* pair_path;   // [n_pairs]
  const int32_t* od_ptr;      // [P+1]   paths grouped by OD
  const int32_t* od_paths;    // [n_paths]
  const int32_t* nz_ptr;      // [nnz+1] pairs grouped by pattern entry
  const int32_t* nz_pairs;    // [n_pairs]
};

struct dode_routes {
  DevRoutes dv{};
  int device = 0;
  int32_t* d_buf = nullptr;   // all index arrays above, one allocation
};

// Optimizer settings as the kernels see them.
struct StepArgs {
  double eta;
  double eps;
  int32_t optimizer;   // 0 Adagrad, 1 fixed step
};

// Schedule of one minibatch ("chunk") for the grouped kernels.  Minibatch j
// of an epoch holds positions j0 = j*bh .. j0+bh-1 of each cluster's
// permutation of the H observation intervals.
//   perm[c][H]      the epoch's permutation of cluster c
//   pos[c][H]       its inverse (position of interval h)
//   touched[c][mt]  departure intervals the minibatch reaches (-1 padded)
struct ChunkSched {
  const int32_t* perm;
  const int32_t* pos;
  const int32_t* touched;
  int32_t j0;
  int32_t bh;
  int32_t max_touched;
};

// Groups of up to 32 days of one cluster (two 16-day MFMA column tiles).
struct DayGroups {
  const int32_t* cluster;   // [n]
  const int32_t* first;     // [n] offset into days
  const int32_t* count;     // [n] 1..32
  const int32_t* days;      // [D] day indices grouped by cluster
  int32_t n;
};

// Minibatch schedule and scratch of spgd_run (see spgd_plan_create).
struct dode_plan {
  const dode_dar* dar = nullptr;
  int device = 0;
  int32_t D = 0, E = 0, C = 0, bh = 0, nch = 0, mt = 0;
  StepArgs sa{};
  int32_t* d_perm = nullptr;      // [E][C][H]
  int32_t* d_pos = nullptr;       // [E][C][H]
  int32_t* d_touched = nullptr;   // [E][nch][C][mt]
  int32_t* d_dc = nullptr;        // [D]
  void* d_R = nullptr;            // [D][bh][L] residual rows of the current minibatch
  double* d_part = nullptr;       // [D][H] loss partials
  int32_t* d_groups = nullptr;    // cluster | first | count (n_groups each) | days [D]
  int32_t n_groups = 0;
  bool use_mfma = false;
  hipStream_t last_stream = nullptr;
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];

  DayGroups groups() const {
    return DayGroups{d_groups, d_groups + n_groups, d_groups + 2 * n_groups, d_groups + 3 * n_groups,
                     n_groups};
  }
  ChunkSched chunk(int32_t e, int32_t j) const {
    const int32_t H = dar->dims.H;
    return ChunkSched{d_perm + (size_t)e * C * H, d_pos + (size_t)e * C * H,
                      d_touched + ((size_t)e * nch + j) * C * mt, j * bh, bh, mt};
  }
};

bool is_f64(const dode_dar* d);

// ---- plain kernels (plain_kernels.hip) ---------------------------------
// All launchers return hipSuccess or the launch error.  `day_cluster` may be
// nullptr, then every day belongs to `cluster`.
hipError_t plain_chunk_resid(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                             const ChunkSched& cs, const void* Q, const void* X, void* R,
                             int32_t n_days, hipStream_t s);
hipError_t plain_chunk_adj_step(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                                const ChunkSched& cs, const void* R, void* Q, void* A,
                                int32_t n_days, const StepArgs& st, hipStream_t s);
// out (nullable) = rho Q (- X if X); part (nullable) = per (day, h) sum of squares of that
hipError_t plain_apply_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                            const void* Q, const void* X, void* out, double* part, int32_t n_days,
                            hipStream_t s);
// G = rho^T R for full residual rows R [n][H][L]
hipError_t plain_adjoint_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                              const void* R, void* G, int32_t n_days, hipStream_t s);

// ---- MFMA tile kernels (mfma_kernels.hip) -------------------------------
hipError_t mfma_chunk_resid(const dode_dar* dar, const ChunkSched& cs, const DayGroups& dg,
                            const float* Q, const float* X, float* R, hipStream_t s);
hipError_t mfma_chunk_adj_step(const dode_dar* dar, const ChunkSched& cs, const DayGroups& dg,
                               const float* R, float* Q, float* A, const StepArgs& st,
                               hipStream_t s);
// host: build the tile layout of all clusters from FP64 values (tiles.hip)
dode_status build_tiles(dode_dar* d, const double* const* values, std::string& err);

// ---- differentiation (route_kernels.hip) --------------------------------
hipError_t routes_rho(const DevRoutes& r, bool f64, const void* Rr, const void* z, void* W,
                      double* pi, hipStream_t s);
hipError_t routes_logits_bwd(const DevRoutes& r, bool f64, const void* Rr, const void* z,
                             const void* dW, void* dz, double* pi, double* dpi, hipStream_t s);
hipError_t loss_bwd_dW(const dode_dar* dar, const void* R, const void* Q, int32_t n_days,
                       double scale, void* dW, hipStream_t s);
hipError_t scale_state(bool f64, void* x, int64_t n, double f, hipStream_t s);
// rewrite the MFMA tiles of one cluster from state-typed values [K][T][nnz]
hipError_t update_tiles(const dode_dar* dar, int32_t cluster, const void* W_state, hipStream_t s);

// ---- small generic kernels (plain_kernels.hip) -------------------------
hipError_t sum_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s);
hipError_t kkt_partials(bool f64, const void* Q, const void* G, int32_t T, int32_t P,
                        int32_t n_days, double* part, hipStream_t s);
hipError_t max_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s);
hipError_t x_moment_partials(bool f64, const void* X, int32_t H, int32_t L, int32_t n_days,
                             const double* sum_x /* nullable: first moment pass */, double* part,
                             hipStream_t s);
hipError_t r2_finish(const double* loss, const double* sst, int32_t n_days, double* r2,
                     hipStream_t s);
hipError_t check_finite(bool f64, const void* X, int64_t n, int32_t* flag, hipStream_t s);
hipError_t clamp_nonneg(bool f64, void* Q, int64_t n, hipStream_t s);
hipError_t quantize_values(const dode_dar* dar, int32_t cluster, const void* W_state,
                           hipStream_t s);

// ---- number formats (host side, exact round-to-nearest-even) -----------
uint16_t host_f64_to_bf16(double v);
uint8_t host_f64_to_e4m3(double v);   // v already scaled into [-448, 448]
double host_bf16_to_f64(uint16_t b);
double host_e4m3_to_f64(uint8_t b);
