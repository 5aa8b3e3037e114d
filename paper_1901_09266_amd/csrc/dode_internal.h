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
  void* d_W = nullptr;
  void* d_WT = nullptr;
  float* d_scale = nullptr;
  int64_t device_bytes = 0;
  std::vector<int32_t> h_row_ptr, h_col, h_col_ptr, h_row, h_csc2csr;

  DevPat pat() const {
    return DevPat{dims.P, dims.L, dims.T, dims.H, dims.K, nnz, d_row_ptr, d_col, d_col_ptr, d_row};
  }
  DevVals vals() const {
    return DevVals{d_W, d_WT, d_scale, (int64_t)dims.K * dims.T * nnz, (dims.P + 63) / 64};
  }
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
