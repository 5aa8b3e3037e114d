// Sparse (pattern-compact) kernels of libdode: the general path for every
// storage type.  Each thread owns one output entry and walks the pattern, so
// results are deterministic (fixed summation order, no atomics).
//
// Algorithm 1 (section "Non-negative least square on GPU") per minibatch:
//   chunk_resid   : r = rho_o q - x_o on the minibatch rows (eq. "finalobj")
//   chunk_adj_step: g = rho_o^T r, then Adagrad / fixed step and max(q, 0),
//                   fused, for every departure interval the minibatch reaches.
#include "dode_internal.h"
#include "numfmt.h"

#include <cmath>

namespace {

constexpr int kRowsBlock = 256;
constexpr int kColsBlock = 64;
constexpr int kRedBlock = 256;
constexpr size_t kQStageBytes = 32768;   // demand rows staged in LDS by the forward

// ---------------------------------------------------------------- values --
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// OCP E4M3FN: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits; exponent
// field 0 is subnormal (m * 2^-9); the all-ones code is NaN (never stored).
__device__ __forceinline__ float e4m3_bits_to_f32(uint8_t b) {
  const uint32_t e = (b >> 3) & 0xF, m = b & 7;
  float v = e == 0 ? static_cast<float>(m) * 0x1p-9f : __uint_as_float(((e + 120u) << 23) | (m << 20));
  return (b & 0x80) ? -v : v;
}

template <int ST>
struct Load;
template <>
struct Load<DODE_F64> {
  __device__ static double get(const void* W, int64_t i, const float*, int64_t) {
    return static_cast<const double*>(W)[i];
  }
};
template <>
struct Load<DODE_F32> {
  __device__ static float get(const void* W, int64_t i, const float*, int64_t) {
    return static_cast<const float*>(W)[i];
  }
};
template <>
struct Load<DODE_BF16> {
  __device__ static float get(const void* W, int64_t i, const float*, int64_t) {
    return bf16_bits_to_f32(static_cast<const uint16_t*>(W)[i]);
  }
};
template <>
struct Load<DODE_FP8_E4M3> {
  __device__ static float get(const void* W, int64_t i, const float* scale, int64_t si) {
    return e4m3_bits_to_f32(static_cast<const uint8_t*>(W)[i]) * scale[si];
  }
};

// Two neighbouring values i, i+1 (i even) with one load.
template <int ST>
struct Load2;
template <>
struct Load2<DODE_F64> {
  __device__ static void get(const void* W, int64_t i, const float*, int64_t, int64_t, double& w0,
                             double& w1) {
    const double2 v = *reinterpret_cast<const double2*>(static_cast<const double*>(W) + i);
    w0 = v.x;
    w1 = v.y;
  }
};
template <>
struct Load2<DODE_F32> {
  __device__ static void get(const void* W, int64_t i, const float*, int64_t, int64_t, float& w0,
                             float& w1) {
    const float2 v = *reinterpret_cast<const float2*>(static_cast<const float*>(W) + i);
    w0 = v.x;
    w1 = v.y;
  }
};
template <>
struct Load2<DODE_BF16> {
  __device__ static void get(const void* W, int64_t i, const float*, int64_t, int64_t, float& w0,
                             float& w1) {
    const uint32_t b = *reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(W) + i);
    w0 = bf16_bits_to_f32(static_cast<uint16_t>(b & 0xFFFFu));
    w1 = bf16_bits_to_f32(static_cast<uint16_t>(b >> 16));
  }
};
template <>
struct Load2<DODE_FP8_E4M3> {
  __device__ static void get(const void* W, int64_t i, const float* scale, int64_t si0, int64_t si1,
                             float& w0, float& w1) {
    const uint16_t b = *reinterpret_cast<const uint16_t*>(static_cast<const uint8_t*>(W) + i);
    w0 = e4m3_bits_to_f32(static_cast<uint8_t>(b & 0xFFu)) * scale[si0];
    w1 = e4m3_bits_to_f32(static_cast<uint8_t>(b >> 8)) * scale[si1];
  }
};

__device__ __forceinline__ int day_cl(const int32_t* day_cluster, int32_t cluster, int d) {
  return day_cluster ? day_cluster[d] : cluster;
}

// Fixed-order block sum of one double per thread (blockDim.x == kRedBlock).
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

// Row (h, a) of rho_c applied to q_d:  sum_l sum_{p in row a} W[l][h-l][a,p] q[h-l][p].
// The row's entries are taken in CSR order from the link-sliced layout, where
// they come in pairs: one load brings two values (and one their two ODs), and
// the loads of four entries are issued together (the sums keep their order).
template <int ST, typename S>
__device__ __forceinline__ S row_dot(const DevPat& pt, const DevVals& v, int c, int h, int a,
                                     const S* q, int64_t q_t, int64_t q_b) {
  S acc = 0;
  const int32_t deg = pt.row_ptr[a + 1] - pt.row_ptr[a];
  const int32_t s0 = pt.sr_first[a];
  for (int l = 0; l < pt.K; ++l) {
    const int t = h - l;
    if (t < 0) break;
    if (t >= pt.T) continue;
    const int64_t base = c * v.cstride_r + ((int64_t)l * pt.T + t) * pt.sr_len;
    const int64_t sbase = (c * (int64_t)pt.K * pt.T + (int64_t)l * pt.T + t) * v.n_ptile;
    const S* qt = q + (int64_t)t * q_t;
    int32_t k = 0;
    for (; k + 4 <= deg; k += 4) {
      const int32_t slot = s0 + 64 * k;   // entries k, k+1; k+2, k+3 one pair further
      const int2 p01 = *reinterpret_cast<const int2*>(pt.sr_col + slot);
      const int2 p23 = *reinterpret_cast<const int2*>(pt.sr_col + slot + 128);
      S w0, w1, w2, w3;
      Load2<ST>::get(v.W, base + slot, v.scale, sbase + (p01.x >> 6), sbase + (p01.y >> 6), w0, w1);
      Load2<ST>::get(v.W, base + slot + 128, v.scale, sbase + (p23.x >> 6), sbase + (p23.y >> 6), w2,
                     w3);
      const S x0 = qt[col_at(p01.x, q_b)], x1 = qt[col_at(p01.y, q_b)];
      const S x2 = qt[col_at(p23.x, q_b)], x3 = qt[col_at(p23.y, q_b)];
      acc += w0 * x0;
      acc += w1 * x1;
      acc += w2 * x2;
      acc += w3 * x3;
    }
    if (k + 2 <= deg) {
      const int32_t slot = s0 + 64 * k;
      const int2 p01 = *reinterpret_cast<const int2*>(pt.sr_col + slot);
      S w0, w1;
      Load2<ST>::get(v.W, base + slot, v.scale, sbase + (p01.x >> 6), sbase + (p01.y >> 6), w0, w1);
      const S x0 = qt[col_at(p01.x, q_b)], x1 = qt[col_at(p01.y, q_b)];
      acc += w0 * x0;
      acc += w1 * x1;
      k += 2;
    }
    if (k < deg) {
      const int32_t slot = s0 + 64 * k;
      const int p = pt.sr_col[slot];
      acc += static_cast<S>(Load<ST>::get(v.W, base + slot, v.scale, sbase + (p >> 6))) *
             qt[col_at(p, q_b)];
    }
  }
  return acc;
}

// Column (t, p) of rho_c^T applied to residual rows: sum over lags l whose row
// block h = t+l is in the minibatch (slot pos[h]-first in [0, bh)) of sum_{a on p} W[l][t][a,p] r[slot][a].
// The column's entries are taken in CSC order from the OD-sliced layout, four
// steps' loads issued together.
template <int ST, typename S>
__device__ __forceinline__ S col_dot_chunk(const DevPat& pt, const DevVals& v, int c, int t, int p,
                                           const int32_t* pos_c, int32_t first, int32_t bh,
                                           const S* Rd, int64_t r_s, int64_t r_b) {
  S acc = 0;
  const int32_t deg = pt.col_ptr[p + 1] - pt.col_ptr[p];
  const int32_t s0 = pt.sc_off[p >> 6] + (p & 63);
  for (int l = 0; l < pt.K; ++l) {
    const int h = t + l;
    if (h >= pt.H) break;
    const int s = pos_c ? pos_c[h] - first : h;
    if (s < 0 || s >= bh) continue;
    const int64_t base = c * v.cstride_c + ((int64_t)l * pt.T + t) * pt.sc_len;
    const int64_t si = (c * (int64_t)pt.K * pt.T + (int64_t)l * pt.T + t) * v.n_ptile + (p >> 6);
    const S* r = Rd + (int64_t)s * r_s;
    int32_t k = 0;
    for (; k + 4 <= deg; k += 4) {
      S w[4], x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t slot = s0 + 64 * (k + u);
        w[u] = static_cast<S>(Load<ST>::get(v.WT, base + slot, v.scale, si));
        x[u] = r[col_at(pt.sc_row[slot], r_b)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += w[u] * x[u];
    }
    for (; k < deg; ++k) {
      const int32_t slot = s0 + 64 * k;
      acc += static_cast<S>(Load<ST>::get(v.WT, base + slot, v.scale, si)) * r[col_at(pt.sc_row[slot], r_b)];
    }
  }
  return acc;
}

// ------------------------------------------------------------- kernels --
// With STAGE the block first copies the K demand rows its links read,
// Q_d[h-l] for l < K, into LDS (row l at l*P; rows outside the day are
// zeros that no lane reads), so the walk's demand gathers are LDS reads.
template <int ST, typename S, bool STAGE>
__global__ void __launch_bounds__(kRowsBlock)
k_chunk_resid(DevPat pt, DevVals v, const int32_t* day_cluster, int32_t cluster, ChunkSched cs,
              Layout ly, const S* __restrict__ Q, const S* __restrict__ X, S* __restrict__ R) {
  extern __shared__ unsigned char q_stage[];
  const int a = blockIdx.x * kRowsBlock + threadIdx.x;
  const int s = blockIdx.y, d = blockIdx.z;
  cs = resolve_epoch(cs);
  const int c = day_cl(day_cluster, cluster, d);
  if (cs.j0 + s >= pt.H) return;   // the whole block
  const int h = cs.perm[c * pt.H + cs.j0 + s];
  S xhat;
  if constexpr (STAGE) {
    S* qs = reinterpret_cast<S*>(q_stage);
    const S* qd = Q + d * ly.q_d;
    for (int i = threadIdx.x; i < pt.K * pt.P; i += kRowsBlock) {
      const int l = i / pt.P, p = i % pt.P, t = h - l;
      qs[i] = (t >= 0 && t < pt.T) ? qd[(int64_t)t * ly.q_t + col_at(p, ly.q_b)] : S(0);
    }
    __syncthreads();
    if (a >= pt.L) return;
    // row t = h - l of the staged copy sits at (h - t) * P: base h*P, stride -P
    xhat = row_dot<ST, S>(pt, v, c, h, a, qs + (int64_t)h * pt.P, -(int64_t)pt.P, 4);
  } else {
    if (a >= pt.L) return;
    xhat = row_dot<ST, S>(pt, v, c, h, a, Q + d * ly.q_d, ly.q_t, ly.q_b);
  }
  R[d * ly.r_d + s * ly.r_s + col_at(a, ly.r_b)] = xhat - X[d * ly.x_d + h * ly.x_h + col_at(a, ly.x_b)];
}

template <int ST, typename S>
__global__ void __launch_bounds__(kColsBlock)
k_chunk_adj_step(DevPat pt, DevVals v, const int32_t* day_cluster, int32_t cluster, ChunkSched cs,
                 Layout ly, const S* __restrict__ R, S* __restrict__ Q, S* __restrict__ A,
                 StepArgs st) {
  const int p = blockIdx.x * kColsBlock + threadIdx.x;
  const int i = blockIdx.y, d = blockIdx.z;
  if (p >= pt.P) return;
  cs = resolve_epoch(cs);
  const int c = day_cl(day_cluster, cluster, d);
  const int t = cs.touched[((int64_t)c * cs.max_touched + i) * desc_width(pt.K) + kDescT];
  if (t < 0) return;
  const S g = col_dot_chunk<ST, S>(pt, v, c, t, p, cs.pos + (int64_t)c * pt.H, cs.j0, cs.bh,
                                   R + d * ly.r_d, ly.r_s, ly.r_b);
  const int64_t idx = d * ly.q_d + t * ly.q_t + col_at(p, ly.q_b);
  S q = Q[idx];
  if (st.optimizer == 0) {
    const S acc = A[idx] + g * g;
    A[idx] = acc;
    q -= static_cast<S>(st.eta) * g / (sqrt(acc) + static_cast<S>(st.eps));
  } else {
    q -= static_cast<S>(st.eta) * g;
  }
  Q[idx] = q > S(0) ? q : S(0);
}

template <int ST, typename S>
__global__ void __launch_bounds__(kRedBlock)
k_apply_rows(DevPat pt, DevVals v, const int32_t* day_cluster, int32_t cluster, Layout ly,
             const S* __restrict__ Q, const S* __restrict__ X, S* __restrict__ out,
             double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const int h = blockIdx.x, d = blockIdx.y;
  const int c = day_cl(day_cluster, cluster, d);
  const S* q = Q + d * ly.q_d;
  double ss = 0.0;
  for (int a = threadIdx.x; a < pt.L; a += kRedBlock) {
    S val = row_dot<ST, S>(pt, v, c, h, a, q, ly.q_t, ly.q_b);
    const int64_t o = d * ly.x_d + h * ly.x_h + col_at(a, ly.x_b);
    if (X) val -= X[o];
    if (out) out[o] = val;
    ss += static_cast<double>(val) * static_cast<double>(val);
  }
  if (part) {
    const double tot = block_sum(ss, sh);
    if (threadIdx.x == 0) part[(int64_t)d * pt.H + h] = tot;
  }
}

template <int ST, typename S>
__global__ void __launch_bounds__(kColsBlock)
k_adjoint_rows(DevPat pt, DevVals v, const int32_t* day_cluster, int32_t cluster, Layout ly,
               const S* __restrict__ R, S* __restrict__ G) {
  const int t = blockIdx.x, d = blockIdx.y;
  const int c = day_cl(day_cluster, cluster, d);
  const S* Rd = R + d * ly.r_d;
  for (int p = threadIdx.x; p < pt.P; p += kColsBlock)
    G[d * ly.q_d + t * ly.q_t + col_at(p, ly.q_b)] =
        col_dot_chunk<ST, S>(pt, v, c, t, p, nullptr, 0, pt.H, Rd, ly.r_s, ly.r_b);
}

__global__ void k_sum_partials(const double* __restrict__ part, int32_t n_per, int32_t n_days,
                               double* __restrict__ out) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_days) return;
  double s = 0.0;
  for (int i = 0; i < n_per; ++i) s += part[(int64_t)d * n_per + i];
  out[d] = s;
}

__global__ void k_max_partials(const double* __restrict__ part, int32_t n_per, int32_t n_days,
                               double* __restrict__ out) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_days) return;
  double m = 0.0;
  for (int i = 0; i < n_per; ++i) m = fmax(m, part[(int64_t)d * n_per + i]);
  out[d] = m;
}

template <typename S>
__global__ void __launch_bounds__(kRedBlock)
k_kkt_partials(const S* __restrict__ Q, const S* __restrict__ G, int32_t T, int32_t P,
               double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const int t = blockIdx.x, d = blockIdx.y;
  double m = 0.0;
  for (int p = threadIdx.x; p < P; p += kRedBlock) {
    const int64_t i = ((int64_t)d * T + t) * P + p;
    const double q = Q[i], g = G[i];
    m = fmax(m, fabs(q < g ? q : g));
  }
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) part[(int64_t)d * T + t] = r;
}

// First pass (sum_x == nullptr): per (d, h) sum of x.  Second pass: sum of (x - mean)^2.
template <typename S>
__global__ void __launch_bounds__(kRedBlock)
k_x_moment(const S* __restrict__ X, int32_t H, int32_t L, const double* __restrict__ sum_x,
           double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const int h = blockIdx.x, d = blockIdx.y;
  const double mean = sum_x ? sum_x[d] / (static_cast<double>(H) * L) : 0.0;
  double s = 0.0;
  for (int a = threadIdx.x; a < L; a += kRedBlock) {
    const double x = X[((int64_t)d * H + h) * L + a];
    s += sum_x ? (x - mean) * (x - mean) : x;
  }
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)d * H + h] = r;
}

__global__ void k_r2(const double* loss, const double* sst, int32_t n, double* r2) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d < n) r2[d] = 1.0 - loss[d] / sst[d];
}

template <typename S>
__global__ void k_check_finite(const S* __restrict__ X, int64_t n, int32_t* flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(X[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

template <typename S>
__global__ void k_clamp(S* __restrict__ Q, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    Q[i] = Q[i] > S(0) ? Q[i] : S(0);
}

template <typename S>
__global__ void __launch_bounds__(kRedBlock)
k_quantize(DevPat pt, int32_t storage, int32_t c, const S* __restrict__ Wsrc, void* W, void* WT,
           float* scale, const int32_t* __restrict__ csc2csr, int64_t cstride_r, int64_t cstride_c,
           int32_t n_ptile) {
  // one block per (l, t) block of cluster c; the source is in CSR order, the
  // two copies are written in their sliced layouts
  const int lt = blockIdx.x;
  const S* src = Wsrc + (int64_t)lt * pt.nnz;
  const int64_t dr = c * cstride_r + (int64_t)lt * pt.sr_len;
  const int64_t dc = c * cstride_c + (int64_t)lt * pt.sc_len;
  __shared__ float smax[64];
  if (storage == DODE_FP8_E4M3) {
    for (int i = threadIdx.x; i < n_ptile; i += blockDim.x) smax[i] = 0.f;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < pt.nnz; j += blockDim.x) {
      const float a = fabsf(static_cast<float>(src[j]));
      atomicMax(reinterpret_cast<unsigned int*>(&smax[pt.col[j] >> 6]), __float_as_uint(a));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_ptile; i += blockDim.x)
      scale[((int64_t)c * pt.K * pt.T + lt) * n_ptile + i] = smax[i] > 0.f ? smax[i] / 448.f : 1.f;
    __syncthreads();
  }
  for (int64_t jj = threadIdx.x; jj < pt.nnz; jj += blockDim.x) {
    const int64_t j = csc2csr[jj];
    const int64_t oj = dr + pt.sr_pos[j], ojj = dc + pt.sc_pos[jj];
    const float w = static_cast<float>(src[j]);
    if (storage == DODE_F32) {
      static_cast<float*>(W)[oj] = w;
      static_cast<float*>(WT)[ojj] = w;
    } else if (storage == DODE_BF16) {
      const uint16_t b = f32_to_bf16_rne(w);
      static_cast<uint16_t*>(W)[oj] = b;
      static_cast<uint16_t*>(WT)[ojj] = b;
    } else if (storage == DODE_FP8_E4M3) {
      const float sc = smax[pt.col[j] >> 6] > 0.f ? smax[pt.col[j] >> 6] / 448.f : 1.f;
      const uint8_t b = f32_to_e4m3_rne(w / sc);
      static_cast<uint8_t*>(W)[oj] = b;
      static_cast<uint8_t*>(WT)[ojj] = b;
    } else {
      static_cast<double*>(W)[oj] = static_cast<double>(src[j]);
      static_cast<double*>(WT)[ojj] = static_cast<double>(src[j]);
    }
  }
}

template <template <int, typename> class F, typename... Args>
hipError_t dispatch(const dode_dar* dar, Args&&... args) {
  switch (dar->storage) {
    case DODE_F64: return F<DODE_F64, double>::run(args...);
    case DODE_F32: return F<DODE_F32, float>::run(args...);
    case DODE_BF16: return F<DODE_BF16, float>::run(args...);
    case DODE_FP8_E4M3: return F<DODE_FP8_E4M3, float>::run(args...);
  }
  return hipErrorInvalidValue;
}

template <int ST, typename S>
struct RunResid {
  static hipError_t run(const dode_dar* dar, const int32_t* dc, int32_t cl, const ChunkSched& cs,
                        const Layout& ly, const void* Q, const void* X, void* R, int32_t n,
                        hipStream_t s) {
    dim3 grid((dar->dims.L + kRowsBlock - 1) / kRowsBlock, cs.bh, n);
    const size_t stage = (size_t)dar->dims.K * dar->dims.P * sizeof(S);
    if (stage <= kQStageBytes)
      hipLaunchKernelGGL((k_chunk_resid<ST, S, true>), grid, dim3(kRowsBlock), stage, s, dar->pat(),
                         dar->vals(), dc, cl, cs, ly, static_cast<const S*>(Q),
                         static_cast<const S*>(X), static_cast<S*>(R));
    else
      hipLaunchKernelGGL((k_chunk_resid<ST, S, false>), grid, dim3(kRowsBlock), 0, s, dar->pat(),
                         dar->vals(), dc, cl, cs, ly, static_cast<const S*>(Q),
                         static_cast<const S*>(X), static_cast<S*>(R));
    return hipGetLastError();
  }
};

template <int ST, typename S>
struct RunAdjStep {
  static hipError_t run(const dode_dar* dar, const int32_t* dc, int32_t cl, const ChunkSched& cs,
                        const Layout& ly, const void* R, void* Q, void* A, int32_t n,
                        const StepArgs& st, hipStream_t s) {
    dim3 grid((dar->dims.P + kColsBlock - 1) / kColsBlock, cs.max_touched, n);
    hipLaunchKernelGGL((k_chunk_adj_step<ST, S>), grid, dim3(kColsBlock), 0, s, dar->pat(),
                       dar->vals(), dc, cl, cs, ly, static_cast<const S*>(R), static_cast<S*>(Q),
                       static_cast<S*>(A), st);
    return hipGetLastError();
  }
};

template <int ST, typename S>
struct RunApplyRows {
  static hipError_t run(const dode_dar* dar, const int32_t* dc, int32_t cl, const Layout& ly,
                        const void* Q, const void* X, void* out, double* part, int32_t n,
                        hipStream_t s) {
    dim3 grid(dar->dims.H, n);
    hipLaunchKernelGGL((k_apply_rows<ST, S>), grid, dim3(kRedBlock), 0, s, dar->pat(), dar->vals(),
                       dc, cl, ly, static_cast<const S*>(Q), static_cast<const S*>(X),
                       static_cast<S*>(out), part);
    return hipGetLastError();
  }
};

template <int ST, typename S>
struct RunAdjRows {
  static hipError_t run(const dode_dar* dar, const int32_t* dc, int32_t cl, const Layout& ly,
                        const void* R, void* G, int32_t n, hipStream_t s) {
    dim3 grid(dar->dims.T, n);
    hipLaunchKernelGGL((k_adjoint_rows<ST, S>), grid, dim3(kColsBlock), 0, s, dar->pat(),
                       dar->vals(), dc, cl, ly, static_cast<const S*>(R), static_cast<S*>(G));
    return hipGetLastError();
  }
};

}  // namespace

hipError_t plain_chunk_resid(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                             const ChunkSched& cs, const Layout& ly, const void* Q, const void* X,
                             void* R, int32_t n_days, hipStream_t s) {
  return dispatch<RunResid>(dar, dar, day_cluster, cluster, cs, ly, Q, X, R, n_days, s);
}

hipError_t plain_chunk_adj_step(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                                const ChunkSched& cs, const Layout& ly, const void* R, void* Q,
                                void* A, int32_t n_days, const StepArgs& st, hipStream_t s) {
  return dispatch<RunAdjStep>(dar, dar, day_cluster, cluster, cs, ly, R, Q, A, n_days, st, s);
}

hipError_t plain_apply_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                            const Layout& ly, const void* Q, const void* X, void* out, double* part,
                            int32_t n_days, hipStream_t s) {
  return dispatch<RunApplyRows>(dar, dar, day_cluster, cluster, ly, Q, X, out, part, n_days, s);
}

hipError_t plain_adjoint_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                              const Layout& ly, const void* R, void* G, int32_t n_days,
                              hipStream_t s) {
  return dispatch<RunAdjRows>(dar, dar, day_cluster, cluster, ly, R, G, n_days, s);
}

namespace {

// dst[r][i][k] = src[order[i]][r][k]; block (i, r), threads over k.
template <typename S>
__global__ void k_gather(const S* __restrict__ src, S* __restrict__ dst, const int32_t* order,
                         int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb, int clamp) {
  const int i = blockIdx.x, r = blockIdx.y;
  const S* a = src + ((int64_t)order[i] * rows + r) * n;
  S* b = dst + (int64_t)i * sd + (int64_t)r * sr;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const S v = a[k];
    b[col_at(k, sb)] = clamp ? (v > S(0) ? v : S(0)) : v;
  }
}

template <typename S>
__global__ void k_scatter(const S* __restrict__ src, S* __restrict__ dst, const int32_t* order,
                          int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb) {
  const int i = blockIdx.x, r = blockIdx.y;
  const S* a = src + (int64_t)i * sd + (int64_t)r * sr;
  S* b = dst + ((int64_t)order[i] * rows + r) * n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) b[k] = a[col_at(k, sb)];
}

template <typename S>
__global__ void k_zero(S* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = S(0);
}

__global__ void k_set_counter(int32_t* c, int32_t v) { *c = v; }
__global__ void k_bump_counter(int32_t* c) { *c += 1; }

__global__ void k_permute_loss(const double* __restrict__ src, const int32_t* __restrict__ order,
                               int32_t D, double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D) dst[order[i]] = src[i];
}

}  // namespace

hipError_t gather_rows(bool f64, const void* src, void* dst, const int32_t* order, int32_t D,
                       int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb, bool clamp,
                       hipStream_t s) {
  const dim3 grid(D, rows);
  if (f64)
    hipLaunchKernelGGL(k_gather<double>, grid, dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<double*>(dst), order, rows, n, sd, sr, sb, (int)clamp);
  else
    hipLaunchKernelGGL(k_gather<float>, grid, dim3(256), 0, s, static_cast<const float*>(src),
                       static_cast<float*>(dst), order, rows, n, sd, sr, sb, (int)clamp);
  return hipGetLastError();
}

hipError_t scatter_rows(bool f64, const void* src, void* dst, const int32_t* order, int32_t D,
                        int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb, hipStream_t s) {
  const dim3 grid(D, rows);
  if (f64)
    hipLaunchKernelGGL(k_scatter<double>, grid, dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<double*>(dst), order, rows, n, sd, sr, sb);
  else
    hipLaunchKernelGGL(k_scatter<float>, grid, dim3(256), 0, s, static_cast<const float*>(src),
                       static_cast<float*>(dst), order, rows, n, sd, sr, sb);
  return hipGetLastError();
}

hipError_t fill_zero(bool f64, void* x, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
  if (f64)
    hipLaunchKernelGGL(k_zero<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(x), n);
  else
    hipLaunchKernelGGL(k_zero<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(x), n);
  return hipGetLastError();
}

hipError_t set_counter(int32_t* c, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, c, v);
  return hipGetLastError();
}

hipError_t bump_counter(int32_t* c, hipStream_t s) {
  hipLaunchKernelGGL(k_bump_counter, dim3(1), dim3(1), 0, s, c);
  return hipGetLastError();
}

hipError_t permute_loss(const double* src, const int32_t* order, int32_t D, double* dst,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_permute_loss, dim3((D + 255) / 256), dim3(256), 0, s, src, order, D, dst);
  return hipGetLastError();
}

hipError_t sum_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3((n_days + 127) / 128), dim3(128), 0, s, part, n_per,
                     n_days, out);
  return hipGetLastError();
}

hipError_t max_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_max_partials, dim3((n_days + 127) / 128), dim3(128), 0, s, part, n_per,
                     n_days, out);
  return hipGetLastError();
}

hipError_t kkt_partials(bool f64, const void* Q, const void* G, int32_t T, int32_t P,
                        int32_t n_days, double* part, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(k_kkt_partials<double>, dim3(T, n_days), dim3(kRedBlock), 0, s,
                       static_cast<const double*>(Q), static_cast<const double*>(G), T, P, part);
  else
    hipLaunchKernelGGL(k_kkt_partials<float>, dim3(T, n_days), dim3(kRedBlock), 0, s,
                       static_cast<const float*>(Q), static_cast<const float*>(G), T, P, part);
  return hipGetLastError();
}

hipError_t x_moment_partials(bool f64, const void* X, int32_t H, int32_t L, int32_t n_days,
                             const double* sum_x, double* part, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(k_x_moment<double>, dim3(H, n_days), dim3(kRedBlock), 0, s,
                       static_cast<const double*>(X), H, L, sum_x, part);
  else
    hipLaunchKernelGGL(k_x_moment<float>, dim3(H, n_days), dim3(kRedBlock), 0, s,
                       static_cast<const float*>(X), H, L, sum_x, part);
  return hipGetLastError();
}

hipError_t r2_finish(const double* loss, const double* sst, int32_t n_days, double* r2,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_r2, dim3((n_days + 127) / 128), dim3(128), 0, s, loss, sst, n_days, r2);
  return hipGetLastError();
}

hipError_t check_finite(bool f64, const void* X, int64_t n, int32_t* flag, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256 > 0 ? (n + 255) / 256 : 1);
  if (f64)
    hipLaunchKernelGGL(k_check_finite<double>, dim3(blocks), dim3(256), 0, s,
                       static_cast<const double*>(X), n, flag);
  else
    hipLaunchKernelGGL(k_check_finite<float>, dim3(blocks), dim3(256), 0, s,
                       static_cast<const float*>(X), n, flag);
  return hipGetLastError();
}

hipError_t clamp_nonneg(bool f64, void* Q, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256 > 0 ? (n + 255) / 256 : 1);
  if (f64)
    hipLaunchKernelGGL(k_clamp<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(Q), n);
  else
    hipLaunchKernelGGL(k_clamp<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(Q), n);
  return hipGetLastError();
}

hipError_t quantize_values(const dode_dar* dar, int32_t cluster, const void* W_state,
                           hipStream_t s) {
  const dim3 grid(dar->dims.K * dar->dims.T);
  const int32_t n_ptile = (dar->dims.P + 63) / 64;
  if (dar->storage == DODE_F64)
    hipLaunchKernelGGL(k_quantize<double>, grid, dim3(kRedBlock), 0, s, dar->pat(),
                       (int32_t)dar->storage, cluster, static_cast<const double*>(W_state), dar->d_W,
                       dar->d_WT, dar->d_scale, dar->d_csc2csr, dar->vals().cstride_r,
                       dar->vals().cstride_c, n_ptile);
  else
    hipLaunchKernelGGL(k_quantize<float>, grid, dim3(kRedBlock), 0, s, dar->pat(),
                       (int32_t)dar->storage, cluster, static_cast<const float*>(W_state), dar->d_W,
                       dar->d_WT, dar->d_scale, dar->d_csc2csr, dar->vals().cstride_r,
                       dar->vals().cstride_c, n_ptile);
  return hipGetLastError();
}
