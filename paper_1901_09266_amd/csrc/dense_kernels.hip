// Algorithm 1 on a dense B [m][n] (section "Solution algorithm"), the
// workload of the efficiency experiment (section "Algorithm efficiency").
//
// A minibatch of rows o = perm[s0 .. s0+nr) takes three launches, all
// HBM-bound on B (each row of the minibatch is streamed twice):
//   k_dense_resid    one wave per minibatch row: r[s] = B[o_s] . q - y[o_s];
//                    lanes read 16-byte vectors across the row and the wave
//                    sums them with a butterfly reduction;
//   k_dense_colsum   split-K adjoint: block (column block, slice of kSliceRows
//                    rows) writes part[slice][j] = sum over its rows of
//                    B[o_s][j] r[s], four consecutive columns per lane, so a
//                    wave reads 1 KiB of one row per step; the block's four
//                    waves split the slice's rows and meet in LDS;
//   k_dense_update   one block per 16 columns: g = the slices' partial sums
//                    (FP64, 16 lane groups over the slices, added in a fixed
//                    order), then Adagrad (or a fixed step) and the
//                    projection q = max(q, 0).
// The epoch loss ||B q - y||^2 (optional) uses the residual kernel over all
// rows in natural order and a one-block FP64 sum in a fixed order.
// B may also be stored as bf16 (FP32 arithmetic and state): the *_bf16
// kernels read 16 bytes = 8 values per lane and load.
#include "dode_internal.h"

#include <algorithm>

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kSliceRows = 128;

template <typename S>
struct Vec;
template <>
struct Vec<float> {
  using T = float4;
  static constexpr int N = 4;
};
template <>
struct Vec<double> {
  using T = double2;
  static constexpr int N = 2;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// r[s] = B[row] . q - y[row] for rows[s], s < nr (rows == nullptr: row s).
// VEC: rows are 16-byte aligned and n is a multiple of the vector width.
template <typename S, bool VEC>
__global__ void __launch_bounds__(kBlock)
k_dense_resid(int32_t n, int32_t nr, const int32_t* __restrict__ rows, const S* __restrict__ B,
              const S* __restrict__ y, const S* __restrict__ q, S* __restrict__ r) {
  const int s = blockIdx.x * kWaves + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= nr) return;
  const int32_t i = rows ? rows[s] : s;
  const S* row = B + (int64_t)i * n;
  S acc = S(0);
  if (VEC) {
    using V = typename Vec<S>::T;
    constexpr int W = Vec<S>::N;
    const V* rv = reinterpret_cast<const V*>(row);
    const V* qv = reinterpret_cast<const V*>(q);
    const int nv = n / W;
    S a2 = S(0);
    int j = lane;
    for (; j + 64 < nv; j += 128) {   // two vectors in flight per lane
      const V b0 = rv[j], b1 = rv[j + 64], q0 = qv[j], q1 = qv[j + 64];
      if constexpr (W == 4) {
        acc += b0.x * q0.x + b0.y * q0.y + b0.z * q0.z + b0.w * q0.w;
        a2 += b1.x * q1.x + b1.y * q1.y + b1.z * q1.z + b1.w * q1.w;
      } else {
        acc += b0.x * q0.x + b0.y * q0.y;
        a2 += b1.x * q1.x + b1.y * q1.y;
      }
    }
    if (j < nv) {
      const V b0 = rv[j], q0 = qv[j];
      if constexpr (W == 4)
        acc += b0.x * q0.x + b0.y * q0.y + b0.z * q0.z + b0.w * q0.w;
      else
        acc += b0.x * q0.x + b0.y * q0.y;
    }
    acc += a2;
  } else {
    for (int j = lane; j < n; j += 64) acc += row[j] * q[j];
  }
  acc = wave_sum(acc);
  if (lane == 0) r[s] = acc - y[i];
}

// part[slice][j] = sum over the slice's rows s of B[rows[s]][j] r[s].  A block
// covers 64*W columns (W per lane) and a slice of kSliceRows rows: wave w
// takes rows w, w+4, ... of the slice (so the four waves stream neighbouring
// rows), and the four wave sums are added in wave order through LDS.
template <typename S, bool VEC>
__global__ void __launch_bounds__(kBlock)
k_dense_colsum(int32_t n, int32_t nr, const int32_t* __restrict__ rows, const S* __restrict__ B,
               const S* __restrict__ r, S* __restrict__ part) {
  constexpr int W = VEC ? Vec<S>::N : 1;
  __shared__ S sh[kWaves][64 * W];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * 64 * W;
  const int64_t j0 = c0 + (int64_t)lane * W;
  const int slice = blockIdx.y;
  const int s_begin = slice * kSliceRows, s_end = min(nr, s_begin + kSliceRows);
  S acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = S(0);
  if (j0 < n) {
    if (VEC) {
      using V = typename Vec<S>::T;
#pragma unroll 4
      for (int s = s_begin + wave; s < s_end; s += kWaves) {
        const V b = *reinterpret_cast<const V*>(B + (int64_t)rows[s] * n + j0);
        const S rs = r[s];
        if constexpr (W == 4) {
          acc[0] += b.x * rs;
          acc[1] += b.y * rs;
          acc[2] += b.z * rs;
          acc[3] += b.w * rs;
        } else if constexpr (W == 2) {
          acc[0] += b.x * rs;
          acc[1] += b.y * rs;
        }
      }
    } else {
      for (int s = s_begin + wave; s < s_end; s += kWaves) acc[0] += B[(int64_t)rows[s] * n + j0] * r[s];
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) sh[wave][lane * W + w] = acc[w];
  __syncthreads();
  // thread t adds column t of the block (and t + 256 when the block is wider)
  for (int c = threadIdx.x; c < 64 * W; c += kBlock) {
    if (c0 + c >= n) break;
    S v = sh[0][c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) v += sh[w][c];
    part[(int64_t)slice * n + c0 + c] = v;
  }
}

// One block per 16 columns: lane group g = threadIdx.x / 16 (four per wave)
// adds slices g, g+16, ... of its column in FP64 (each group reads 64
// neighbouring bytes of a slice row), the 16 partial sums of a column are
// added in order of g through LDS, then Adagrad (or the fixed step) and the
// projection.
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_dense_update(int32_t n, int32_t n_slices, const S* __restrict__ part, S* __restrict__ q,
               S* __restrict__ A, StepArgs st) {
  constexpr int kCols = 16, kParts = kBlock / kCols;
  __shared__ double sh[kParts][kCols];
  const int c = threadIdx.x % kCols, g = threadIdx.x / kCols;
  const int64_t j = (int64_t)blockIdx.x * kCols + c;
  double gd = 0.0;
  if (j < n)
    for (int k = g; k < n_slices; k += kParts) gd += static_cast<double>(part[(int64_t)k * n + j]);
  sh[g][c] = gd;
  __syncthreads();
  if (threadIdx.x >= kCols || j >= n) return;
  gd = sh[0][c];
#pragma unroll
  for (int p = 1; p < kParts; ++p) gd += sh[p][c];
  const S g_j = static_cast<S>(gd);
  S v = q[j];
  if (st.optimizer == 0) {
    const S acc = A[j] + g_j * g_j;
    A[j] = acc;
    v -= static_cast<S>(st.eta) * g_j / (sqrt(acc) + static_cast<S>(st.eps));
  } else {
    v -= static_cast<S>(st.eta) * g_j;
  }
  q[j] = v > S(0) ? v : S(0);
}

// loss[e] = sum over rows of r^2 (FP64, fixed order: strided per thread, then a tree).
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_dense_sq_sum(int32_t m, const S* __restrict__ r, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += kBlock) s += static_cast<double>(r[i]) * r[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// ---- B stored as bf16 (FP32 arithmetic and state) -------------------------
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ float dot8(const uint4 b, const float4 q0, const float4 q1) {
  return bf16_lo(b.x) * q0.x + bf16_hi(b.x) * q0.y + bf16_lo(b.y) * q0.z + bf16_hi(b.y) * q0.w +
         bf16_lo(b.z) * q1.x + bf16_hi(b.z) * q1.y + bf16_lo(b.w) * q1.z + bf16_hi(b.w) * q1.w;
}

// r[s] = B[row] . q - y[row]; VEC: 16-byte rows (8 values per load)
template <bool VEC>
__global__ void __launch_bounds__(kBlock)
k_dense_resid_bf16(int32_t n, int32_t nr, const int32_t* __restrict__ rows,
                   const uint16_t* __restrict__ B, const float* __restrict__ y,
                   const float* __restrict__ q, float* __restrict__ r) {
  const int s = blockIdx.x * kWaves + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= nr) return;
  const int32_t i = rows ? rows[s] : s;
  const uint16_t* row = B + (int64_t)i * n;
  float acc = 0.f;
  if (VEC) {
    const uint4* rv = reinterpret_cast<const uint4*>(row);
    const float4* qv = reinterpret_cast<const float4*>(q);
    const int nv = n / 8;
    float a2 = 0.f;
    int j = lane;
    for (; j + 64 < nv; j += 128) {   // two 16-byte loads in flight per lane
      const uint4 b0 = rv[j], b1 = rv[j + 64];
      acc += dot8(b0, qv[2 * j], qv[2 * j + 1]);
      a2 += dot8(b1, qv[2 * (j + 64)], qv[2 * (j + 64) + 1]);
    }
    if (j < nv) acc += dot8(rv[j], qv[2 * j], qv[2 * j + 1]);
    acc += a2;
  } else {
    for (int j = lane; j < n; j += 64) acc += __uint_as_float((uint32_t)row[j] << 16) * q[j];
  }
  acc = wave_sum(acc);
  if (lane == 0) r[s] = acc - y[i];
}

// part[slice][j] = sum over the slice's rows of B[rows[s]][j] r[s]; a lane
// covers 8 columns (one 16-byte load) in VEC mode, else 1.
template <bool VEC>
__global__ void __launch_bounds__(kBlock)
k_dense_colsum_bf16(int32_t n, int32_t nr, const int32_t* __restrict__ rows,
                    const uint16_t* __restrict__ B, const float* __restrict__ r,
                    float* __restrict__ part) {
  constexpr int W = VEC ? 8 : 1;
  __shared__ float sh[kWaves][64 * W];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * 64 * W;
  const int64_t j0 = c0 + (int64_t)lane * W;
  const int slice = blockIdx.y;
  const int s_begin = slice * kSliceRows, s_end = min(nr, s_begin + kSliceRows);
  float acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0.f;
  if (j0 < n) {
    if (VEC) {
#pragma unroll 4
      for (int s = s_begin + wave; s < s_end; s += kWaves) {
        const uint4 b = *reinterpret_cast<const uint4*>(B + (int64_t)rows[s] * n + j0);
        const float rs = r[s];
        acc[0] += bf16_lo(b.x) * rs;
        acc[1] += bf16_hi(b.x) * rs;
        acc[2] += bf16_lo(b.y) * rs;
        acc[3] += bf16_hi(b.y) * rs;
        acc[4] += bf16_lo(b.z) * rs;
        acc[5] += bf16_hi(b.z) * rs;
        acc[6] += bf16_lo(b.w) * rs;
        acc[7] += bf16_hi(b.w) * rs;
      }
    } else {
      for (int s = s_begin + wave; s < s_end; s += kWaves)
        acc[0] += __uint_as_float((uint32_t)B[(int64_t)rows[s] * n + j0] << 16) * r[s];
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) sh[wave][lane * W + w] = acc[w];
  __syncthreads();
  for (int c = threadIdx.x; c < 64 * W; c += kBlock) {
    if (c0 + c >= n) break;
    float v = sh[0][c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) v += sh[w][c];
    part[(int64_t)slice * n + c0 + c] = v;
  }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <typename S, bool VEC>
hipError_t run(const DenseArgs& a, hipStream_t s) {
  const S* B = static_cast<const S*>(a.B);
  const S* y = static_cast<const S*>(a.y);
  S* q = static_cast<S*>(a.q);
  S* A = static_cast<S*>(a.A);
  S* r = static_cast<S*>(a.r);
  S* part = static_cast<S*>(a.part);
  constexpr int W = VEC ? Vec<S>::N : 1;
  const unsigned col_blocks = blocks_for(a.n, 64 * W);
  for (int32_t e = 0; e < a.E; ++e) {
    for (int32_t s0 = 0; s0 < a.m; s0 += a.chunk) {
      const int32_t nr = std::min(a.chunk, a.m - s0);
      const int32_t* rows = a.perms + (int64_t)e * a.m + s0;
      const int32_t n_slices = (nr + kSliceRows - 1) / kSliceRows;
      hipLaunchKernelGGL((k_dense_resid<S, VEC>), dim3(blocks_for(nr, kWaves)), dim3(kBlock), 0, s,
                         a.n, nr, rows, B, y, q, r);
      hipLaunchKernelGGL((k_dense_colsum<S, VEC>), dim3(col_blocks, n_slices), dim3(kBlock), 0, s,
                         a.n, nr, rows, B, r, part);
      hipLaunchKernelGGL(k_dense_update<S>, dim3(blocks_for(a.n, 16)), dim3(kBlock), 0, s, a.n,
                         n_slices, part, q, A, a.st);
    }
    if (a.loss) {
      hipLaunchKernelGGL((k_dense_resid<S, VEC>), dim3(blocks_for(a.m, kWaves)), dim3(kBlock), 0, s,
                         a.n, a.m, (const int32_t*)nullptr, B, y, q, r);
      hipLaunchKernelGGL(k_dense_sq_sum<S>, dim3(1), dim3(kBlock), 0, s, a.m, r, a.loss + e);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <bool VEC>
hipError_t run_bf16(const DenseArgs& a, hipStream_t s) {
  const uint16_t* B = static_cast<const uint16_t*>(a.B);
  const float* y = static_cast<const float*>(a.y);
  float* q = static_cast<float*>(a.q);
  float* A = static_cast<float*>(a.A);
  float* r = static_cast<float*>(a.r);
  float* part = static_cast<float*>(a.part);
  constexpr int W = VEC ? 8 : 1;
  const unsigned col_blocks = blocks_for(a.n, 64 * W);
  for (int32_t e = 0; e < a.E; ++e) {
    for (int32_t s0 = 0; s0 < a.m; s0 += a.chunk) {
      const int32_t nr = std::min(a.chunk, a.m - s0);
      const int32_t* rows = a.perms + (int64_t)e * a.m + s0;
      const int32_t n_slices = (nr + kSliceRows - 1) / kSliceRows;
      hipLaunchKernelGGL(k_dense_resid_bf16<VEC>, dim3(blocks_for(nr, kWaves)), dim3(kBlock), 0, s,
                         a.n, nr, rows, B, y, q, r);
      hipLaunchKernelGGL(k_dense_colsum_bf16<VEC>, dim3(col_blocks, n_slices), dim3(kBlock), 0, s,
                         a.n, nr, rows, B, r, part);
      hipLaunchKernelGGL(k_dense_update<float>, dim3(blocks_for(a.n, 16)), dim3(kBlock), 0, s, a.n,
                         n_slices, part, q, A, a.st);
    }
    if (a.loss) {
      hipLaunchKernelGGL(k_dense_resid_bf16<VEC>, dim3(blocks_for(a.m, kWaves)), dim3(kBlock), 0, s,
                         a.n, a.m, (const int32_t*)nullptr, B, y, q, r);
      hipLaunchKernelGGL(k_dense_sq_sum<float>, dim3(1), dim3(kBlock), 0, s, a.m, r, a.loss + e);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

int32_t dense_slice_rows() { return kSliceRows; }

hipError_t dense_spgd_bf16(const DenseArgs& a, bool vec, hipStream_t s) {
  return vec ? run_bf16<true>(a, s) : run_bf16<false>(a, s);
}

hipError_t dense_spgd(const DenseArgs& a, bool f64, bool vec, hipStream_t s) {
  if (f64) return vec ? run<double, true>(a, s) : run<double, false>(a, s);
  return vec ? run<float, true>(a, s) : run<float, false>(a, s);
}
