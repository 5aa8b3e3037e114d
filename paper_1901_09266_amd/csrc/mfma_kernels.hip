// Matrix-core kernels of one SPGD minibatch (Algorithm 1) for BF16 storage.
//
// The day batch is the MFMA N dimension: a wave owns 16 rows of the output
// (16 links in the forward product, 16 ODs in the adjoint) for a group of up
// to 32 days of one cluster (two 16-column tiles), and walks the packed 16x32
// k-steps of the assignment blocks it needs with v_mfma_f32_16x16x32_bf16.
//
// Precision: the assignment values are bfloat16; the FP32 operand (demand in
// the forward product, residual in the adjoint) is split into a bfloat16 head
// and tail, x = hi + lo, and both halves are multiplied (two MFMAs per k-step),
// so the products keep ~16 significant bits of the FP32 operand; accumulation
// is FP32.  The Adagrad step, the projection and the residual are FP32.
//
// Layouts (caller-owned, day-major): Q, A [D][T][P]; X [D][H][L]; the residual
// scratch R [D][bh][L] holds the rows of the current minibatch.
#include "dode_internal.h"

namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// hi = bf16(v), lo = bf16(v - hi), packed 8 values per operand register set.
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t h = bf16_rne_bits(v[e]);
    const float hf = __uint_as_float(h << 16);
    hi[e] = static_cast<short>(h);
    lo[e] = static_cast<short>(bf16_rne_bits(v[e] - hf));
  }
}

// 8 consecutive entries [k0, k0+8) of row `row` of a day-major [D][rows][n] array,
// zero outside [0, n) or for an absent day (d < 0).
__device__ __forceinline__ void load8(const float* __restrict__ base, int d, int64_t row_stride_d,
                                      int row, int n, int k0, float (&v)[8]) {
  if (d < 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = 0.f;
    return;
  }
  const float* p = base + (int64_t)d * row_stride_d + (int64_t)row * n;
  if (k0 + 8 <= n) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = p[k0 + e];
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (k0 + e < n) ? p[k0 + e] : 0.f;
  }
}

__device__ __forceinline__ void mma2(const bf16x8& a, const float (&v)[8], f32x4& acc) {
  bf16x8 hi, lo;
  split8(v, hi, lo);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, acc, 0, 0, 0);
}

// Forward product and residual of the minibatch rows:
//   R[d][s][a] = sum_l rho_c[l][h-l][a, :] . Q_d[h-l][:] - X_d[h][a],  h = perm[j0+s].
// grid (ceil(nLT/4), bh, n_groups), 4 waves per block, wave = link tile.
__global__ void __launch_bounds__(256)
k_fwd_bf16(DevPat pt, DevTiles tl, ChunkSched cs, DayGroups dg, const float* __restrict__ Q,
           const float* __restrict__ X, float* __restrict__ R) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  const int s = blockIdx.y, g = blockIdx.z;
  if (i >= tl.nLT || cs.j0 + s >= pt.H) return;
  const int c = dg.cluster[g];
  const int h = cs.perm[c * pt.H + cs.j0 + s];
  const int n = lane & 15, kg = lane >> 4;
  const int first = dg.first[g], cnt = dg.count[g];
  const int d0 = n < cnt ? dg.days[first + n] : -1;
  const int d1 = 16 + n < cnt ? dg.days[first + 16 + n] : -1;
  const int nks = tl.f_ks[i], plo = tl.f_plo[i];
  const int64_t qstride = (int64_t)pt.T * pt.P;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const bf16x8* Fv = static_cast<const bf16x8*>(tl.Fv);
  for (int l = 0; l < pt.K; ++l) {
    const int t = h - l;
    if (t < 0) break;
    if (t >= pt.T) continue;
    const bf16x8* Ab = Fv + ((((int64_t)c * pt.K + l) * pt.T + t) * tl.kf_total + tl.f_koff[i]) * 64;
    for (int ks = 0; ks < nks; ++ks) {
      const bf16x8 a = Ab[ks * 64 + lane];
      const int p0 = plo + 32 * ks + 8 * kg;
      float v0[8], v1[8];
      load8(Q, d0, qstride, t, pt.P, p0, v0);
      load8(Q, d1, qstride, t, pt.P, p0, v1);
      mma2(a, v0, acc0);
      mma2(a, v1, acc1);
    }
  }
  const int a0 = 16 * i + 4 * kg;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = a0 + r;
    if (a >= pt.L) break;
    if (d0 >= 0)
      R[((int64_t)d0 * cs.bh + s) * pt.L + a] = acc0[r] - X[((int64_t)d0 * pt.H + h) * pt.L + a];
    if (d1 >= 0)
      R[((int64_t)d1 * cs.bh + s) * pt.L + a] = acc1[r] - X[((int64_t)d1 * pt.H + h) * pt.L + a];
  }
}

__device__ __forceinline__ void adagrad_update(float* __restrict__ Q, float* __restrict__ A,
                                               int64_t idx, float g, const StepArgs& st) {
  float q = Q[idx];
  if (st.optimizer == 0) {
    const float acc = A[idx] + g * g;
    A[idx] = acc;
    q -= static_cast<float>(st.eta) * g / (sqrtf(acc) + static_cast<float>(st.eps));
  } else {
    q -= static_cast<float>(st.eta) * g;
  }
  Q[idx] = q > 0.f ? q : 0.f;
}

// Adjoint of the minibatch and the fused Adagrad step + projection:
//   g_d[t][p] = sum_{l: t+l in minibatch} rho_c[l][t][:, p] . R_d[slot(t+l)][:]
// grid (ceil(nPT/4), max_touched, n_groups), wave = OD tile.
__global__ void __launch_bounds__(256)
k_adj_bf16(DevPat pt, DevTiles tl, ChunkSched cs, DayGroups dg, const float* __restrict__ R,
           float* __restrict__ Q, float* __restrict__ A, StepArgs st) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + wave;
  const int g = blockIdx.z;
  if (j >= tl.nPT) return;
  const int c = dg.cluster[g];
  const int t = cs.touched[c * cs.max_touched + blockIdx.y];
  if (t < 0) return;
  const int n = lane & 15, kg = lane >> 4;
  const int first = dg.first[g], cnt = dg.count[g];
  const int d0 = n < cnt ? dg.days[first + n] : -1;
  const int d1 = 16 + n < cnt ? dg.days[first + 16 + n] : -1;
  const int nks = tl.g_ks[j], alo = tl.g_alo[j];
  const int64_t rstride = (int64_t)cs.bh * pt.L;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const bf16x8* Gv = static_cast<const bf16x8*>(tl.Gv);
  const int32_t* pos = cs.pos + (int64_t)c * pt.H;
  for (int l = 0; l < pt.K; ++l) {
    const int h = t + l;
    if (h >= pt.H) break;
    const int s = pos[h] - cs.j0;
    if (s < 0 || s >= cs.bh) continue;
    const bf16x8* Ab = Gv + ((((int64_t)c * pt.K + l) * pt.T + t) * tl.kg_total + tl.g_koff[j]) * 64;
    for (int ks = 0; ks < nks; ++ks) {
      const bf16x8 a = Ab[ks * 64 + lane];
      const int k0 = alo + 32 * ks + 8 * kg;
      float v0[8], v1[8];
      load8(R, d0, rstride, s, pt.L, k0, v0);
      load8(R, d1, rstride, s, pt.L, k0, v1);
      mma2(a, v0, acc0);
      mma2(a, v1, acc1);
    }
  }
  const int p0 = 16 * j + 4 * kg;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = p0 + r;
    if (p >= pt.P) break;
    if (d0 >= 0) adagrad_update(Q, A, ((int64_t)d0 * pt.T + t) * pt.P + p, acc0[r], st);
    if (d1 >= 0) adagrad_update(Q, A, ((int64_t)d1 * pt.T + t) * pt.P + p, acc1[r], st);
  }
}

}  // namespace

hipError_t mfma_chunk_resid(const dode_dar* dar, const ChunkSched& cs, const DayGroups& dg,
                            const float* Q, const float* X, float* R, hipStream_t s) {
  const dim3 grid((dar->tiles.nLT + 3) / 4, cs.bh, dg.n);
  hipLaunchKernelGGL(k_fwd_bf16, grid, dim3(256), 0, s, dar->pat(), dar->tiles, cs, dg, Q, X, R);
  return hipGetLastError();
}

hipError_t mfma_chunk_adj_step(const dode_dar* dar, const ChunkSched& cs, const DayGroups& dg,
                               const float* R, float* Q, float* A, const StepArgs& st,
                               hipStream_t s) {
  const dim3 grid((dar->tiles.nPT + 3) / 4, cs.max_touched, dg.n);
  hipLaunchKernelGGL(k_adj_bf16, grid, dim3(256), 0, s, dar->pat(), dar->tiles, cs, dg, R, Q, A,
                     st);
  return hipGetLastError();
}
