// Matrix-core kernels of one SPGD minibatch (Algorithm 1) for BF16 and FP8
// storage.
//
// The day batch is the MFMA N dimension: a wave owns 16 rows of the output
// (16 links in the forward product, 16 ODs in the adjoint) for a group of up
// to 16*NT days of one cluster (NT 16-column tiles), and walks the packed
// 16x32 k-steps of the assignment blocks it needs with v_mfma_f32_16x16x32_bf16.
// Every day is its own MFMA column with the same summation order, so results
// do not depend on NT.
//
// Precision: the assignment values are bfloat16 (or OCP E4M3FN codes with one
// FP32 scale per (lag block, 64-OD group), widened exactly to bfloat16 in
// registers, the scale moved onto the other operand); the FP32 operand (demand in
// the forward product, residual in the adjoint) is split into a bfloat16 head
// and tail, x = hi + lo (both rounded to nearest even by v_cvt_pk_bf16_f32),
// and both halves are multiplied (two MFMAs per k-step), so the products keep
// ~16 significant bits of the FP32 operand; accumulation is FP32.  The
// Adagrad step, the projection and the residual are FP32.
//
// Layouts: the plan's day-blocked copies of Q, A (rows t), X (rows h) and the
// residual rows of the current minibatch R (rows = slots): entry (day d, row
// r, col k) at d*4 + r*row_stride + (k/4)*4D + k%4 (strides in Layout).
#include "dode_internal.h"

// No fused multiply-add contraction in this file: the FP8 scale product feeds
// the hi/lo split, and a contraction chosen differently per template
// instantiation would make the result depend on the day tile.
#pragma clang fp contract(off)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// four floats at a 4-byte-aligned address (one global_load_dwordx4 on gfx950)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int kXcds = 8;   // gfx950: workgroups are dealt to 8 XCDs round-robin

// Logical block of physical block b: each XCD gets one contiguous range of
// logical blocks, so blocks that share operands run under the same L2.
__device__ __forceinline__ int xcd_logical_block(int nblk) {
  const int b = blockIdx.x;
  const int per = (nblk + kXcds - 1) / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

// Operand loads are always full vectors over the day-blocked plan layout
// ([row][col/4][day][4], Layout): 4 consecutive columns of one day are 16
// contiguous bytes, and the 16 days of a column tile follow each other.  Where
// a tile's columns run past the last one the loads meet the zero blocks that
// end every row; the assignment entries there are zero as well.  Only stores
// are cut at the row end.
// B operand of one lane: k-step columns 4g..4g+3 and 16+4g..16+4g+3 of its
// day (p points at column 4g; the second half is 4 blocks further), matching
// the packed tile order.
__device__ __forceinline__ f32x8 load8(const float* __restrict__ p, int64_t sb) {
  const f32x4u a = *reinterpret_cast<const f32x4u*>(p);
  const f32x4u b = *reinterpret_cast<const f32x4u*>(p + 4 * sb);
  return f32x8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

__device__ __forceinline__ f32x4 load4(const float* __restrict__ p) {
  const f32x4u v = *reinterpret_cast<const f32x4u*>(p);
  return f32x4{v[0], v[1], v[2], v[3]};
}

// Value modes of the assignment operand.
//   kBF16     bfloat16 tiles.
//   kFP8      E4M3FN codes widened exactly to bf16; the FP8 scale is applied by
//             the caller to the other operand.
//   kFP8Corr  the corrected FP8 values h + c of refinement steps: h =
//             bf16(fp32(scale * e4m3)) is formed in registers, c comes from the
//             bf16 correction tiles; the other operand is not scaled.
enum { kBF16 = 0, kFP8 = 1, kFP8Corr = 2 };

typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x8 fp8_codes(const void* tiles, int64_t kidx, int lane) {
  const uint2 w = static_cast<const uint2*>(tiles)[kidx * 64 + lane];
  const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.x, false);
  const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.x, true);
  const f32x2 c = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.y, false);
  const f32x2 d = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.y, true);
  return f32x8{a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
}

// A operand of k-step `kidx` (element offset kidx*512 of the packed tiles):
// 8 values per lane (kBF16, kFP8; see the modes above).
template <int MODE>
__device__ __forceinline__ bf16x8 load_a(const void* tiles, int64_t kidx, int lane) {
  if constexpr (MODE == kBF16) {
    return static_cast<const bf16x8*>(tiles)[kidx * 64 + lane];
  } else {
    return __builtin_convertvector(fp8_codes(tiles, kidx, lane), bf16x8);
  }
}

// h = bf16(fp32(scale * e4m3)) of the lane's 8 codes, elements 0-3 with s0 and
// 4-7 with s1 (kFP8Corr).
__device__ __forceinline__ bf16x8 load_a_scaled(const void* tiles, int64_t kidx, int lane,
                                                float s0, float s1) {
  f32x8 v = fp8_codes(tiles, kidx, lane);
  v[0] *= s0; v[1] *= s0; v[2] *= s0; v[3] *= s0;
  v[4] *= s1; v[5] *= s1; v[6] *= s1; v[7] *= s1;
  return __builtin_convertvector(v, bf16x8);
}

__device__ __forceinline__ bf16x8 load_corr(const void* tiles, int64_t kidx, int lane) {
  return static_cast<const bf16x8*>(tiles)[kidx * 64 + lane];
}

// acc += a * (hi + lo) with hi = bf16(v), lo = bf16(v - hi).
__device__ __forceinline__ void mma_split(const bf16x8& a, const f32x8& v, f32x4& acc) {
  const bf16x8 hi = __builtin_convertvector(v, bf16x8);
  const bf16x8 lo = __builtin_convertvector(v - __builtin_convertvector(hi, f32x8), bf16x8);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, acc, 0, 0, 0);
}

// Four consecutive floats, or the first `valid` when the row ends earlier.
__device__ __forceinline__ void store4(float* __restrict__ p, const f32x4& v, bool full, int valid) {
  if (full) {
    *reinterpret_cast<f32x4u*>(p) = f32x4u{v[0], v[1], v[2], v[3]};
    return;
  }
  for (int k = 0; k < valid; ++k) p[k] = v[k];
}

// Forward product and residual of the minibatch rows:
//   R[d][s][a] = sum_l rho_c[l][h-l][a, :] . Q_d[h-l][:] - X_d[h][a],  h = perm[j0+s].
// A wave covers NT 16-day column tiles; its (lag, k-step) iterations run in
// batches of kBatch k-steps whose operand loads are all issued before the
// first product, so a batch costs one memory round trip.  Column n of tile u
// is day first+16u+n; past the group's end it reads day `first` and its
// result is dropped.
// One forward item (the one-launch-per-minibatch kernel): link tile i of
// minibatch slot s (interval h) for day group g of cluster c, written to the
// residual rows R[.][s].
template <int MODE, int NT>
__device__ __forceinline__ void fwd_item(const DevPat& pt, const DevTiles& tl, const Layout& ly,
                                         const WaveWork& w, int h, const float* __restrict__ Q,
                                         const float* __restrict__ X, float* __restrict__ R) {
  constexpr int kBatch = NT == 2 ? 3 : 8 / NT;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, kg = lane >> 4;
  const int c = w.c, s = w.row, i = w.tile;
  const int first = w.first, cnt = w.count;
  const int a0 = 16 * i + 4 * kg;
  bool live[NT];
  const float* qcol[NT];
  f32x4 x[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    live[u] = 16 * u + n < cnt;
    const int64_t du = live[u] ? first + 16 * u + n : first;
    qcol[u] = Q + du * ly.q_d;
    x[u] = load4(X + du * ly.x_d + h * ly.x_h + (a0 >> 2) * ly.x_b);   // observations first
  }
  // lags with t = h - l inside [0, T)
  const int l_lo = h - pt.T + 1 > 0 ? h - pt.T + 1 : 0;
  const int l_hi = h < pt.K - 1 ? h : pt.K - 1;
  const int nks = w.nks, plo = w.lo;
  const int n_it = l_hi >= l_lo ? (l_hi - l_lo + 1) * nks : 0;
  // k-step index of block (c, l, t): ((c*K + l)*T + t)*kf_total + f_koff[i] + ks
  const int64_t kbase = (int64_t)c * pt.K * pt.T * tl.kf_total + w.koff;
  f32x4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = __builtin_convertvector(f32x8{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, bf16x8);
  int l = l_lo, ks = 0;
  for (int it0 = 0; it0 < n_it; it0 += kBatch) {
    bf16x8 a[kBatch], ac[MODE == kFP8Corr ? kBatch : 1];
    f32x8 v[kBatch][NT];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int t = h - l;
      const int64_t kidx = kbase + ((int64_t)l * pt.T + t) * tl.kf_total + ks;
      const int p0 = plo + 32 * ks + 4 * kg;
#pragma unroll
      for (int u = 0; u < NT; ++u) v[b][u] = load8(qcol[u] + t * ly.q_t + (p0 >> 2) * ly.q_b, ly.q_b);
      if constexpr (MODE == kBF16) {
        a[b] = load_a<MODE>(tl.Fv, kidx, lane);
      } else {
        // each 4-OD half of the lane lies in one 64-OD scale group (p0 is a
        // multiple of 4); the two halves may fall in neighbouring groups
        const float* scl = tl.scale + (((int64_t)c * pt.K + l) * pt.T + t) * tl.n_ptile;
        const float s0 = scl[min(p0 >> 6, tl.n_ptile - 1)];
        const float s1 = scl[min((p0 + 16) >> 6, tl.n_ptile - 1)];
        if constexpr (MODE == kFP8) {
          a[b] = load_a<MODE>(tl.Fv, kidx, lane);
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            v[b][u][0] *= s0; v[b][u][1] *= s0; v[b][u][2] *= s0; v[b][u][3] *= s0;
            v[b][u][4] *= s1; v[b][u][5] *= s1; v[b][u][6] *= s1; v[b][u][7] *= s1;
          }
        } else {
          a[b] = load_a_scaled(tl.Fv, kidx, lane, s0, s1);
          ac[b] = load_corr(tl.Fc, kidx, lane);
        }
      }
      // past the last iteration: repeat its loads with a zero operand
      if (it0 + b >= n_it) {
        a[b] = zero;
        if constexpr (MODE == kFP8Corr) ac[b] = zero;
      } else if (it0 + b + 1 < n_it && ++ks == nks) {
        ks = 0;
        ++l;
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        mma_split(a[b], v[b][u], acc[u]);
        if constexpr (MODE == kFP8Corr) mma_split(ac[b], v[b][u], acc[u]);
      }
  }
  if (a0 >= pt.L) return;
  const bool full = a0 + 4 <= pt.L;
  const int valid = pt.L - a0;
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (live[u])
      store4(R + (int64_t)(first + 16 * u + n) * ly.r_d + s * ly.r_s + (a0 >> 2) * ly.r_b,
             acc[u] - x[u], full, valid);
}

// Forward product and residual for a group of TP link tiles i0..i0+TP-1
// (kFwdTileGroup) of one minibatch slot and day group: the tiles share their
// OD range, so each demand operand (and its head/tail split) is loaded once
// per k-step and multiplied with every tile of the group.  Per tile the
// products come in increasing lag and k-step order, as in fwd_item.  Tile
// i0+tt's k-steps follow tile i0's in the packed blocks (equal counts).
template <int MODE, int NT, int TP>
__device__ __forceinline__ void fwd_group(const DevPat& pt, const DevTiles& tl, const Layout& ly,
                                          const WaveWork& w, int h, const float* __restrict__ Q,
                                          const float* __restrict__ X, float* __restrict__ R) {
  constexpr int kBatch = NT == 2 ? 2 : 4 / NT;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, kg = lane >> 4;
  const int c = w.c, s = w.row, i0 = w.tile;
  const int first = w.first, cnt = w.count;
  const int n_tt = min(TP, tl.nLT - i0);   // tiles of this group (the last may be short)
  // The observed rows X are fetched after the product: the registers they
  // would hold across it cost occupancy (measured faster in every mode with
  // the benchmark schedules).
  bool live[NT];
  const float* qcol[NT];
  f32x4 x[TP][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    live[u] = 16 * u + n < cnt;
    const int64_t du = live[u] ? first + 16 * u + n : first;
    qcol[u] = Q + du * ly.q_d;
  }
  const int l_lo = h - pt.T + 1 > 0 ? h - pt.T + 1 : 0;
  const int l_hi = h < pt.K - 1 ? h : pt.K - 1;
  const int nks = w.nks, plo = w.lo;
  const int n_it = l_hi >= l_lo ? (l_hi - l_lo + 1) * nks : 0;
  const int64_t kbase = (int64_t)c * pt.K * pt.T * tl.kf_total + w.koff;
  f32x4 acc[TP][NT];
#pragma unroll
  for (int tt = 0; tt < TP; ++tt)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[tt][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = __builtin_convertvector(f32x8{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, bf16x8);
  int l = l_lo, ks = 0;
  for (int it0 = 0; it0 < n_it; it0 += kBatch) {
    bf16x8 a[kBatch][TP], ac[MODE == kFP8Corr ? kBatch : 1][TP];
    f32x8 v[kBatch][NT];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int t = h - l;
      const int64_t kidx = kbase + ((int64_t)l * pt.T + t) * tl.kf_total + ks;
      const int p0 = plo + 32 * ks + 4 * kg;
#pragma unroll
      for (int u = 0; u < NT; ++u) v[b][u] = load8(qcol[u] + t * ly.q_t + (p0 >> 2) * ly.q_b, ly.q_b);
      float s0 = 1.f, s1 = 1.f;
      if constexpr (MODE != kBF16) {
        const float* scl = tl.scale + (((int64_t)c * pt.K + l) * pt.T + t) * tl.n_ptile;
        s0 = scl[min(p0 >> 6, tl.n_ptile - 1)];
        s1 = scl[min((p0 + 16) >> 6, tl.n_ptile - 1)];
      }
#pragma unroll
      for (int tt = 0; tt < TP; ++tt) {
        const int64_t kt = kidx + tt * nks;
        if (tt >= n_tt || it0 + b >= n_it) {
          a[b][tt] = zero;
          if constexpr (MODE == kFP8Corr) ac[b][tt] = zero;
        } else if constexpr (MODE == kFP8Corr) {
          a[b][tt] = load_a_scaled(tl.Fv, kt, lane, s0, s1);
          ac[b][tt] = load_corr(tl.Fc, kt, lane);
        } else {
          a[b][tt] = load_a<MODE>(tl.Fv, kt, lane);
        }
      }
      if constexpr (MODE == kFP8) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          v[b][u][0] *= s0; v[b][u][1] *= s0; v[b][u][2] *= s0; v[b][u][3] *= s0;
          v[b][u][4] *= s1; v[b][u][5] *= s1; v[b][u][6] *= s1; v[b][u][7] *= s1;
        }
      }
      if (it0 + b < n_it && it0 + b + 1 < n_it && ++ks == nks) {
        ks = 0;
        ++l;
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const bf16x8 hi = __builtin_convertvector(v[b][u], bf16x8);
        const bf16x8 lo = __builtin_convertvector(v[b][u] - __builtin_convertvector(hi, f32x8), bf16x8);
#pragma unroll
        for (int tt = 0; tt < TP; ++tt) {
          acc[tt][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[b][tt], hi, acc[tt][u], 0, 0, 0);
          acc[tt][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[b][tt], lo, acc[tt][u], 0, 0, 0);
          if constexpr (MODE == kFP8Corr) {
            acc[tt][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac[b][tt], hi, acc[tt][u], 0, 0, 0);
            acc[tt][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac[b][tt], lo, acc[tt][u], 0, 0, 0);
          }
        }
      }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int64_t du = live[u] ? first + 16 * u + n : first;
#pragma unroll
    for (int tt = 0; tt < TP; ++tt)
      x[tt][u] = tt < n_tt ? load4(X + du * ly.x_d + h * ly.x_h + ((16 * (i0 + tt) + 4 * kg) >> 2) * ly.x_b)
                           : f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int tt = 0; tt < TP; ++tt) {
    const int a0 = 16 * (i0 + tt) + 4 * kg;
    if (tt >= n_tt || a0 >= pt.L) continue;
    const bool full = a0 + 4 <= pt.L;
    const int valid = pt.L - a0;
#pragma unroll
    for (int u = 0; u < NT; ++u)
      if (live[u])
        store4(R + (int64_t)(first + 16 * u + n) * ly.r_d + s * ly.r_s + (a0 >> 2) * ly.r_b,
               acc[tt][u] - x[tt][u], full, valid);
  }
}

// Work item of a wave: its entry of the launch's work table (one scalar load).
__device__ __forceinline__ WaveWork load_work(const WaveWork* __restrict__ wt, int item) {
  const int4* p = reinterpret_cast<const int4*>(wt + item);
  const int4 a = p[0], b = p[1];
  return WaveWork{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// Forward product and residual of the minibatch rows, one wave per entry of
// the launch's work table (slot, day group, link-tile group of a cluster), 4
// per block; blocks remapped so each XCD walks a contiguous range of the table.
template <int MODE, int NT>
__global__ void __launch_bounds__(256)
k_fwd_mfma(DevPat pt, DevTiles tl, ChunkSched cs, const WaveWork* __restrict__ wt, int n_items,
           Layout ly, const float* __restrict__ Q, const float* __restrict__ X,
           float* __restrict__ R) {
  // the wave index is uniform: everything derived from it lives in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_logical_block((n_items + 3) / 4) * 4 + wave;
  if (item >= n_items) return;
  const WaveWork w = load_work(wt, item);
  if (cs.j0 + w.row >= pt.H) return;
  cs = resolve_epoch(cs);
  const int h = cs.perm[w.c * pt.H + cs.j0 + w.row];
  fwd_group<MODE, NT, kFwdTileGroup>(pt, tl, ly, w, h, Q, X, R);
}

__device__ __forceinline__ f32x4 step4(f32x4 q, f32x4& a, const f32x4& g, const StepArgs& st) {
  const float eta = static_cast<float>(st.eta), eps = static_cast<float>(st.eps);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (st.optimizer == 0) {
      a[k] += g[k] * g[k];
      q[k] -= eta * g[k] / (sqrtf(a[k]) + eps);
    } else {
      q[k] -= eta * g[k];
    }
    q[k] = q[k] > 0.f ? q[k] : 0.f;
  }
  return q;
}

// Adjoint of the minibatch and the fused Adagrad step + projection:
//   g_d[t][p] = sum_{l: t+l in minibatch} rho_c[l][t][:, p] . R_d[slot(t+l)][:]
// Same batching and day columns as the forward product.  The demand and
// accumulator rows are fetched before the product.
// One adjoint item: OD tile j of the reached departure interval described by
// dsc, for day group g of cluster c, with the step and projection fused.
template <int MODE, int NT>
__device__ __forceinline__ void adj_item(const DevPat& pt, const DevTiles& tl, const Layout& ly,
                                         const WaveWork& w, const int32_t* dsc,
                                         const float* __restrict__ R, float* __restrict__ Q,
                                         float* __restrict__ A, const StepArgs& st) {
  const int c = w.c, j = w.tile;
  constexpr int kBatch = NT == 2 ? 3 : 8 / NT;
  const int lane = threadIdx.x & 63;
  const int t = dsc[kDescT];
  // lags whose row block h = t + l is in this minibatch
  const uint64_t lmask = (uint64_t)(uint32_t)dsc[kDescMask] |
                         (uint64_t)(uint32_t)dsc[kDescMask + 1] << 32;
  const int n = lane & 15, kg = lane >> 4;
  const int first = w.first, cnt = w.count;
  const int p0 = 16 * j + 4 * kg;
  const bool adagrad = st.optimizer == 0;
  bool live[NT];
  const float* rcol[NT];
  f32x4 q[NT], a[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    live[u] = 16 * u + n < cnt;
    const int64_t du = live[u] ? first + 16 * u + n : first;
    rcol[u] = R + du * ly.r_d;
    const int64_t idx = du * ly.q_d + t * ly.q_t + (p0 >> 2) * ly.q_b;
    q[u] = load4(Q + idx);
    a[u] = adagrad ? load4(A + idx) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int nks = w.nks, alo = w.lo;
  const int n_it = __popcll(lmask) * nks;
  const int64_t kbase = (int64_t)c * pt.K * pt.T * tl.kg_total + w.koff;
  f32x4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = __builtin_convertvector(f32x8{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, bf16x8);
  // iteration -> (lag = next set bit of lmask, k-step)
  uint64_t m = lmask;
  int l = m ? __builtin_ctzll(m) : 0, ks = 0;
  for (int it0 = 0; it0 < n_it; it0 += kBatch) {
    bf16x8 w[kBatch], wc[MODE == kFP8Corr ? kBatch : 1];
    f32x8 v[kBatch][NT];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int64_t kidx = kbase + ((int64_t)l * pt.T + t) * tl.kg_total + ks;
      const int sl = dsc[kDescSlot + l];
      const int k0 = alo + 32 * ks + 4 * kg;
#pragma unroll
      for (int u = 0; u < NT; ++u) v[b][u] = load8(rcol[u] + sl * ly.r_s + (k0 >> 2) * ly.r_b, ly.r_b);
      if constexpr (MODE == kBF16) {
        w[b] = load_a<MODE>(tl.Gv, kidx, lane);
      } else {
        // the tile's 16 ODs lie in one 64-OD scale group
        const float sc = tl.scale[(((int64_t)c * pt.K + l) * pt.T + t) * tl.n_ptile + ((16 * j) >> 6)];
        if constexpr (MODE == kFP8) {
          w[b] = load_a<MODE>(tl.Gv, kidx, lane);
#pragma unroll
          for (int u = 0; u < NT; ++u) v[b][u] *= sc;
        } else {
          w[b] = load_a_scaled(tl.Gv, kidx, lane, sc, sc);
          wc[b] = load_corr(tl.Gc, kidx, lane);
        }
      }
      if (it0 + b >= n_it) {
        w[b] = zero;
        if constexpr (MODE == kFP8Corr) wc[b] = zero;
      } else if (it0 + b + 1 < n_it && ++ks == nks) {
        ks = 0;
        m &= m - 1;
        l = __builtin_ctzll(m);
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        mma_split(w[b], v[b][u], acc[u]);
        if constexpr (MODE == kFP8Corr) mma_split(wc[b], v[b][u], acc[u]);
      }
  }
  if (p0 >= pt.P) return;
  const bool full = p0 + 4 <= pt.P;
  const int valid = pt.P - p0;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (!live[u]) continue;
    const int64_t idx = (int64_t)(first + 16 * u + n) * ly.q_d + t * ly.q_t + (p0 >> 2) * ly.q_b;
    q[u] = step4(q[u], a[u], acc[u], st);
    store4(Q + idx, q[u], full, valid);
    if (adagrad) store4(A + idx, a[u], full, valid);
  }
}

// Adjoint of the minibatch and the fused Adagrad step + projection, one wave
// per entry of the launch's work table (reached interval index, day group, OD
// tile of a cluster), 4 per block; blocks remapped so each XCD walks a
// contiguous range of the table.
template <int MODE, int NT>
__global__ void __launch_bounds__(256)
k_adj_mfma(DevPat pt, DevTiles tl, ChunkSched cs, const WaveWork* __restrict__ wt, int n_items,
           Layout ly, const float* __restrict__ R, float* __restrict__ Q, float* __restrict__ A,
           StepArgs st) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_logical_block((n_items + 3) / 4) * 4 + wave;
  if (item >= n_items) return;
  const WaveWork w = load_work(wt, item);
  cs = resolve_epoch(cs);
  const int32_t* dsc = cs.touched + ((int64_t)w.c * cs.max_touched + w.row) * desc_width(pt.K);
  if (dsc[kDescT] < 0) return;
  adj_item<MODE, NT>(pt, tl, ly, w, dsc, R, Q, A, st);
}

// Adjoint + step for one chunk of reached departure intervals t0..t0+n_t-1
// (consecutive, of one component) for OD tile j and one day group: every
// residual row h that reaches the chunk is loaded once per k-step and
// multiplied into each t with 0 <= h - t < K (the lag block (h - t, t)).  Each
// t gets its products in increasing lag and k-step order, as in adj_item, so
// the results are the same bits; the residual loads (and, in BF16 mode, their
// head/tail split) are shared by up to kChunkT intervals.  Iterations (row,
// k-step) run in batches of CB whose loads are all issued before the first
// product.
template <int MODE, int NT>
__device__ __forceinline__ void adj_chunk_item(const DevPat& pt, const DevTiles& tl,
                                               const Layout& ly, const ChunkList& ck,
                                               const WaveWork& w, const float* __restrict__ R,
                                               float* __restrict__ Q, float* __restrict__ A,
                                               const StepArgs& st) {
  constexpr int CB = NT == 1 ? 1 : 2;   // 4 and 3 waves per SIMD
  constexpr int G = kChunkT;
  const int lane = threadIdx.x & 63;
  const int32_t* cr = ck.chunk + ((int64_t)w.c * ck.max_chunks + w.row) * ck.w;
  const int t0 = cr[0], n_t = cr[1], n_h = cr[2];
  if (n_t == 0) return;
  const int c = w.c, j = w.tile;
  const int n = lane & 15, kg = lane >> 4;
  const int first = w.first, cnt = w.count;
  const int p0 = 16 * j + 4 * kg;
  bool live[NT];
  const float* rcol[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    live[u] = 16 * u + n < cnt;
    const int64_t du = live[u] ? first + 16 * u + n : first;
    rcol[u] = R + du * ly.r_d;
  }
  const int nks = w.nks, alo = w.lo;
  const int n_it = n_h * nks;
  const int64_t kbase = (int64_t)c * pt.K * pt.T * tl.kg_total + w.koff;
  f32x4 acc[G][NT];
#pragma unroll
  for (int k = 0; k < G; ++k)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[k][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  int ih = 0, ks = 0;
  int h = cr[3], sl = cr[4];
  for (int it0 = 0; it0 < n_it; it0 += CB) {
    f32x8 v[CB][NT];
    bf16x8 wa[CB][G], wc[MODE == kFP8Corr ? CB : 1][G];
    float sc[CB][G];
    bool use[CB][G];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const bool in = it0 + b < n_it;
      const int k0 = alo + 32 * ks + 4 * kg;
#pragma unroll
      for (int u = 0; u < NT; ++u) v[b][u] = load8(rcol[u] + sl * ly.r_s + (k0 >> 2) * ly.r_b, ly.r_b);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int lag = h - (t0 + k);
        use[b][k] = in && k < n_t && lag >= 0 && lag < pt.K;
        if (use[b][k]) {
          const int64_t kidx = kbase + ((int64_t)lag * pt.T + t0 + k) * tl.kg_total + ks;
          if constexpr (MODE != kBF16)
            sc[b][k] = tl.scale[(((int64_t)c * pt.K + lag) * pt.T + t0 + k) * tl.n_ptile +
                                ((16 * j) >> 6)];
          if constexpr (MODE == kFP8Corr) {
            wa[b][k] = load_a_scaled(tl.Gv, kidx, lane, sc[b][k], sc[b][k]);
            wc[b][k] = load_corr(tl.Gc, kidx, lane);
          } else {
            wa[b][k] = load_a<MODE>(tl.Gv, kidx, lane);
          }
        }
      }
      if (in && it0 + b + 1 < n_it && ++ks == nks) {
        ks = 0;
        ++ih;
        h = cr[3 + 2 * ih];
        sl = cr[4 + 2 * ih];
      }
    }
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        if constexpr (MODE != kFP8) {
          const bf16x8 hi = __builtin_convertvector(v[b][u], bf16x8);
          const bf16x8 lo =
              __builtin_convertvector(v[b][u] - __builtin_convertvector(hi, f32x8), bf16x8);
#pragma unroll
          for (int k = 0; k < G; ++k)
            if (use[b][k]) {
              acc[k][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[b][k], hi, acc[k][u], 0, 0, 0);
              acc[k][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[b][k], lo, acc[k][u], 0, 0, 0);
              if constexpr (MODE == kFP8Corr) {
                acc[k][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wc[b][k], hi, acc[k][u], 0, 0, 0);
                acc[k][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wc[b][k], lo, acc[k][u], 0, 0, 0);
              }
            }
        } else {
#pragma unroll
          for (int k = 0; k < G; ++k)
            if (use[b][k]) mma_split(wa[b][k], v[b][u] * sc[b][k], acc[k][u]);
        }
      }
  }
  if (p0 >= pt.P) return;
  const bool full = p0 + 4 <= pt.P;
  const int valid = pt.P - p0;
  const bool adagrad = st.optimizer == 0;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    if (k >= n_t) break;
    const int t = t0 + k;
    f32x4 q[NT], a[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int64_t du = live[u] ? first + 16 * u + n : first;
      const int64_t idx = du * ly.q_d + t * ly.q_t + (p0 >> 2) * ly.q_b;
      q[u] = load4(Q + idx);
      a[u] = adagrad ? load4(A + idx) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (!live[u]) continue;
      const int64_t idx = (int64_t)(first + 16 * u + n) * ly.q_d + t * ly.q_t + (p0 >> 2) * ly.q_b;
      q[u] = step4(q[u], a[u], acc[k][u], st);
      store4(Q + idx, q[u], full, valid);
      if (adagrad) store4(A + idx, a[u], full, valid);
    }
  }
}

// Chunked adjoint and step, one wave per entry of the launch's work table
// (chunk, OD tile, day group of a cluster), 4 per block; blocks remapped so
// each XCD walks a contiguous range of the table.
template <int MODE, int NT>
__global__ void __launch_bounds__(256)
k_adj_chunk(DevPat pt, DevTiles tl, ChunkList ck, const WaveWork* __restrict__ wt, int n_items,
            Layout ly, const float* __restrict__ R, float* __restrict__ Q, float* __restrict__ A,
            StepArgs st) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_logical_block((n_items + 3) / 4) * 4 + wave;
  if (item >= n_items) return;
  const WaveWork w = load_work(wt, item);
  adj_chunk_item<MODE, NT>(pt, tl, ly, resolve_epoch(ck), w, R, Q, A, st);
}

// One whole minibatch in one launch, one workgroup per (cluster, component,
// day group).  A component is a maximal run of the minibatch's intervals whose
// reached departure intervals overlap (sorted intervals less than K apart); the
// reached intervals of different components are disjoint, so components are
// independent within the minibatch.  The workgroup's four waves first compute
// the residual rows of the component's intervals (every link tile), wait at a
// barrier, then run the adjoint and the step for every reached interval of the
// component (every OD tile).  The residual rows travel through the L2 of the
// workgroup's XCD, and the demand rows the forward product read are the rows
// the step rewrites.  Each item does exactly the arithmetic of the separate
// forward and adjoint kernels, so results are the same bits.
template <int MODE, int NT>
__global__ void __launch_bounds__(256)
k_minibatch_mfma(DevPat pt, DevTiles tl, CompSched ks, DayGroups dg, Layout ly,
                 const float* __restrict__ X, float* __restrict__ R, float* __restrict__ Q,
                 float* __restrict__ A, StepArgs st) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_items = dg.n * ks.max_comp;
  const int item = xcd_logical_block(n_items);
  if (item >= n_items) return;   // uniform over the workgroup
  int c, k, unused;
  const int g = decode_item(dg, item, ks.max_comp, 1, c, k, unused);
  ks = resolve_epoch(ks);
  const int32_t* cp = ks.comp + ((int64_t)c * ks.max_comp + k) * 4;
  const int h0 = cp[0], n_h = cp[1], d0 = cp[2], n_t = cp[3];
  if (n_h == 0) return;          // padding entry, uniform over the workgroup
  const int32_t* slots = ks.slot + (int64_t)c * ks.bh;
  const int first = dg.first[g], cnt = dg.count[g];
  for (int task = wave; task < n_h * tl.nLT; task += 4) {
    const int a = task / tl.nLT, i = task - a * tl.nLT;
    const int s = slots[h0 + a];
    const int h = ks.perm[c * pt.H + ks.j0 + s];
    const WaveWork w{c, first, cnt, s, i, tl.f_ks[i], tl.f_plo[i], tl.f_koff[i]};
    fwd_item<MODE, NT>(pt, tl, ly, w, h, Q, X, R);
  }
  __syncthreads();
  const int dw = desc_width(pt.K);
  for (int task = wave; task < n_t * tl.nPT; task += 4) {
    const int b = task / tl.nPT, j = task - b * tl.nPT;
    const int32_t* dsc = ks.desc + ((int64_t)c * ks.mt + d0 + b) * dw;
    const WaveWork w{c, first, cnt, d0 + b, j, tl.g_ks[j], tl.g_alo[j], tl.g_koff[j]};
    adj_item<MODE, NT>(pt, tl, ly, w, dsc, R, Q, A, st);
  }
}

// Grid barrier of the persistent epoch kernel.  Every wave first waits until
// its own stores have reached its XCD's L2 (a fence by one thread after a
// workgroup barrier does not wait for the other waves' stores); the block's
// first thread then writes the L2 back (device-scope release: the XCDs' L2s
// are not coherent with each other), arrives on the counter, waits until the
// last arrival moves the generation on, and invalidates its L2 and the L1 the
// block's waves share (device-scope acquire).  The wait is bounded: after
// `spin_limit` polls, or once any block has given up, the block sets the
// error word and returns false, and every later barrier returns false at
// once, so every block leaves the kernel; the host turns the error word into
// an error.  The kernel must be launched with all its blocks resident (a
// cooperative launch).
__device__ bool grid_barrier(PersistBarrier* b, unsigned n_blocks, unsigned& gen,
                             unsigned spin_limit) {
  __shared__ int ok;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    if (good) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned arrived =
          __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == n_blocks - 1) {
        __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&b->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        // relaxed polls (no cache invalidation while the other blocks work),
        // one acquire fence once the generation has moved on
        unsigned polls = 0;
        while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          if (++polls > spin_limit ||
              __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_store(&b->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            good = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ok = good;
  }
  __syncthreads();
  ++gen;
  return ok != 0;
}

// The epoch held by a device-epoch schedule, taken from an argument instead.
__device__ __forceinline__ ChunkSched at_epoch(ChunkSched cs, int e) {
  cs.perm += e * cs.perm_e;
  cs.pos += e * cs.perm_e;
  cs.touched += e * cs.touched_e;
  cs.epoch = nullptr;
  return cs;
}
__device__ __forceinline__ ChunkList at_epoch(ChunkList ck, int e) {
  ck.chunk += e * ck.chunk_e;
  ck.epoch = nullptr;
  return ck;
}

// Every minibatch of one epoch in one launch: the blocks stay resident and
// walk the forward work table of minibatch j, meet at a grid barrier, walk the
// adjoint work table (with the step and projection), meet again, and go on to
// minibatch j + 1.  Each XCD takes one contiguous eighth of each table (its
// blocks are those with blockIdx % 8 equal to it, items strided over them),
// so items that share tiles run under one L2.  Every item does the
// arithmetic of the separate forward and adjoint kernels, so the results are
// the same bits.  (Handing out items from an atomic counter per phase and XCD
// instead of the fixed stride made the epoch twice as slow.)
template <int MODE, int NT, bool CHUNKED>
__global__ void __launch_bounds__(256)
k_epoch_persistent(DevPat pt, DevTiles tl, const PersistMinibatch* __restrict__ mb, int nch,
                   int epoch, const WaveWork* __restrict__ wt_fwd, int n_fwd,
                   const WaveWork* __restrict__ wt_adj, int n_adj, Layout ly,
                   const float* __restrict__ X, float* __restrict__ R, float* __restrict__ Q,
                   float* __restrict__ A, StepArgs st, PersistBarrier* bar, unsigned spin_limit) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const int stride = (gridDim.x / kXcds) * 4;
  const int f_lo = (int)((int64_t)n_fwd * xcd / kXcds), f_hi = (int)((int64_t)n_fwd * (xcd + 1) / kXcds);
  const int a_lo = (int)((int64_t)n_adj * xcd / kXcds), a_hi = (int)((int64_t)n_adj * (xcd + 1) / kXcds);
  unsigned gen = 0;
  for (int j = 0; j < nch; ++j) {
    const ChunkSched cs = at_epoch(mb[j].cs, epoch);
    for (int item = f_lo + local * 4 + wave; item < f_hi; item += stride) {
      const WaveWork w = load_work(wt_fwd, item);
      if (cs.j0 + w.row >= pt.H) continue;
      const int h = cs.perm[w.c * pt.H + cs.j0 + w.row];
      fwd_group<MODE, NT, kFwdTileGroup>(pt, tl, ly, w, h, Q, X, R);
    }
    if (!grid_barrier(bar, gridDim.x, gen, spin_limit)) return;
    if constexpr (CHUNKED) {
      const ChunkList ck = at_epoch(mb[j].ck, epoch);
      for (int item = a_lo + local * 4 + wave; item < a_hi; item += stride)
        adj_chunk_item<MODE, NT>(pt, tl, ly, ck, load_work(wt_adj, item), R, Q, A, st);
    } else {
      for (int item = a_lo + local * 4 + wave; item < a_hi; item += stride) {
        const WaveWork w = load_work(wt_adj, item);
        const int32_t* dsc = cs.touched + ((int64_t)w.c * cs.max_touched + w.row) * desc_width(pt.K);
        if (dsc[kDescT] < 0) continue;
        adj_item<MODE, NT>(pt, tl, ly, w, dsc, R, Q, A, st);
      }
    }
    if (j + 1 < nch && !grid_barrier(bar, gridDim.x, gen, spin_limit)) return;
  }
}

// Copy the pattern-form codes of one (cluster, l, t) block (link-sliced, just
// rewritten by the quantisation kernel) into its packed tiles.
template <typename E>
__global__ void __launch_bounds__(256)
k_update_tiles(DevPat pt, DevTiles tl, int32_t c, const E* __restrict__ codes,
               const int32_t* __restrict__ posf, const int32_t* __restrict__ posg,
               const int32_t* __restrict__ csc2csr, E* __restrict__ F, E* __restrict__ G) {
  const int64_t lt = blockIdx.x;
  const int l = (int)(lt / pt.T), t = (int)(lt % pt.T);
  if (t + l >= pt.H) return;   // block never read
  const int64_t blk = (int64_t)c * pt.K * pt.T + lt;
  const E* w = codes + blk * pt.sr_len;   // link-sliced codes
  E* f = F + blk * tl.kf_total * 512;
  E* g = G + blk * tl.kg_total * 512;
  for (int64_t j = threadIdx.x; j < pt.nnz; j += blockDim.x) f[posf[j]] = w[pt.sr_pos[j]];
  for (int64_t jj = threadIdx.x; jj < pt.nnz; jj += blockDim.x)
    g[posg[jj]] = w[pt.sr_pos[csc2csr[jj]]];
}

}  // namespace

hipError_t update_tiles(const dode_dar* dar, int32_t cluster, hipStream_t s) {
  const dim3 grid(dar->dims.K * dar->dims.T);
  if (dar->storage == DODE_FP8_E4M3)
    hipLaunchKernelGGL(k_update_tiles<uint8_t>, grid, dim3(256), 0, s, dar->pat(), dar->tiles,
                       cluster, static_cast<const uint8_t*>(dar->d_W), dar->d_posf, dar->d_posg,
                       dar->d_csc2csr, static_cast<uint8_t*>(dar->d_Fv),
                       static_cast<uint8_t*>(dar->d_Gv));
  else
    hipLaunchKernelGGL(k_update_tiles<uint16_t>, grid, dim3(256), 0, s, dar->pat(), dar->tiles,
                       cluster, static_cast<const uint16_t*>(dar->d_W), dar->d_posf, dar->d_posg,
                       dar->d_csc2csr, static_cast<uint16_t*>(dar->d_Fv),
                       static_cast<uint16_t*>(dar->d_Gv));
  return hipGetLastError();
}

template <int MODE, int NT>
hipError_t launch_fwd(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt, int64_t n,
                      const Layout& ly, const float* Q, const float* X, float* R, hipStream_t s) {
  const int64_t nblk = (n + 3) / 4;
  const dim3 grid((unsigned)(((nblk + kXcds - 1) / kXcds) * kXcds));
  hipLaunchKernelGGL((k_fwd_mfma<MODE, NT>), grid, dim3(256), 0, s, dar->pat(), dar->tiles, cs, wt,
                     (int)n, ly, Q, X, R);
  return hipGetLastError();
}

template <int MODE, int NT>
hipError_t launch_adj(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt, int64_t n,
                      const Layout& ly, const float* R, float* Q, float* A, const StepArgs& st,
                      hipStream_t s) {
  const int64_t nblk = (n + 3) / 4;
  const dim3 grid((unsigned)(((nblk + kXcds - 1) / kXcds) * kXcds));
  hipLaunchKernelGGL((k_adj_mfma<MODE, NT>), grid, dim3(256), 0, s, dar->pat(), dar->tiles, cs, wt,
                     (int)n, ly, R, Q, A, st);
  return hipGetLastError();
}

template <int MODE, int NT>
hipError_t launch_minibatch(const dode_dar* dar, const CompSched& ks, const DayGroups& dg,
                            const Layout& ly, const float* X, float* R, float* Q, float* A,
                            const StepArgs& st, hipStream_t s) {
  const int64_t nblk = (int64_t)dg.n * ks.max_comp;
  const dim3 grid((unsigned)(((nblk + kXcds - 1) / kXcds) * kXcds));
  hipLaunchKernelGGL((k_minibatch_mfma<MODE, NT>), grid, dim3(256), 0, s, dar->pat(), dar->tiles,
                     ks, dg, ly, X, R, Q, A, st);
  return hipGetLastError();
}

template <int NT>
hipError_t minibatch_mode(const dode_dar* dar, const CompSched& ks, const DayGroups& dg,
                          const Layout& ly, const float* X, float* R, float* Q, float* A,
                          const StepArgs& st, hipStream_t s) {
  if (dar->storage != DODE_FP8_E4M3) return launch_minibatch<kBF16, NT>(dar, ks, dg, ly, X, R, Q, A, st, s);
  return launch_minibatch<kFP8, NT>(dar, ks, dg, ly, X, R, Q, A, st, s);
}

template <int MODE, int NT>
hipError_t launch_adj_chunk(const dode_dar* dar, const ChunkList& ck, const WaveWork* wt, int64_t n,
                            const Layout& ly, const float* R, float* Q, float* A,
                            const StepArgs& st, hipStream_t s) {
  const int64_t nblk = (n + 3) / 4;
  const dim3 grid((unsigned)(((nblk + kXcds - 1) / kXcds) * kXcds));
  hipLaunchKernelGGL((k_adj_chunk<MODE, NT>), grid, dim3(256), 0, s, dar->pat(), dar->tiles, ck,
                     wt, (int)n, ly, R, Q, A, st);
  return hipGetLastError();
}

template <int NT>
hipError_t fwd_mode(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt, int64_t n,
                    const Layout& ly, const float* Q, const float* X, float* R, bool corr,
                    hipStream_t s) {
  if (dar->storage != DODE_FP8_E4M3) return launch_fwd<kBF16, NT>(dar, cs, wt, n, ly, Q, X, R, s);
  if (corr) return launch_fwd<kFP8Corr, NT>(dar, cs, wt, n, ly, Q, X, R, s);
  return launch_fwd<kFP8, NT>(dar, cs, wt, n, ly, Q, X, R, s);
}

template <int NT>
hipError_t adj_mode(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt, int64_t n,
                    const Layout& ly, const float* R, float* Q, float* A, const StepArgs& st,
                    bool corr, hipStream_t s) {
  if (dar->storage != DODE_FP8_E4M3)
    return launch_adj<kBF16, NT>(dar, cs, wt, n, ly, R, Q, A, st, s);
  if (corr) return launch_adj<kFP8Corr, NT>(dar, cs, wt, n, ly, R, Q, A, st, s);
  return launch_adj<kFP8, NT>(dar, cs, wt, n, ly, R, Q, A, st, s);
}

hipError_t mfma_chunk_resid(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt,
                            int64_t n, int32_t day_tile, const Layout& ly, const float* Q,
                            const float* X, float* R, bool corr, hipStream_t s) {
  if (corr && !dar->has_corr) return hipErrorInvalidValue;
  if (n > INT32_MAX) return hipErrorInvalidValue;
  switch (day_tile) {
    case 16: return fwd_mode<1>(dar, cs, wt, n, ly, Q, X, R, corr, s);
    case 64: return fwd_mode<4>(dar, cs, wt, n, ly, Q, X, R, corr, s);
    default: return fwd_mode<2>(dar, cs, wt, n, ly, Q, X, R, corr, s);
  }
}

hipError_t mfma_chunk_adj_step(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt,
                               int64_t n, int32_t day_tile, const Layout& ly, const float* R,
                               float* Q, float* A, const StepArgs& st, bool corr, hipStream_t s) {
  if (corr && !dar->has_corr) return hipErrorInvalidValue;
  if (n > INT32_MAX) return hipErrorInvalidValue;
  switch (day_tile) {
    case 16: return adj_mode<1>(dar, cs, wt, n, ly, R, Q, A, st, corr, s);
    case 64: return adj_mode<4>(dar, cs, wt, n, ly, R, Q, A, st, corr, s);
    default: return adj_mode<2>(dar, cs, wt, n, ly, R, Q, A, st, corr, s);
  }
}

hipError_t mfma_minibatch(const dode_dar* dar, const CompSched& ks, const DayGroups& dg,
                          const Layout& ly, const float* X, float* R, float* Q, float* A,
                          const StepArgs& st, hipStream_t s) {
  switch (dg.tile) {
    case 16: return minibatch_mode<1>(dar, ks, dg, ly, X, R, Q, A, st, s);
    case 64: return minibatch_mode<4>(dar, ks, dg, ly, X, R, Q, A, st, s);
    default: return minibatch_mode<2>(dar, ks, dg, ly, X, R, Q, A, st, s);
  }
}

hipError_t mfma_adj_chunks(const dode_dar* dar, const ChunkList& ck, const WaveWork* wt, int64_t n,
                           int32_t day_tile, const Layout& ly, const float* R, float* Q, float* A,
                           const StepArgs& st, bool corr, hipStream_t s) {
  if (n > INT32_MAX || day_tile == 64) return hipErrorInvalidValue;
  if (corr && !dar->has_corr) return hipErrorInvalidValue;
  const bool fp8 = dar->storage == DODE_FP8_E4M3;
  if (day_tile == 16) {
    if (corr) return launch_adj_chunk<kFP8Corr, 1>(dar, ck, wt, n, ly, R, Q, A, st, s);
    return fp8 ? launch_adj_chunk<kFP8, 1>(dar, ck, wt, n, ly, R, Q, A, st, s)
               : launch_adj_chunk<kBF16, 1>(dar, ck, wt, n, ly, R, Q, A, st, s);
  }
  if (corr) return launch_adj_chunk<kFP8Corr, 2>(dar, ck, wt, n, ly, R, Q, A, st, s);
  return fp8 ? launch_adj_chunk<kFP8, 2>(dar, ck, wt, n, ly, R, Q, A, st, s)
             : launch_adj_chunk<kBF16, 2>(dar, ck, wt, n, ly, R, Q, A, st, s);
}

template <int MODE, int NT, bool CHUNKED>
hipError_t launch_persistent(const dode_dar* dar, const PersistMinibatch* mb, int nch, int epoch,
                             const WaveWork* wt_fwd, int64_t n_fwd, const WaveWork* wt_adj,
                             int64_t n_adj, const Layout& ly, const float* X, float* R, float* Q,
                             float* A, const StepArgs& st, PersistBarrier* bar,
                             unsigned spin_limit, hipStream_t s) {
  auto kern = k_epoch_persistent<MODE, NT, CHUNKED>;
  int per_cu = 0, dev = 0, n_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // every block resident; no more blocks than the larger table has waves,
  // and a multiple of the XCD count
  const int64_t need = (std::max(n_fwd, n_adj) + 3) / 4;
  int64_t blocks = std::min<int64_t>((int64_t)per_cu * n_cu, need);
  blocks = std::max<int64_t>(kXcds, blocks / kXcds * kXcds);
  if (blocks > (int64_t)per_cu * n_cu) return hipErrorCooperativeLaunchTooLarge;
  DevPat pt = dar->pat();
  DevTiles tl = dar->tiles;
  int nf = (int)n_fwd, na = (int)n_adj;
  void* args[] = {&pt, &tl, &mb, &nch, &epoch, &wt_fwd, &nf, &wt_adj, &na,
                  const_cast<Layout*>(&ly), &X, &R, &Q, &A, const_cast<StepArgs*>(&st), &bar,
                  &spin_limit};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)blocks),
                                    dim3(256), args, 0, s);
}

template <int NT, bool CHUNKED>
hipError_t persistent_mode(const dode_dar* dar, const PersistMinibatch* mb, int nch, int epoch,
                           const WaveWork* wt_fwd, int64_t n_fwd, const WaveWork* wt_adj,
                           int64_t n_adj, const Layout& ly, const float* X, float* R, float* Q,
                           float* A, const StepArgs& st, PersistBarrier* bar, unsigned spin_limit,
                           hipStream_t s) {
  if (dar->storage != DODE_FP8_E4M3)
    return launch_persistent<kBF16, NT, CHUNKED>(dar, mb, nch, epoch, wt_fwd, n_fwd, wt_adj, n_adj,
                                                 ly, X, R, Q, A, st, bar, spin_limit, s);
  return launch_persistent<kFP8, NT, CHUNKED>(dar, mb, nch, epoch, wt_fwd, n_fwd, wt_adj, n_adj,
                                              ly, X, R, Q, A, st, bar, spin_limit, s);
}

hipError_t mfma_epoch_persistent(const dode_dar* dar, const PersistMinibatch* mb, int32_t nch,
                                 int32_t epoch, const WaveWork* wt_fwd, int64_t n_fwd,
                                 const WaveWork* wt_adj, int64_t n_adj, int32_t order,
                                 int32_t day_tile, const Layout& ly, const float* X, float* R,
                                 float* Q, float* A, const StepArgs& st, PersistBarrier* bar,
                                 uint32_t spin_limit, hipStream_t s) {
  if (n_fwd > INT32_MAX || n_adj > INT32_MAX || (order == 2 && day_tile == 64))
    return hipErrorInvalidValue;
#define PERSIST_ARGS dar, mb, nch, epoch, wt_fwd, n_fwd, wt_adj, n_adj, ly, X, R, Q, A, st, bar, spin_limit, s
  const bool chunked = order == 2;
  switch (day_tile) {
    case 16: return chunked ? persistent_mode<1, true>(PERSIST_ARGS)
                            : persistent_mode<1, false>(PERSIST_ARGS);
    case 64: return persistent_mode<4, false>(PERSIST_ARGS);
    default: return chunked ? persistent_mode<2, true>(PERSIST_ARGS)
                            : persistent_mode<2, false>(PERSIST_ARGS);
  }
#undef PERSIST_ARGS
}
