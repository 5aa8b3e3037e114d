// Dynamic assignment ratios from link speeds (section "Dynamic assignment
// ratio", eqs. "dar2"/"dar" and Example "DAR matrix computation"; section
// "Link/path travel time", eq. "cost").
//
// Time is in minutes and observation intervals are [h*dt, (h+1)*dt).  A link
// entered at time t is crossed in len/speed(interval of t); the last
// interval's speed holds after the end of the day.  A vehicle of path k
// departing at t enters the path's i-th link at tau_i(t): tau_0(t) = t,
// tau_{i+1}(t) = tau_i(t) + c(tau_i(t)).  Departure interval h maps onto the
// arrival window [tau_i(h dt), tau_i((h+1) dt)] at that link, and the ratio of
// observation interval h2 is the share of the window inside it.
//
// Two kernels per chunk of days:
//   k_trajectories  one thread per (eight days, path, boundary b in 0..H): the travel
//                   time from the b*dt departure to the entry of every link of
//                   the path, traj[day][pair][b] (pairs = (path, i) in path
//                   order), and optionally the whole path's travel time (the
//                   path cost of eq. "cost" for a departure at b*dt), whose
//                   day mean k_exit_sums forms;
//   k_dar_windows   one thread per (pair, departure interval h): the shares
//                   of the day windows, [r_h, dt + r_{h+1}] relative to h*dt,
//                   summed over the chunk's days in order, added into the
//                   running sums; the last chunk divides by the day count.
//                   The share of interval h+l is F((l+1) dt) - F(l dt), with
//                   F(x) = clamp((x - lo) / w, 0, 1) the fraction of the window
//                   before x (the window's overlap with the interval over w).
// Keeping times relative to the departure keeps the window arithmetic at the
// precision of travel times (tens of minutes), not of times of day.
//
// Mean path travel times (eqs. "cost", "logit", "rt"): the same walk from the
// departure at t*dt to the exit of the path's last link, for every day of a
// pattern, averaged over the days.  Two kernels:
//   k_path_cost_slices  one thread per (slice of days, path, t), t fastest:
//                       the FP64 sum of the slice's day costs; four days walk
//                       the path together (the link index and length are
//                       loaded once, four speed loads are in flight);
//   k_cost_mean         one thread per (path, t): the slice sums in slice
//                       order, divided by the day count.
#include "dode_internal.h"

#include <algorithm>

namespace {

constexpr int kBlock = 256;
constexpr int kTrajDays = 8;   // days walked together by one trajectory thread

template <typename S>
__device__ __forceinline__ S link_time(const S* __restrict__ len, const S* __restrict__ speed_day,
                                       int32_t H_speed, S dt, int32_t a, S t) {
  int64_t h = static_cast<int64_t>(floor(t / dt));
  h = h < 0 ? 0 : (h >= H_speed ? H_speed - 1 : h);
  return len[a] / speed_day[(int64_t)a * H_speed + h];
}

// One thread per (group of eight days, path, boundary b), b fastest: the
// eight days' trajectories are walked together, so eight independent chains
// of speed gathers are in flight (days past the chunk repeat its last day and
// are not stored).
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_trajectories(int32_t n_paths, const int32_t* __restrict__ path_ptr,
               const int32_t* __restrict__ path_link, int32_t L, const S* __restrict__ len,
               const S* __restrict__ speed, int32_t day0, int32_t n_days, int32_t H_speed, S dt,
               int32_t H, int64_t n_pairs, S* __restrict__ traj, S* __restrict__ exit_time) {
  // The entry time t0 + r is a sum of its own, never fused with the product
  // b * dt: which interval's speed a link takes is decided by the rounded sum.
#pragma clang fp contract(off)
  constexpr int kDays = kTrajDays;
  const int64_t per_group = (int64_t)n_paths * (H + 1);
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int32_t n_groups = (n_days + kDays - 1) / kDays;
  if (idx >= per_group * n_groups) return;
  const int32_t dg = (int32_t)(idx / per_group);
  const int64_t kb = idx % per_group;   // k * (H+1) + b
  const int32_t k = (int32_t)(kb / (H + 1));
  const int32_t b = (int32_t)(kb % (H + 1));
  const int64_t day_stride = (int64_t)L * H_speed, traj_stride = n_pairs * (H + 1);
  const S* sp[kDays];
  S* out[kDays];
  bool on[kDays];
#pragma unroll
  for (int u = 0; u < kDays; ++u) {
    const int32_t d = min(dg * kDays + u, n_days - 1);
    on[u] = dg * kDays + u < n_days;
    sp[u] = speed + (int64_t)(day0 + d) * day_stride;
    out[u] = traj + (int64_t)d * traj_stride;
  }
  const S t0 = static_cast<S>(b) * dt;
  S r[kDays];   // travel time so far
#pragma unroll
  for (int u = 0; u < kDays; ++u) r[u] = S(0);
  for (int32_t m = path_ptr[k]; m < path_ptr[k + 1]; ++m) {
    const int32_t a = path_link[m];
#pragma unroll
    for (int u = 0; u < kDays; ++u) {
      if (on[u]) out[u][(int64_t)m * (H + 1) + b] = r[u];
      r[u] += link_time(len, sp[u], H_speed, dt, a, t0 + r[u]);
    }
  }
  if (exit_time)   // [d][k][b]: the whole path's travel time
#pragma unroll
    for (int u = 0; u < kDays; ++u)
      if (on[u]) exit_time[(int64_t)(dg * kDays + u) * per_group + kb] = r[u];
}

// Running FP64 sums of the chunk's path travel times, days in order, for the
// departures at the interval starts (boundaries b < H); the last chunk writes
// cost[t][k] = sum / n_days.
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_exit_sums(int32_t n_paths, int32_t H, int32_t n_days_chunk, const S* __restrict__ exit_time,
            bool first_chunk, bool last_chunk, int32_t n_days_total, double* __restrict__ sums,
            S* __restrict__ cost) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (int64_t)n_paths * H) return;
  const int32_t k = (int32_t)(idx / H), t = (int32_t)(idx % H);
  const int64_t per_day = (int64_t)n_paths * (H + 1);
  const S* e = exit_time + (int64_t)k * (H + 1) + t;
  double s = first_chunk ? 0.0 : sums[idx];
  for (int32_t d = 0; d < n_days_chunk; ++d) s += static_cast<double>(e[d * per_day]);
  if (last_chunk)
    cost[(int64_t)t * n_paths + k] = static_cast<S>(s / n_days_total);
  else
    sums[idx] = s;
}

// 1 / w for the window shares: the hardware reciprocal in FP32 (within 1 ulp;
// the kernel is bound by its instruction count), the quotient in FP64.
__device__ __forceinline__ float share_recip(float w) { return __builtin_amdgcn_rcpf(w); }
__device__ __forceinline__ double share_recip(double w) { return 1.0 / w; }
// min(max(x, 0), 1): one v_med3 in FP32
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }
__device__ __forceinline__ double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

template <typename S, int KMAX>
__global__ void __launch_bounds__(kBlock)
k_dar_windows(int64_t n_pairs, int32_t n_days_chunk, int32_t H, int32_t K, S dt,
              const S* __restrict__ traj, bool first_chunk, bool last_chunk, int32_t n_days_total,
              S* __restrict__ Rr) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n_pairs * H) return;
  const int64_t m = idx / H;
  const int32_t h = (int32_t)(idx % H);
  const int kk = min(K, H - h);   // lags that stay inside the day
  S acc[KMAX];
#pragma unroll
  for (int l = 0; l < KMAX; ++l) acc[l] = first_chunk || l >= K ? S(0) : Rr[((int64_t)l * H + h) * n_pairs + m];
  const int64_t day_stride = n_pairs * (H + 1);
  const S* tr = traj + m * (H + 1) + h;
  // interval h+l ends at (l+1)*dt relative to the departure
  S edge[KMAX];
#pragma unroll
  for (int l = 0; l < KMAX; ++l) edge[l] = static_cast<S>(l + 1) * dt;
  // One day's window [lo, hi] (relative to h*dt; observation interval h+l is
  // [l*dt, (l+1)*dt)) added into acc.  Every lag is accumulated; lags past the
  // day (l >= kk) are written as zeros below.
  auto add_day = [&](S lo, S hi) {
    // FIFO violation (hi < lo): the window between the two end points
    const S a0 = fmin(lo, hi), w = fmax(lo, hi) - a0;
    if (w <= S(0)) {   // all of the interval arrives at one instant
      const int la = static_cast<int>(fmin(floor(a0 / dt), static_cast<S>(KMAX)));
#pragma unroll
      for (int ll = 0; ll < KMAX; ++ll)
        if (ll == la) acc[ll] += S(1);
      return;
    }
    const S inv_w = share_recip(w);
    S f_prev = S(0);   // F(0) = 0: windows start at or after their departure
#pragma unroll
    for (int ll = 0; ll < KMAX; ++ll) {
      const S f = clamp01((edge[ll] - a0) * inv_w);
      acc[ll] += f - f_prev;
      f_prev = f;
    }
  };
  // days in order: groups of eight whose loads are in flight together, then
  // the rest one by one
  constexpr int kDays = 8;
  const S* p = tr;
  int32_t d = 0;
  for (; d + kDays <= n_days_chunk; d += kDays, p += kDays * day_stride) {
    S lo[kDays], hi[kDays];
#pragma unroll
    for (int u = 0; u < kDays; ++u) {
      lo[u] = p[u * day_stride];
      hi[u] = dt + p[u * day_stride + 1];
    }
#pragma unroll
    for (int u = 0; u < kDays; ++u) add_day(lo[u], hi[u]);
  }
  for (; d < n_days_chunk; ++d, p += day_stride) add_day(p[0], dt + p[1]);
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l >= K) break;
    const S v = l >= kk ? S(0) : (last_chunk ? acc[l] / static_cast<S>(n_days_total) : acc[l]);
    Rr[((int64_t)l * H + h) * n_pairs + m] = v;
  }
}

template <typename S>
__global__ void __launch_bounds__(kBlock)
k_path_cost_slices(int32_t n_paths, const int32_t* __restrict__ path_ptr,
                   const int32_t* __restrict__ path_link, int32_t L, const S* __restrict__ len,
                   const S* __restrict__ speed, int32_t n_days, int32_t per_slice, int32_t n_slices,
                   int32_t H_speed, S dt, int32_t T, double* __restrict__ partial) {
#pragma clang fp contract(off)   // as in k_trajectories
  const int64_t per = (int64_t)n_paths * T;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= per * n_slices) return;
  const int32_t g = (int32_t)(idx / per);
  const int32_t k = (int32_t)((idx % per) / T);
  const int32_t t = (int32_t)(idx % T);
  const S t0 = static_cast<S>(t) * dt;
  const int32_t m0 = path_ptr[k], m1 = path_ptr[k + 1];
  const int32_t d_begin = g * per_slice, d_end = min(n_days, d_begin + per_slice);
  constexpr int kDays = 4;
  const int64_t day_stride = (int64_t)L * H_speed;
  double sum = 0.0;
  for (int32_t d0 = d_begin; d0 < d_end; d0 += kDays) {
    const S* sp[kDays];
    S r[kDays];
#pragma unroll
    for (int u = 0; u < kDays; ++u) {
      sp[u] = speed + (int64_t)min(d0 + u, d_end - 1) * day_stride;
      r[u] = S(0);
    }
    for (int32_t m = m0; m < m1; ++m) {
      const int32_t a = path_link[m];
#pragma unroll
      for (int u = 0; u < kDays; ++u) r[u] += link_time(len, sp[u], H_speed, dt, a, t0 + r[u]);
    }
#pragma unroll
    for (int u = 0; u < kDays; ++u)
      if (d0 + u < d_end) sum += static_cast<double>(r[u]);
  }
  partial[idx] = sum;
}

template <typename S>
__global__ void __launch_bounds__(kBlock)
k_cost_mean(int32_t n_paths, int32_t T, int32_t n_slices, int32_t n_days,
            const double* __restrict__ partial, S* __restrict__ cost) {
  const int64_t per = (int64_t)n_paths * T;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= per) return;
  const int32_t k = (int32_t)(idx / T), t = (int32_t)(idx % T);
  double s = 0.0;
  for (int32_t g = 0; g < n_slices; ++g) s += partial[g * per + idx];
  cost[(int64_t)t * n_paths + k] = static_cast<S>(s / n_days);
}

template <typename S>
__global__ void k_check_speeds(const S* __restrict__ x, int64_t n, int32_t* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!(x[i] > S(0)) || !isfinite(x[i])) *flag = 1;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename S>
hipError_t run(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link, int64_t n_pairs,
               int32_t L, const S* len, const S* speed, int32_t n_days, int32_t H_speed, S dt,
               int32_t H, int32_t K, S* traj, int32_t chunk, S* Rr, S* exit_time, double* sums,
               S* cost, hipStream_t s) {
  for (int32_t d0 = 0; d0 < n_days; d0 += chunk) {
    const int32_t nd = std::min(chunk, n_days - d0);
    const int64_t n1 = (int64_t)((nd + kTrajDays - 1) / kTrajDays) * n_paths * (H + 1);
    hipLaunchKernelGGL(k_trajectories<S>, dim3(blocks_for(n1)), dim3(kBlock), 0, s, n_paths,
                       path_ptr, path_link, L, len, speed, d0, nd, H_speed, dt, H, n_pairs, traj,
                       cost ? exit_time : nullptr);
    const bool first = d0 == 0, last = d0 + nd >= n_days;
    if (cost)
      hipLaunchKernelGGL(k_exit_sums<S>, dim3(blocks_for((int64_t)n_paths * H)), dim3(kBlock), 0, s,
                         n_paths, H, nd, exit_time, first, last, n_days, sums, cost);
    // the window loop is unrolled to KMAX lags: the common K = 6 gets its own
    if (K <= 6)
      hipLaunchKernelGGL((k_dar_windows<S, 6>), dim3(blocks_for(n_pairs * H)), dim3(kBlock), 0, s,
                         n_pairs, nd, H, K, dt, traj, first, last, n_days, Rr);
    else if (K <= 8)
      hipLaunchKernelGGL((k_dar_windows<S, 8>), dim3(blocks_for(n_pairs * H)), dim3(kBlock), 0, s,
                         n_pairs, nd, H, K, dt, traj, first, last, n_days, Rr);
    else
      hipLaunchKernelGGL((k_dar_windows<S, kMaxDarLags>), dim3(blocks_for(n_pairs * H)),
                         dim3(kBlock), 0, s, n_pairs, nd, H, K, dt, traj, first, last, n_days, Rr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename S>
hipError_t run_costs(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link, int32_t L,
                     const S* len, const S* speed, int32_t n_days, int32_t H_speed, S dt, int32_t T,
                     int32_t per_slice, double* partial, S* cost, hipStream_t s) {
  const int32_t n_slices = (n_days + per_slice - 1) / per_slice;
  const int64_t per = (int64_t)n_paths * T;
  hipLaunchKernelGGL(k_path_cost_slices<S>, dim3(blocks_for(per * n_slices)), dim3(kBlock), 0, s,
                     n_paths, path_ptr, path_link, L, len, speed, n_days, per_slice, n_slices,
                     H_speed, dt, T, partial);
  hipLaunchKernelGGL(k_cost_mean<S>, dim3(blocks_for(per)), dim3(kBlock), 0, s, n_paths, T,
                     n_slices, n_days, partial, cost);
  return hipGetLastError();
}

}  // namespace

hipError_t path_costs(bool f64, int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                      int32_t L, const void* len, const void* speed, int32_t n_days, int32_t H_speed,
                      double dt, int32_t T, int32_t per_slice, double* partial, void* cost,
                      hipStream_t s) {
  if (f64)
    return run_costs<double>(n_paths, path_ptr, path_link, L, static_cast<const double*>(len),
                             static_cast<const double*>(speed), n_days, H_speed, dt, T, per_slice,
                             partial, static_cast<double*>(cost), s);
  return run_costs<float>(n_paths, path_ptr, path_link, L, static_cast<const float*>(len),
                          static_cast<const float*>(speed), n_days, H_speed, static_cast<float>(dt),
                          T, per_slice, partial, static_cast<float*>(cost), s);
}

hipError_t dar_check_speeds(bool f64, const void* speed, int64_t n, int32_t* flag, hipStream_t s) {
  const unsigned b = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, blocks_for(n)));
  if (f64)
    hipLaunchKernelGGL(k_check_speeds<double>, dim3(b), dim3(kBlock), 0, s,
                       static_cast<const double*>(speed), n, flag);
  else
    hipLaunchKernelGGL(k_check_speeds<float>, dim3(b), dim3(kBlock), 0, s,
                       static_cast<const float*>(speed), n, flag);
  return hipGetLastError();
}

hipError_t dar_from_speeds(bool f64, int32_t n_paths, const int32_t* path_ptr,
                           const int32_t* path_link, int64_t n_pairs, int32_t L, const void* len,
                           const void* speed, int32_t n_days, int32_t H_speed, double dt, int32_t H,
                           int32_t K, void* traj, int32_t chunk, void* Rr, void* exit_time,
                           double* sums, void* cost, hipStream_t s) {
  if (f64)
    return run<double>(n_paths, path_ptr, path_link, n_pairs, L, static_cast<const double*>(len),
                       static_cast<const double*>(speed), n_days, H_speed, dt, H, K,
                       static_cast<double*>(traj), chunk, static_cast<double*>(Rr),
                       static_cast<double*>(exit_time), sums, static_cast<double*>(cost), s);
  return run<float>(n_paths, path_ptr, path_link, n_pairs, L, static_cast<const float*>(len),
                    static_cast<const float*>(speed), n_days, H_speed, static_cast<float>(dt), H, K,
                    static_cast<float*>(traj), chunk, static_cast<float*>(Rr),
                    static_cast<float*>(exit_time), sums, static_cast<float*>(cost), s);
}
