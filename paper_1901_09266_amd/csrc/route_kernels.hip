// Route-choice kernels: the assignment matrix from route portions (eqs.
// "logit", "rt", "flow", "assign"), with portions from free logits per path or
// from the mean path costs of a pattern, and the loss gradient with respect to
// the assignment values and the free logits.  One thread or block per output
// entry, fixed summation order, FP64 accumulation for the reductions.
#include "dode_internal.h"

#include <cmath>

namespace {

constexpr int kBlock = 256;

__device__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per row t < n_rows and OD p: pi[t][k] = exp(a z[t][k] - max) / sum over the
// paths of OD p (FP64); one thread per (t, p).  z rows are zs apart (zs = 0
// repeats one row); a = 1 for free logits, -theta for costs.  When pi_out is
// set the portions are also written there in the storage type.
template <typename S>
__global__ void k_softmax(DevRoutes r, int32_t n_rows, const S* __restrict__ z, int64_t zs,
                          double a, double* __restrict__ pi, S* __restrict__ pi_out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_rows * r.P) return;
  const int32_t t = (int32_t)(idx / r.P), p = (int32_t)(idx % r.P);
  const S* zt = z + t * zs;
  double* pt = pi + (int64_t)t * r.n_paths;
  const int k0 = r.od_ptr[p], k1 = r.od_ptr[p + 1];
  double zmax = -INFINITY;
  for (int i = k0; i < k1; ++i) zmax = fmax(zmax, a * static_cast<double>(zt[r.od_paths[i]]));
  double s = 0.0;
  for (int i = k0; i < k1; ++i) s += exp(a * static_cast<double>(zt[r.od_paths[i]]) - zmax);
  for (int i = k0; i < k1; ++i) {
    const int k = r.od_paths[i];
    const double v = exp(a * static_cast<double>(zt[k]) - zmax) / s;
    pt[k] = v;
    if (pi_out) pi_out[(int64_t)t * r.n_paths + k] = static_cast<S>(v);
  }
}

// W[l][t][nz] = sum over pairs m feeding nz of Rr[l][t][m] * pi[t][path(m)]
// (eq. "assign"); pi rows are ps apart (ps = 0: portions that do not depend
// on the interval).  Pairs are summed in increasing order.
template <typename S>
__global__ void k_rho_from_pi(DevRoutes r, const S* __restrict__ Rr, const double* __restrict__ pi,
                              int64_t ps, S* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)r.K * r.T * r.nnz;
  if (idx >= total) return;
  const int64_t lt = idx / r.nnz, nz = idx % r.nnz;
  const double* pt = pi + (lt % r.T) * ps;
  double s = 0.0;
  for (int i = r.nz_ptr[nz]; i < r.nz_ptr[nz + 1]; ++i) {
    const int m = r.nz_pairs[i];
    s += static_cast<double>(Rr[lt * r.n_pairs + m]) * pt[r.pair_path[m]];
  }
  W[idx] = static_cast<S>(s);
}

// dpi_k = sum_{lt, pairs m of k} Rr[lt][m] dW[lt][pair_nz[m]]; one block per path.
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_dpi(DevRoutes r, const S* __restrict__ Rr, const S* __restrict__ dW, double* __restrict__ dpi) {
  __shared__ double sh[kBlock];
  const int k = blockIdx.x;
  const int m0 = r.pair_ptr[k], m1 = r.pair_ptr[k + 1];
  const int64_t per = m1 - m0;
  const int64_t total = (int64_t)r.K * r.T * per;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += kBlock) {
    const int64_t lt = i / per;
    const int m = m0 + (int)(i % per);
    s += static_cast<double>(Rr[lt * r.n_pairs + m]) * static_cast<double>(dW[lt * r.nnz + r.pair_nz[m]]);
  }
  const double tot = block_sum256(s, sh);
  if (threadIdx.x == 0) dpi[k] = tot;
}

// dz_k = pi_k (dpi_k - sum_{k' serving od(k)} pi_k' dpi_k'); one thread per path.
template <typename S>
__global__ void k_dz(DevRoutes r, const double* __restrict__ pi, const double* __restrict__ dpi,
                     S* __restrict__ dz) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.n_paths) return;
  const int p = r.path_od[k];
  double s = 0.0;
  for (int i = r.od_ptr[p]; i < r.od_ptr[p + 1]; ++i) {
    const int k2 = r.od_paths[i];
    s += pi[k2] * dpi[k2];
  }
  dz[k] = static_cast<S>(pi[k] * (dpi[k] - s));
}

// dW[l][t][nz(a,p)] = scale * sum_d R[d][t+l][a] Q[d][t][p]   (0 where t+l >= H).
template <typename S>
__global__ void k_dW(DevPat pt, const int32_t* __restrict__ row_of_nz, const S* __restrict__ R,
                     const S* __restrict__ Q, int32_t n_days, double scale, S* __restrict__ dW) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)pt.K * pt.T * pt.nnz;
  if (idx >= total) return;
  const int64_t lt = idx / pt.nnz, nz = idx % pt.nnz;
  const int l = (int)(lt / pt.T), t = (int)(lt % pt.T);
  double s = 0.0;
  if (t + l < pt.H) {
    const int a = row_of_nz[nz], p = pt.col[nz];
    for (int d = 0; d < n_days; ++d)
      s += static_cast<double>(R[((int64_t)d * pt.H + t + l) * pt.L + a]) *
           static_cast<double>(Q[((int64_t)d * pt.T + t) * pt.P + p]);
  }
  dW[idx] = static_cast<S>(scale * s);
}

template <typename S>
__global__ void k_scale(S* __restrict__ x, int64_t n, double f) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = static_cast<S>(static_cast<double>(x[i]) * f);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename S>
void launch_rho(const DevRoutes& r, int32_t n_rows, const S* Rr, const S* z, int64_t zs, double a,
                double* pi, S* pi_out, S* W, hipStream_t s) {
  const int64_t total = (int64_t)r.K * r.T * r.nnz;
  hipLaunchKernelGGL(k_softmax<S>, dim3(blocks_for((int64_t)n_rows * r.P)), dim3(kBlock), 0, s, r,
                     n_rows, z, zs, a, pi, pi_out);
  hipLaunchKernelGGL(k_rho_from_pi<S>, dim3(blocks_for(total)), dim3(kBlock), 0, s, r, Rr, pi,
                     n_rows > 1 ? (int64_t)r.n_paths : 0, W);
}

}  // namespace

hipError_t routes_rho(const DevRoutes& r, bool f64, const void* Rr, const void* z, void* W,
                      double* pi, hipStream_t s) {
  if (f64)
    launch_rho<double>(r, 1, static_cast<const double*>(Rr), static_cast<const double*>(z), 0, 1.0,
                       pi, nullptr, static_cast<double*>(W), s);
  else
    launch_rho<float>(r, 1, static_cast<const float*>(Rr), static_cast<const float*>(z), 0, 1.0, pi,
                      nullptr, static_cast<float*>(W), s);
  return hipGetLastError();
}

hipError_t routes_rho_costs(const DevRoutes& r, bool f64, const void* Rr, const void* cost,
                            double theta, void* portions, void* W, double* pi, hipStream_t s) {
  if (f64)
    launch_rho<double>(r, r.T, static_cast<const double*>(Rr), static_cast<const double*>(cost),
                       r.n_paths, -theta, pi, static_cast<double*>(portions),
                       static_cast<double*>(W), s);
  else
    launch_rho<float>(r, r.T, static_cast<const float*>(Rr), static_cast<const float*>(cost),
                      r.n_paths, -theta, pi, static_cast<float*>(portions), static_cast<float*>(W),
                      s);
  return hipGetLastError();
}

hipError_t routes_logits_bwd(const DevRoutes& r, bool f64, const void* Rr, const void* z,
                             const void* dW, void* dz, double* pi, double* dpi, hipStream_t s) {
  if (f64) {
    hipLaunchKernelGGL(k_softmax<double>, dim3(blocks_for(r.P)), dim3(kBlock), 0, s, r, 1,
                       static_cast<const double*>(z), (int64_t)0, 1.0, pi, (double*)nullptr);
    hipLaunchKernelGGL(k_dpi<double>, dim3(r.n_paths), dim3(kBlock), 0, s, r,
                       static_cast<const double*>(Rr), static_cast<const double*>(dW), dpi);
    hipLaunchKernelGGL(k_dz<double>, dim3(blocks_for(r.n_paths)), dim3(kBlock), 0, s, r, pi, dpi,
                       static_cast<double*>(dz));
  } else {
    hipLaunchKernelGGL(k_softmax<float>, dim3(blocks_for(r.P)), dim3(kBlock), 0, s, r, 1,
                       static_cast<const float*>(z), (int64_t)0, 1.0, pi, (float*)nullptr);
    hipLaunchKernelGGL(k_dpi<float>, dim3(r.n_paths), dim3(kBlock), 0, s, r,
                       static_cast<const float*>(Rr), static_cast<const float*>(dW), dpi);
    hipLaunchKernelGGL(k_dz<float>, dim3(blocks_for(r.n_paths)), dim3(kBlock), 0, s, r, pi, dpi,
                       static_cast<float*>(dz));
  }
  return hipGetLastError();
}

hipError_t loss_bwd_dW(const dode_dar* dar, const void* R, const void* Q, int32_t n_days,
                       double scale, void* dW, hipStream_t s) {
  const int64_t total = (int64_t)dar->dims.K * dar->dims.T * dar->nnz;
  if (dar->storage == DODE_F64)
    hipLaunchKernelGGL(k_dW<double>, dim3(blocks_for(total)), dim3(kBlock), 0, s, dar->pat(),
                       dar->d_row_of_nz, static_cast<const double*>(R),
                       static_cast<const double*>(Q), n_days, scale, static_cast<double*>(dW));
  else
    hipLaunchKernelGGL(k_dW<float>, dim3(blocks_for(total)), dim3(kBlock), 0, s, dar->pat(),
                       dar->d_row_of_nz, static_cast<const float*>(R), static_cast<const float*>(Q),
                       n_days, scale, static_cast<float*>(dW));
  return hipGetLastError();
}

hipError_t scale_state(bool f64, void* x, int64_t n, double f, hipStream_t s) {
  const unsigned b = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, blocks_for(n)));
  if (f64)
    hipLaunchKernelGGL(k_scale<double>, dim3(b), dim3(kBlock), 0, s, static_cast<double*>(x), n, f);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(b), dim3(kBlock), 0, s, static_cast<float*>(x), n, f);
  return hipGetLastError();
}
