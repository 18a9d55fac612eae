// BLAS-1 kernels of the Krylov solver: dot products and norms with
// deterministic two-stage reductions (a fixed grid of blocks, a fixed
// wavefront butterfly, then a fixed-order sum of the block partials), the
// multi-vector products of classical Gram-Schmidt, and vector updates.
// HBM-bound: every kernel streams its vectors once with 16-byte loads.
#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kRedThreads = 256;
constexpr int kChunk = 8;  // vectors per multi-dot block row

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum in a fixed order: butterfly inside each 64-lane wavefront, then
// wavefront 0 adds the 4 wavefront sums in order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kRedThreads / 64; ++w) t += sh[w];
  }
  return t;
}

// partials[(c*kChunk + j) * nb + b] = sum over the block's indices of V_j[i] w[i]
__global__ void __launch_bounds__(kRedThreads)
    k_multidot(const double* __restrict__ V, long long ld, int k, const double* __restrict__ w,
               long long n, double* __restrict__ partials) {
  __shared__ double sh[kRedThreads / 64];
  const int c = blockIdx.y;
  const int nb = gridDim.x;
  double acc[kChunk];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) acc[j] = 0.0;
  const int j0 = c * kChunk;
  const long long n2 = n / 2;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
       i += (long long)nb * kRedThreads) {
    const double2 wi = w2[i];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      if (j0 + j < k) {
        const double2 vi = reinterpret_cast<const double2*>(V + (long long)(j0 + j) * ld)[i];
        acc[j] = fma(vi.x, wi.x, acc[j]);
        acc[j] = fma(vi.y, wi.y, acc[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    if (j0 + j < k) {
      const double t = block_sum(acc[j], sh);
      if (threadIdx.x == 0) partials[(long long)(j0 + j) * nb + blockIdx.x] = t;
    }
  }
}

// out[j] = scale * sum_b partials[j * nparts + b], fixed order per thread then
// fixed block butterfly; one block per j.
__global__ void __launch_bounds__(kRedThreads)
    k_reduce(const double* __restrict__ partials, int nparts, double* __restrict__ out,
             double scale) {
  __shared__ double sh[kRedThreads / 64];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kRedThreads) acc += partials[(long long)j * nparts + b];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = scale * t;
}

// x[i] += sum_j coef[j] * V_j[i]  (runtime k, coefficients on the device)
__global__ void __launch_bounds__(256)
    k_combine(const double* __restrict__ V, long long ld, int k, const double* __restrict__ coef,
              double* __restrict__ x, long long n) {
  const long long n2 = n / 2;
  double2* x2 = reinterpret_cast<double2*>(x);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    double2 a = x2[i];
    for (int j = 0; j < k; ++j) {
      const double c = coef[j];
      const double2 v = reinterpret_cast<const double2*>(V + (long long)j * ld)[i];
      a.x = fma(c, v.x, a.x);
      a.y = fma(c, v.y, a.y);
    }
    x2[i] = a;
  }
}

// w[i] -= sum_j coef[j] V_j[i]; partials of |w_new|^2 when want_norm
__global__ void __launch_bounds__(kRedThreads)
    k_axpy_norm(const double* __restrict__ V, long long ld, int k, const double* __restrict__ coef,
                double* __restrict__ w, long long n, double* __restrict__ partials, int want_norm) {
  __shared__ double sh[kRedThreads / 64];
  const long long n2 = n / 2;
  double2* w2 = reinterpret_cast<double2*>(w);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
       i += (long long)gridDim.x * kRedThreads) {
    double2 a = w2[i];
    for (int j = 0; j < k; ++j) {
      const double c = coef[j];
      const double2 v = reinterpret_cast<const double2*>(V + (long long)j * ld)[i];
      a.x = fma(-c, v.x, a.x);
      a.y = fma(-c, v.y, a.y);
    }
    w2[i] = a;
    acc = fma(a.x, a.x, acc);
    acc = fma(a.y, a.y, acc);
  }
  if (want_norm) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// w <- w - sum_j coef[j] V_j (j < k) and, in the same sweep, the partials of
// V_j . w_new (rows j < k) and of |w_new|^2 (row k): exactly the products the
// second Gram-Schmidt projection needs, so that pass does not read V again.
// KMAX bounds k at compile time so the accumulators stay in registers.
template <int KMAX>
__global__ void __launch_bounds__(kRedThreads)
    k_axpy_multidot(const double* __restrict__ V, long long ld, int k,
                    const double* __restrict__ coef, double* __restrict__ w, long long n,
                    double* __restrict__ partials) {
  __shared__ double sh[kRedThreads / 64];
  const int nb = gridDim.x;
  const long long n2 = n / 2;
  double2* w2 = reinterpret_cast<double2*>(w);
  double acc[KMAX + 1];
#pragma unroll
  for (int j = 0; j <= KMAX; ++j) acc[j] = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
       i += (long long)nb * kRedThreads) {
    double2 a = w2[i];
    double2 v[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        v[j] = reinterpret_cast<const double2*>(V + (long long)j * ld)[i];
        const double c = coef[j];
        a.x = fma(-c, v[j].x, a.x);
        a.y = fma(-c, v[j].y, a.y);
      }
    }
    w2[i] = a;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        acc[j] = fma(v[j].x, a.x, acc[j]);
        acc[j] = fma(v[j].y, a.y, acc[j]);
      }
    }
    acc[KMAX] = fma(a.x, a.x, acc[KMAX]);
    acc[KMAX] = fma(a.y, a.y, acc[KMAX]);
  }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      const double t = block_sum(acc[j], sh);
      if (threadIdx.x == 0) partials[(long long)j * nb + blockIdx.x] = t;
    }
  }
  const double t = block_sum(acc[KMAX], sh);
  if (threadIdx.x == 0) partials[(long long)k * nb + blockIdx.x] = t;
}

// w <- scale * (w - sum_j coef[j] V_j)
__global__ void __launch_bounds__(256)
    k_axpy_scale(const double* __restrict__ V, long long ld, int k,
                 const double* __restrict__ coef, double scale, double* __restrict__ w,
                 long long n) {
  const long long n2 = n / 2;
  double2* w2 = reinterpret_cast<double2*>(w);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    double2 a = w2[i];
    for (int j = 0; j < k; ++j) {
      const double c = coef[j];
      const double2 v = reinterpret_cast<const double2*>(V + (long long)j * ld)[i];
      a.x = fma(-c, v.x, a.x);
      a.y = fma(-c, v.y, a.y);
    }
    w2[i] = make_double2(scale * a.x, scale * a.y);
  }
}

// y = x * alpha (invert = 0) or x / alpha (invert = 1), alpha on the device
__global__ void __launch_bounds__(256)
    k_scale(const double* __restrict__ x, const double* __restrict__ alpha, int invert,
            double* __restrict__ y, long long n) {
  const double a = invert ? 1.0 / *alpha : *alpha;
  const long long n2 = n / 2;
  const double2* x2 = reinterpret_cast<const double2*>(x);
  double2* y2 = reinterpret_cast<double2*>(y);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 v = x2[i];
    y2[i] = make_double2(a * v.x, a * v.y);
  }
}

__global__ void __launch_bounds__(256)
    k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
            double* __restrict__ z, long long n) {
  const long long n2 = n / 2;
  const double2* x2 = reinterpret_cast<const double2*>(x);
  const double2* y2 = reinterpret_cast<const double2*>(y);
  double2* z2 = reinterpret_cast<double2*>(z);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 u = x2[i], v = y2[i];
    z2[i] = make_double2(fma(a, u.x, b * v.x), fma(a, u.y, b * v.y));
  }
}

// eps = sqrt(2^-52) (1 + sqrt(uu)) / sqrt(vv), 0 when v = 0
__global__ void k_fd_eps(const double* __restrict__ uu, const double* __restrict__ vv,
                         double* __restrict__ eps) {
  const double nu = sqrt(uu[0]), nv = sqrt(vv[0]);
  eps[0] = (nv > 0.0) ? 1.4901161193847656e-08 * (1.0 + nu) / nv : 0.0;
}

__global__ void k_sub_scalars(double* acc, const double* x, int k) {
  const int j = threadIdx.x;
  if (j < k) acc[j] -= x[j];
}

unsigned grid_for(long long n2, int threads, unsigned cap) {
  long long b = (n2 + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

int blas_multidot(pf_problem* pb, const double* V, long long ld, int k, const double* w,
                  long long n, double* out_dev, hipStream_t s) {
  if (k <= 0) return PF_OK;
  const int nb = pb->n_red_blocks;
  const int chunks = (k + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_multidot, dim3(nb, chunks), dim3(kRedThreads), 0, s, V, ld, k, w, n,
                     pb->red_partials);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, s, pb->red_partials, nb, out_dev, 1.0);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_dot(pf_problem* pb, const double* x, const double* y, long long n, double* out_dev,
             hipStream_t s) {
  return blas_multidot(pb, x, n, 1, y, n, out_dev, s);
}

int blas_axpy_dot(pf_problem* pb, const double* V, long long ld, int k, const double* coef_dev,
                  double* w, long long n, double* dots_dev, int want_norm, hipStream_t s) {
  const int nb = pb->n_red_blocks;
  hipLaunchKernelGGL(k_axpy_norm, dim3(nb), dim3(kRedThreads), 0, s, V, ld, k, coef_dev, w, n,
                     pb->red_partials, want_norm);
  PF_HIP_CHECK(hipGetLastError());
  if (want_norm) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, pb->red_partials, nb, dots_dev,
                       1.0);
    PF_HIP_CHECK(hipGetLastError());
  }
  return PF_OK;
}

int blas_axpy_multidot(pf_problem* pb, const double* V, long long ld, int k,
                       const double* coef_dev, double* w, long long n, double* out_dev,
                       hipStream_t s) {
  if (k < 1 || k > kAxpyMultidotMax) return PF_ERR_INVALID_ARG;
  const int nb = pb->n_red_blocks;
  if (k <= 8)
    hipLaunchKernelGGL(k_axpy_multidot<8>, dim3(nb), dim3(kRedThreads), 0, s, V, ld, k, coef_dev,
                       w, n, pb->red_partials);
  else if (k <= 16)
    hipLaunchKernelGGL(k_axpy_multidot<16>, dim3(nb), dim3(kRedThreads), 0, s, V, ld, k,
                       coef_dev, w, n, pb->red_partials);
  else
    hipLaunchKernelGGL(k_axpy_multidot<32>, dim3(nb), dim3(kRedThreads), 0, s, V, ld, k,
                       coef_dev, w, n, pb->red_partials);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(k + 1), dim3(kRedThreads), 0, s, pb->red_partials, nb,
                     out_dev, 1.0);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_axpy_scale(const double* V, long long ld, int k, const double* coef_dev, double scale,
                    double* w, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_scale, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, V, ld, k,
                     coef_dev, scale, w, n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_combine(pf_problem* pb, const double* V, long long ld, int k, const double* coef_dev,
                 double* x, long long n, hipStream_t s) {
  (void)pb;
  if (k <= 0) return PF_OK;
  hipLaunchKernelGGL(k_combine, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, V, ld, k,
                     coef_dev, x, n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_scale_copy(const double* x, const double* alpha_dev, int invert, double* y, long long n,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, x, alpha_dev,
                     invert, y, n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_axpby(double a, const double* x, double b, const double* y, double* z, long long n,
               hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, a, x, b, y, z, n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_fd_eps(pf_problem* pb, const double* U, const double* v, long long n, double* eps_dev,
                hipStream_t s) {
  double* nrm = pb->red_out + 200;
  PF_TRY(blas_multidot(pb, U, n, 1, U, n, nrm, s));
  PF_TRY(blas_multidot(pb, v, n, 1, v, n, nrm + 1, s));
  hipLaunchKernelGGL(k_fd_eps, dim3(1), dim3(1), 0, s, nrm, nrm + 1, eps_dev);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_fd_eps_cached(pf_problem* pb, const double* unorm2_dev, const double* v, long long n,
                       double* eps_dev, hipStream_t s) {
  double* nv = pb->red_out + 201;
  PF_TRY(blas_multidot(pb, v, n, 1, v, n, nv, s));
  hipLaunchKernelGGL(k_fd_eps, dim3(1), dim3(1), 0, s, unorm2_dev, nv, eps_dev);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_reduce_partials(const double* partials, int nparts, int k, double* out_dev, double scale,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, s, partials, nparts, out_dev, scale);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_sub_scalars(double* acc_dev, const double* x_dev, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_scalars, dim3(1), dim3(64), 0, s, acc_dev, x_dev, k);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace pf
