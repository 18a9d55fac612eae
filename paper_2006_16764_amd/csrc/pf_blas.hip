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
  if (k == 1 && V == w) {
    // a squared norm: one load per entry instead of two of the same address
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
         i += (long long)nb * kRedThreads) {
      const double2 wi = w2[i];
      acc[0] = fma(wi.x, wi.x, acc[0]);
      acc[0] = fma(wi.y, wi.y, acc[0]);
    }
  } else {
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
  }
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    if (j0 + j < k) {
      const double t = block_sum(acc[j], sh);
      if (threadIdx.x == 0) partials[(long long)(j0 + j) * nb + blockIdx.x] = t;
    }
  }
}

// z = a x + b y as k_axpby, and the partials of |z|^2 in the squared-norm
// order of k_multidot (same grid, same per-thread and block sums): with
// k_reduce, the same |z|^2 as a multi-dot of z with itself.
__global__ void __launch_bounds__(kRedThreads)
    k_axpby_norm(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                 double* __restrict__ z, long long n, double* __restrict__ partials) {
  __shared__ double sh[kRedThreads / 64];
  const int nb = gridDim.x;
  const long long n2 = n / 2;
  const double2* x2 = reinterpret_cast<const double2*>(x);
  const double2* y2 = reinterpret_cast<const double2*>(y);
  double2* z2 = reinterpret_cast<double2*>(z);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
       i += (long long)nb * kRedThreads) {
    const double2 u = x2[i], v = y2[i];
    const double2 w = make_double2(fma(a, u.x, b * v.x), fma(a, u.y, b * v.y));
    z2[i] = w;
    acc = fma(w.x, w.x, acc);
    acc = fma(w.y, w.y, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// out[j] = scale * sum_b partials[j * nparts + b], fixed order per thread then
// fixed block butterfly; one block per j.  out_host (may be NULL): the same
// values into mapped host memory, read by the host after the stream syncs.
__global__ void __launch_bounds__(kRedThreads)
    k_reduce(const double* __restrict__ partials, int nparts, double* __restrict__ out,
             double scale, double* __restrict__ out_host) {
  __shared__ double sh[kRedThreads / 64];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kRedThreads) acc += partials[(long long)j * nparts + b];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    out[j] = scale * t;
    if (out_host) out_host[j] = scale * t;
  }
}

// x[i] += sum_j coef[j] * V_j[i]  (runtime k, coefficients on the device), or
// x[i] = that sum (assign)
__global__ void __launch_bounds__(256)
    k_combine(const double* __restrict__ V, long long ld, int k, const double* __restrict__ coef,
              double* __restrict__ x, long long n, int assign) {
  const long long n2 = n / 2;
  double2* x2 = reinterpret_cast<double2*>(x);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    // assign: x = sum_j coef[j] V_j, the same sums as from an x of zeros
    double2 a = assign ? make_double2(0.0, 0.0) : x2[i];
    for (int j = 0; j < k; ++j) {
      const double c = coef[j];
      const double2 v = reinterpret_cast<const double2*>(V + (long long)j * ld)[i];
      a.x = fma(c, v.x, a.x);
      a.y = fma(c, v.y, a.y);
    }
    x2[i] = a;
  }
}

// Products of one Gram-Schmidt step with a delayed second projection, in one
// sweep.  t = V_j (the previous direction, projected once) and w = V_{j+1} (the
// new operator output); rows of partials:
//   k < j: V_k . t,   j: t . t,   j + 1 + k (k < j): V_k . w,
//   2j + 1: t . w,    2j + 2: w . w.
// blockIdx.y takes V_k for k in [KMAX y, KMAX (y + 1)); chunk 0 also forms the
// three products of t and w.
template <int KMAX>
__global__ void __launch_bounds__(kRedThreads)
    k_dcgs_dots(const double* __restrict__ V, long long ld, int j, long long n,
                double* __restrict__ partials) {
  __shared__ double sh[kRedThreads / 64];
  const int nb = gridDim.x;
  const int k0 = blockIdx.y * KMAX;
  const bool first = blockIdx.y == 0;
  const long long n2 = n / 2;
  const double2* t2 = reinterpret_cast<const double2*>(V + (long long)j * ld);
  const double2* w2 = reinterpret_cast<const double2*>(V + (long long)(j + 1) * ld);
  double at[KMAX], aw[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) at[q] = aw[q] = 0.0;
  double tt = 0.0, tw = 0.0, ww = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n2;
       i += (long long)nb * kRedThreads) {
    const double2 t = t2[i], w = w2[i];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (k0 + q < j) {
        const double2 v = reinterpret_cast<const double2*>(V + (long long)(k0 + q) * ld)[i];
        at[q] = fma(v.x, t.x, at[q]);
        at[q] = fma(v.y, t.y, at[q]);
        aw[q] = fma(v.x, w.x, aw[q]);
        aw[q] = fma(v.y, w.y, aw[q]);
      }
    }
    if (first) {
      tt = fma(t.x, t.x, tt);
      tt = fma(t.y, t.y, tt);
      tw = fma(t.x, w.x, tw);
      tw = fma(t.y, w.y, tw);
      ww = fma(w.x, w.x, ww);
      ww = fma(w.y, w.y, ww);
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (k0 + q < j) {
      const double a = block_sum(at[q], sh);
      if (threadIdx.x == 0) partials[(long long)(k0 + q) * nb + blockIdx.x] = a;
      const double b = block_sum(aw[q], sh);
      if (threadIdx.x == 0) partials[(long long)(j + 1 + k0 + q) * nb + blockIdx.x] = b;
    }
  }
  if (first) {
    const double a = block_sum(tt, sh);
    if (threadIdx.x == 0) partials[(long long)j * nb + blockIdx.x] = a;
    const double b = block_sum(tw, sh);
    if (threadIdx.x == 0) partials[(long long)(2 * j + 1) * nb + blockIdx.x] = b;
    const double c = block_sum(ww, sh);
    if (threadIdx.x == 0) partials[(long long)(2 * j + 2) * nb + blockIdx.x] = c;
  }
}

// The two updates of that step in one sweep, in place:
//   t <- (t - sum_{k<j} cs[k] V_k) * inv_rho           (the final V_j; j > 0)
//   w <- (w - sum_{k<j} ch[k] V_k - hj t_new) * inv_eta
// cs and ch are rows of the products above, still on the device.
__global__ void __launch_bounds__(256)
    k_dcgs_update(double* __restrict__ V, long long ld, int j, const double* __restrict__ cs,
                  const double* __restrict__ ch, double hj, double inv_rho, double inv_eta,
                  long long n) {
  const long long n2 = n / 2;
  double2* t2 = reinterpret_cast<double2*>(V + (long long)j * ld);
  double2* w2 = reinterpret_cast<double2*>(V + (long long)(j + 1) * ld);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    double2 t = t2[i], w = w2[i];
    for (int k = 0; k < j; ++k) {
      const double2 v = reinterpret_cast<const double2*>(V + (long long)k * ld)[i];
      const double a = cs[k], b = ch[k];
      t.x = fma(-a, v.x, t.x);
      t.y = fma(-a, v.y, t.y);
      w.x = fma(-b, v.x, w.x);
      w.y = fma(-b, v.y, w.y);
    }
    t.x *= inv_rho;
    t.y *= inv_rho;
    w.x = fma(-hj, t.x, w.x) * inv_eta;
    w.y = fma(-hj, t.y, w.y) * inv_eta;
    if (j > 0) t2[i] = t;  // V_0 is final as given
    w2[i] = w;
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
  const double e = (nv > 0.0) ? 1.4901161193847656e-08 * (1.0 + nu) / nv : 0.0;
  eps[0] = e;
  eps[1] = e == 0.0 ? 0.0 : 1.0 / e;  // read by the product kernels instead of dividing
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
                  long long n, double* out_dev, hipStream_t s, double* out_host) {
  if (k <= 0) return PF_OK;
  const int nb = pb->n_red_blocks;
  const int chunks = (k + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_multidot, dim3(nb, chunks), dim3(kRedThreads), 0, s, V, ld, k, w, n,
                     pb->red_partials);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, s, pb->red_partials, nb, out_dev, 1.0,
                     out_host);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_axpby_norm(pf_problem* pb, double a, const double* x, double b, const double* y, double* z,
                    long long n, double* out_dev, hipStream_t s) {
  const int nb = pb->n_red_blocks;
  hipLaunchKernelGGL(k_axpby_norm, dim3(nb), dim3(kRedThreads), 0, s, a, x, b, y, z, n,
                     pb->red_partials);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, pb->red_partials, nb, out_dev, 1.0,
                     nullptr);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_dot(pf_problem* pb, const double* x, const double* y, long long n, double* out_dev,
             hipStream_t s) {
  return blas_multidot(pb, x, n, 1, y, n, out_dev, s);
}

int blas_dcgs_dots(pf_problem* pb, const double* V, long long ld, int j, long long n,
                   double* out_dev, hipStream_t s, double* out_host) {
  if (j < 0 || 2 * j + 3 > kRedRows) return PF_ERR_INVALID_ARG;
  const int nb = pb->n_red_blocks;
  if (j <= 8) {
    hipLaunchKernelGGL(k_dcgs_dots<8>, dim3(nb, 1), dim3(kRedThreads), 0, s, V, ld, j, n,
                       pb->red_partials);
  } else if (j <= 16) {
    hipLaunchKernelGGL(k_dcgs_dots<16>, dim3(nb, 1), dim3(kRedThreads), 0, s, V, ld, j, n,
                       pb->red_partials);
  } else {
    hipLaunchKernelGGL(k_dcgs_dots<16>, dim3(nb, (j + 15) / 16), dim3(kRedThreads), 0, s, V, ld,
                       j, n, pb->red_partials);
  }
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(2 * j + 3), dim3(kRedThreads), 0, s, pb->red_partials, nb,
                     out_dev, 1.0, out_host);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_dcgs_update(double* V, long long ld, int j, const double* dots_dev, double hj,
                     double inv_rho, double inv_eta, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_update, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, V, ld, j,
                     dots_dev, dots_dev + j + 1, hj, inv_rho, inv_eta, n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_combine(pf_problem* pb, const double* V, long long ld, int k, const double* coef_dev,
                 double* x, long long n, hipStream_t s, bool assign) {
  (void)pb;
  if (k <= 0 && !assign) return PF_OK;
  hipLaunchKernelGGL(k_combine, dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, s, V, ld, k,
                     coef_dev, x, n, assign ? 1 : 0);
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
  double* nrm = pb->red_out + kSlotFdU;
  PF_TRY(blas_multidot(pb, U, n, 1, U, n, nrm, s));
  PF_TRY(blas_multidot(pb, v, n, 1, v, n, nrm + 1, s));
  hipLaunchKernelGGL(k_fd_eps, dim3(1), dim3(1), 0, s, nrm, nrm + 1, eps_dev);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_fd_eps_cached(pf_problem* pb, const double* unorm2_dev, const double* v, long long n,
                       double* eps_dev, hipStream_t s) {
  double* nv = pb->red_out + kSlotFdV;
  PF_TRY(blas_multidot(pb, v, n, 1, v, n, nv, s));
  hipLaunchKernelGGL(k_fd_eps, dim3(1), dim3(1), 0, s, unorm2_dev, nv, eps_dev);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_reduce_partials(const double* partials, int nparts, int k, double* out_dev, double scale,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, s, partials, nparts, out_dev, scale,
                     nullptr);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int blas_sub_scalars(double* acc_dev, const double* x_dev, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_scalars, dim3(1), dim3(64), 0, s, acc_dev, x_dev, k);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace pf
