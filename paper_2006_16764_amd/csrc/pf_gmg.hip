// Preconditioner of the Newton-Krylov solver: M = diag(M11, M22) (the block
// Jacobi operator of the paper's Sec. 2.3.2, Eq. pre), each block of the form
//   A = sum_e c_e (sm M_e + sk K_e)
// with c_e the cell mean of a(grad phi)^2 for M11 (sm = 1/dt, sk = 1) and
// c_e = 1 for M22 (sm = 1/dt, sk = D) (Eqs. m11/pref2 and m22/preconc2 with
// k = 1).  Two inverses:
//   Jacobi  z = diag(A)^-1 r                                    (FP64)
//   GMG     one V-cycle per block, FP32 or FP64 arithmetic:
//           2x coarsening per axis, child-mean coarse coefficients,
//           multilinear prolongation P and restriction P^T, Jacobi-Chebyshev
//           smoothing of degree 2 on [max(lmin, lmax/4), 1.1 lmax] and
//           degree 16 on [lmin, 1.1 lmax] on the coarsest grid, with lmin,
//           lmax the exact extreme eigenvalues of D^-1 A for constant
//           coefficients (frequency corners of the Q1 symbol).
// The operator is applied matrix-free: a Q1 element matrix on a box depends
// only on which axes separate its two corners, so A x at a node is
// sum over its cells e of c_e sum_b Ae[a ^ b] x_b with 2^dim table entries.
#include <cmath>
#include <vector>

#include "pf_element.h"

namespace pf {

namespace {

constexpr int kT = 256;

struct LevelGeo {
  int dim;
  int n[3];
  int nn[3];
  long long nnodes, ncells;
  double Ae[8];  // element-matrix entry by corner-difference pattern
};

template <class T>
struct Level {
  LevelGeo g;
  double h[3];
  double lmin, lmax;
  T* c;     // cell coefficients
  T* dinv;  // inverse diagonal
  T* xa;
  T* xb;
  T* b;
  T* r;
  T* d;
};

template <class T>
struct Hier {
  std::vector<Level<T>> lv;
  double sm = 0.0, sk = 0.0;
  bool allocated = false;
};

struct PcState {
  Hier<float> h32[2];
  Hier<double> h64[2];
  double* jacobi_dinv = nullptr;  // [2 * n_nodes] interleaved, FP64
  double* coef0 = nullptr;        // FP64 cell coefficient of the phi block
};

__host__ __device__ inline long long node_of(const LevelGeo& g, int i, int j, int k) {
  return i + (long long)g.nn[0] * (j + (long long)g.nn[1] * k);
}

// ----------------------------------------------------------------- kernels
// c_e = sum_q w_q a(grad phi_q)^2 / sum_q w_q on every fine cell (FP64)
template <int DIM>
__global__ void __launch_bounds__(kT)
    k_cell_coef(Geo G, const double2* __restrict__ U, double* __restrict__ c) {
  const long long e = (long long)blockIdx.x * kT + threadIdx.x;
  if (e >= G.n_elems) return;
  const long long n0 = G.n[0], n1 = G.n[1];
  const long long ex = e % n0, rest = e / n0;
  const long long ey = DIM == 2 ? rest : rest % n1, ez = DIM == 2 ? 0 : rest / n1;
  const long long s1 = G.nn[0], s2 = (long long)G.nn[0] * G.nn[1];
  const long long base = ex + s1 * ey + s2 * ez;
  double p[1 << DIM];
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a)
    p[a] = U[base + (a & 1) + ((a >> 1) & 1) * s1 + (DIM == 3 ? ((a >> 2) & 1) * s2 : 0)].x;
  double acc = 0.0, wsum = 0.0;
#pragma unroll
  for (int gz = 0; gz < (DIM == 3 ? 3 : 1); ++gz) {
#pragma unroll
    for (int gy = 0; gy < 3; ++gy) {
#pragma unroll
      for (int gx = 0; gx < 3; ++gx) {
        double g[3] = {0.0, 0.0, 0.0};
        // gradient of the multilinear interpolant at the Gauss point
#pragma unroll
        for (int a = 0; a < (1 << DIM); ++a) {
          const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
          const double bx = ax ? Q1::b1(gx) : Q1::b0(gx);
          const double by = ay ? Q1::b1(gy) : Q1::b0(gy);
          const double bz = DIM == 3 ? (az ? Q1::b1(gz) : Q1::b0(gz)) : 1.0;
          const double dx = ax ? G.ih[0] : -G.ih[0];
          const double dy = ay ? G.ih[1] : -G.ih[1];
          const double dzz = az ? G.ih[2] : -G.ih[2];
          g[0] += p[a] * dx * by * bz;
          g[1] += p[a] * bx * dy * bz;
          if (DIM == 3) g[2] += p[a] * bx * by * dzz;
        }
        Aniso<DIM> A;
        A.eval(g, G.eps4, G.delta2);
        const double w = Q1::w(gx) * Q1::w(gy) * (DIM == 3 ? Q1::w(gz) : 1.0);
        acc += w * A.a * A.a;
        wsum += w;
      }
    }
  }
  c[e] = acc / wsum;
}

template <class T>
__global__ void k_convert(const double* __restrict__ x, T* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) y[i] = (T)x[i];
}

template <class T>
__global__ void k_fill(T* __restrict__ y, T v, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) y[i] = v;
}

// coarse cell = mean of its 2^dim children
template <int DIM, class T>
__global__ void k_coarsen(LevelGeo fg, LevelGeo cg, const T* __restrict__ cf, T* __restrict__ cc) {
  const long long E = (long long)blockIdx.x * kT + threadIdx.x;
  if (E >= cg.ncells) return;
  const int EX = (int)(E % cg.n[0]);
  const long long rest = E / cg.n[0];
  const int EY = DIM == 2 ? (int)rest : (int)(rest % cg.n[1]);
  const int EZ = DIM == 2 ? 0 : (int)(rest / cg.n[1]);
  T acc = 0;
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx)
        acc += cf[(2 * EX + dx) + (long long)fg.n[0] * ((2 * EY + dy) + (long long)fg.n[1] * (2 * EZ + dz))];
  cc[E] = acc * (T)(DIM == 3 ? 0.125 : 0.25);
}

// y_i = (A x)_i; optionally r_i = b_i - (A x)_i.  Deterministic fixed order.
template <int DIM, class T>
__device__ __forceinline__ T apply_A(const LevelGeo& g, const T* __restrict__ c,
                                     const T* __restrict__ x, int ix, int iy, int iz) {
  T acc = 0;
#pragma unroll
  for (int bz = 0; bz < (DIM == 3 ? 2 : 1); ++bz) {
    const int ez = DIM == 3 ? iz - 1 + bz : 0;
    if (DIM == 3 && (ez < 0 || ez >= g.n[2])) continue;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int ey = iy - 1 + by;
      if (ey < 0 || ey >= g.n[1]) continue;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int ex = ix - 1 + bx;
        if (ex < 0 || ex >= g.n[0]) continue;
        const T ce = c ? c[ex + (long long)g.n[0] * (ey + (long long)g.n[1] * ez)] : (T)1;
        const int a = (1 - bx) + 2 * (1 - by) + (DIM == 3 ? 4 * (1 - bz) : 0);
        T s = 0;
#pragma unroll
        for (int b = 0; b < (1 << DIM); ++b) {
          const T xb = x[node_of(g, ex + (b & 1), ey + ((b >> 1) & 1), ez + (DIM == 3 ? ((b >> 2) & 1) : 0))];
          s += (T)g.Ae[a ^ b] * xb;
        }
        acc += ce * s;
      }
    }
  }
  return acc;
}

template <int DIM>
__device__ __forceinline__ void node_ijk(const LevelGeo& g, long long i, int& ix, int& iy, int& iz) {
  ix = (int)(i % g.nn[0]);
  const long long r = i / g.nn[0];
  iy = DIM == 2 ? (int)r : (int)(r % g.nn[1]);
  iz = DIM == 2 ? 0 : (int)(r / g.nn[1]);
}

template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_diag(LevelGeo g, const T* __restrict__ c, T* __restrict__ dinv) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= g.nnodes) return;
  int ix, iy, iz;
  node_ijk<DIM>(g, i, ix, iy, iz);
  T acc = 0;
#pragma unroll
  for (int bz = 0; bz < (DIM == 3 ? 2 : 1); ++bz) {
    const int ez = DIM == 3 ? iz - 1 + bz : 0;
    if (DIM == 3 && (ez < 0 || ez >= g.n[2])) continue;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int ey = iy - 1 + by;
      if (ey < 0 || ey >= g.n[1]) continue;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int ex = ix - 1 + bx;
        if (ex < 0 || ex >= g.n[0]) continue;
        acc += c ? c[ex + (long long)g.n[0] * (ey + (long long)g.n[1] * ez)] : (T)1;
      }
    }
  }
  dinv[i] = (T)1 / (acc * (T)g.Ae[0]);
}

// One Jacobi-Chebyshev step.  zero_start: x = d = beta * dinv * b (x_in = 0).
// Otherwise d = alpha d + beta dinv (b - A x_in), x_out = x_in + d.
template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_cheb(LevelGeo g, const T* __restrict__ c, const T* __restrict__ dinv,
           const T* __restrict__ b, const T* __restrict__ x_in, T* __restrict__ x_out,
           T* __restrict__ d, T alpha, T beta, int zero_start) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= g.nnodes) return;
  if (zero_start) {
    const T v = beta * dinv[i] * b[i];
    d[i] = v;
    x_out[i] = v;
    return;
  }
  int ix, iy, iz;
  node_ijk<DIM>(g, i, ix, iy, iz);
  const T r = b[i] - apply_A<DIM, T>(g, c, x_in, ix, iy, iz);
  const T dn = (alpha == (T)0 ? (T)0 : alpha * d[i]) + beta * dinv[i] * r;
  d[i] = dn;
  x_out[i] = x_in[i] + dn;
}

template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_resid(LevelGeo g, const T* __restrict__ c, const T* __restrict__ b,
            const T* __restrict__ x, T* __restrict__ r) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= g.nnodes) return;
  int ix, iy, iz;
  node_ijk<DIM>(g, i, ix, iy, iz);
  r[i] = b[i] - apply_A<DIM, T>(g, c, x, ix, iy, iz);
}

// b_c[I] = sum_i P[i, I] r_f[i]: fine neighbours 2I-1, 2I, 2I+1 per axis with
// weights 1/2, 1, 1/2.
template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_restrict(LevelGeo fg, LevelGeo cg, const T* __restrict__ rf, T* __restrict__ bc) {
  const long long I = (long long)blockIdx.x * kT + threadIdx.x;
  if (I >= cg.nnodes) return;
  int cx, cy, cz;
  node_ijk<DIM>(cg, I, cx, cy, cz);
  T acc = 0;
#pragma unroll
  for (int dz = -1; dz <= (DIM == 3 ? 1 : -1); ++dz) {
    const int fz = DIM == 3 ? 2 * cz + dz : 0;
    if (DIM == 3 && (fz < 0 || fz >= fg.nn[2])) continue;
    const T wz = DIM == 3 ? (dz == 0 ? (T)1 : (T)0.5) : (T)1;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int fy = 2 * cy + dy;
      if (fy < 0 || fy >= fg.nn[1]) continue;
      const T wy = dy == 0 ? (T)1 : (T)0.5;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int fx = 2 * cx + dx;
        if (fx < 0 || fx >= fg.nn[0]) continue;
        const T wx = dx == 0 ? (T)1 : (T)0.5;
        acc += (wx * wy * wz) * rf[node_of(fg, fx, fy, fz)];
      }
    }
  }
  bc[I] = acc;
}

// x_f[i] += sum_I P[i, I] e_c[I]
template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_prolong_add(LevelGeo fg, LevelGeo cg, const T* __restrict__ ec, T* __restrict__ xf) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= fg.nnodes) return;
  int fx, fy, fz;
  node_ijk<DIM>(fg, i, fx, fy, fz);
  const int x0 = fx >> 1, x1 = (fx + 1) >> 1;
  const int y0 = fy >> 1, y1 = (fy + 1) >> 1;
  const int z0 = DIM == 3 ? fz >> 1 : 0, z1 = DIM == 3 ? (fz + 1) >> 1 : 0;
  const T wx = (fx & 1) ? (T)0.5 : (T)1;
  const T wy = (fy & 1) ? (T)0.5 : (T)1;
  const T wz = (DIM == 3 && (fz & 1)) ? (T)0.5 : (T)1;
  T acc = wx * wy * wz * ec[node_of(cg, x0, y0, z0)];
  if (fx & 1) acc += wx * wy * wz * ec[node_of(cg, x1, y0, z0)];
  if (fy & 1) acc += wx * wy * wz * ec[node_of(cg, x0, y1, z0)];
  if ((fx & 1) && (fy & 1)) acc += wx * wy * wz * ec[node_of(cg, x1, y1, z0)];
  if (DIM == 3 && (fz & 1)) {
    acc += wx * wy * wz * ec[node_of(cg, x0, y0, z1)];
    if (fx & 1) acc += wx * wy * wz * ec[node_of(cg, x1, y0, z1)];
    if (fy & 1) acc += wx * wy * wz * ec[node_of(cg, x0, y1, z1)];
    if ((fx & 1) && (fy & 1)) acc += wx * wy * wz * ec[node_of(cg, x1, y1, z1)];
  }
  xf[i] += acc;
}

template <class T>
__global__ void k_split(const double2* __restrict__ r, T* __restrict__ b0, T* __restrict__ b1,
                        long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double2 v = r[i];
  b0[i] = (T)v.x;
  b1[i] = (T)v.y;
}

template <class T>
__global__ void k_merge(const T* __restrict__ x0, const T* __restrict__ x1, double2* __restrict__ z,
                        long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  z[i] = make_double2((double)x0[i], (double)x1[i]);
}

__global__ void k_jacobi(const double2* __restrict__ r, const double2* __restrict__ dinv,
                         double2* __restrict__ z, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double2 a = r[i], d = dinv[i];
  z[i] = make_double2(a.x * d.x, a.y * d.y);
}

template <class T>
__global__ void k_interleave_dinv(const T* __restrict__ d0, const T* __restrict__ d1,
                                  double2* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  out[i] = make_double2((double)d0[i], (double)d1[i]);
}

__global__ void k_copy2(const double2* __restrict__ x, double2* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) y[i] = x[i];
}

inline unsigned blocks(long long n) { return (unsigned)((n + kT - 1) / kT); }

// ----------------------------------------------------------------- host side
// Element-matrix entries sm M_e[a,b] + sk K_e[a,b] indexed by p = a ^ b: the
// 1-D factors are m(same) = h/3, m(diff) = h/6, k(same) = 1/h, k(diff) = -1/h.
void element_table(int dim, const double* h, double sm, double sk, double* Ae) {
  for (int p = 0; p < (1 << dim); ++p) {
    double M = 1.0;
    for (int k = 0; k < dim; ++k) M *= ((p >> k) & 1) ? h[k] / 6.0 : h[k] / 3.0;
    double K = 0.0;
    for (int k = 0; k < dim; ++k) {
      double t = ((p >> k) & 1) ? -1.0 / h[k] : 1.0 / h[k];
      for (int j = 0; j < dim; ++j)
        if (j != k) t *= ((p >> j) & 1) ? h[j] / 6.0 : h[j] / 3.0;
      K += t;
    }
    Ae[p] = sm * M + sk * K;
  }
  for (int p = (1 << dim); p < 8; ++p) Ae[p] = 0.0;
}

// Extreme eigenvalues of D^-1 A for constant coefficients: the Q1 symbol is
// multilinear in cos(theta_k), so they sit at the corners cos = +-1.
void symbol_extremes(int dim, const double* h, double sm, double sk, double* lo, double* hi) {
  double diagM = 1.0;
  for (int k = 0; k < dim; ++k) diagM *= 2.0 * h[k] / 3.0;
  double diagK = 0.0;
  for (int k = 0; k < dim; ++k) {
    double t = 2.0 / h[k];
    for (int j = 0; j < dim; ++j)
      if (j != k) t *= 2.0 * h[j] / 3.0;
    diagK += t;
  }
  const double diag = sm * diagM + sk * diagK;
  double mn = 1e300, mx = -1e300;
  for (int corner = 0; corner < (1 << dim); ++corner) {
    double m[3], kk[3];
    for (int k = 0; k < dim; ++k) {
      const double cs = ((corner >> k) & 1) ? -1.0 : 1.0;
      m[k] = h[k] * (2.0 + cs) / 3.0;
      kk[k] = (2.0 - 2.0 * cs) / h[k];
    }
    double M = 1.0;
    for (int k = 0; k < dim; ++k) M *= m[k];
    double K = 0.0;
    for (int k = 0; k < dim; ++k) {
      double t = kk[k];
      for (int j = 0; j < dim; ++j)
        if (j != k) t *= m[j];
      K += t;
    }
    const double v = (sm * M + sk * K) / diag;
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  *lo = mn;
  *hi = mx;
}

constexpr int kCoarseMin = 4;
constexpr int kCoarseDegree = 16;
constexpr double kChebRatio = 4.0;
constexpr double kChebSafety = 1.1;

template <class T>
int hier_alloc(pf_problem* pb, Hier<T>& H, bool with_coef) {
  const Geo& G = pb->geo;
  int n[3] = {G.n[0], G.n[1], G.dim == 3 ? G.n[2] : 1};
  double h[3] = {G.h[0], G.h[1], G.h[2]};
  H.lv.clear();
  while (true) {
    Level<T> L{};
    L.g.dim = G.dim;
    for (int k = 0; k < 3; ++k) {
      L.g.n[k] = (k < G.dim) ? n[k] : 1;
      L.g.nn[k] = (k < G.dim) ? n[k] + 1 : 1;
      L.h[k] = h[k];
    }
    L.g.nnodes = (long long)L.g.nn[0] * L.g.nn[1] * L.g.nn[2];
    L.g.ncells = (long long)L.g.n[0] * L.g.n[1] * L.g.n[2];
    const size_t nb = (size_t)L.g.nnodes * sizeof(T);
    if (with_coef) {
      if (hipMalloc(&L.c, (size_t)L.g.ncells * sizeof(T)) != hipSuccess) return PF_ERR_OOM;
    }
    T** bufs[] = {&L.dinv, &L.xa, &L.xb, &L.b, &L.r, &L.d};
    for (T** p : bufs)
      if (hipMalloc(p, nb) != hipSuccess) return PF_ERR_OOM;
    H.lv.push_back(L);
    bool even = true;
    int mn = 1 << 30;
    for (int k = 0; k < G.dim; ++k) {
      even = even && (n[k] % 2 == 0);
      mn = n[k] < mn ? n[k] : mn;
    }
    if (!even || mn <= kCoarseMin) break;
    for (int k = 0; k < G.dim; ++k) {
      n[k] /= 2;
      h[k] *= 2.0;
    }
  }
  H.allocated = true;
  return PF_OK;
}

template <class T>
hipError_t hier_free(Hier<T>& H) {
  hipError_t first = hipSuccess;
  for (auto& L : H.lv) {
    T* bufs[] = {L.c, L.dinv, L.xa, L.xb, L.b, L.r, L.d};
    for (T* p : bufs) {
      if (!p) continue;
      const hipError_t e = hipFree(p);
      if (first == hipSuccess) first = e;
    }
  }
  H.lv.clear();
  H.allocated = false;
  return first;
}

template <int DIM, class T>
int hier_setup(Hier<T>& H, const double* c0_dev, double sm, double sk, hipStream_t s) {
  H.sm = sm;
  H.sk = sk;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level<T>& L = H.lv[l];
    element_table(DIM, L.h, sm, sk, L.g.Ae);
    symbol_extremes(DIM, L.h, sm, sk, &L.lmin, &L.lmax);
    if (L.c) {
      if (l == 0) {
        hipLaunchKernelGGL((k_convert<T>), dim3(blocks(L.g.ncells)), dim3(kT), 0, s, c0_dev, L.c,
                           L.g.ncells);
      } else {
        hipLaunchKernelGGL((k_coarsen<DIM, T>), dim3(blocks(L.g.ncells)), dim3(kT), 0, s,
                           H.lv[l - 1].g, L.g, H.lv[l - 1].c, L.c);
      }
      PF_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL((k_diag<DIM, T>), dim3(blocks(L.g.nnodes)), dim3(kT), 0, s, L.g,
                       (const T*)L.c, L.dinv);
    PF_HIP_CHECK(hipGetLastError());
  }
  return PF_OK;
}

// Run a Jacobi-Chebyshev iteration of the given degree on level L for A x = b,
// starting from *x (nullptr = zero).  Returns the buffer holding the result.
template <int DIM, class T>
int chebyshev(Level<T>& L, T* x0, int degree, bool coarse, hipStream_t s, T** result) {
  const double hi = kChebSafety * L.lmax;
  double lo = coarse ? L.lmin : L.lmax / kChebRatio;
  if (!coarse && L.lmin > lo) lo = L.lmin;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  T* cur = x0;
  T* bufs[2] = {L.xa, L.xb};
  int which = (x0 == L.xa) ? 1 : 0;
  for (int k = 0; k < degree; ++k) {
    T alpha, beta;
    if (k == 0) {
      alpha = 0;
      beta = (T)(1.0 / theta);
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      alpha = (T)(rn * rho);
      beta = (T)(2.0 * rn / delta);
      rho = rn;
    }
    T* out = bufs[which];
    hipLaunchKernelGGL((k_cheb<DIM, T>), dim3(blocks(L.g.nnodes)), dim3(kT), 0, s, L.g,
                       (const T*)L.c, (const T*)L.dinv, (const T*)L.b, (const T*)cur, out, L.d,
                       alpha, beta, cur == nullptr ? 1 : 0);
    PF_HIP_CHECK(hipGetLastError());
    cur = out;
    which ^= 1;
  }
  *result = cur;
  return PF_OK;
}

// V-cycle on levels l..end for the right-hand side already in lv[l].b.
template <int DIM, class T>
int vcycle(Hier<T>& H, size_t l, hipStream_t s, T** result) {
  Level<T>& L = H.lv[l];
  if (l + 1 == H.lv.size()) return chebyshev<DIM, T>(L, nullptr, kCoarseDegree, true, s, result);
  T* x = nullptr;
  PF_TRY((chebyshev<DIM, T>(L, nullptr, 2, false, s, &x)));
  hipLaunchKernelGGL((k_resid<DIM, T>), dim3(blocks(L.g.nnodes)), dim3(kT), 0, s, L.g,
                     (const T*)L.c, (const T*)L.b, (const T*)x, L.r);
  PF_HIP_CHECK(hipGetLastError());
  Level<T>& C = H.lv[l + 1];
  hipLaunchKernelGGL((k_restrict<DIM, T>), dim3(blocks(C.g.nnodes)), dim3(kT), 0, s, L.g, C.g,
                     (const T*)L.r, C.b);
  PF_HIP_CHECK(hipGetLastError());
  T* ec = nullptr;
  PF_TRY((vcycle<DIM, T>(H, l + 1, s, &ec)));
  hipLaunchKernelGGL((k_prolong_add<DIM, T>), dim3(blocks(L.g.nnodes)), dim3(kT), 0, s, L.g, C.g,
                     (const T*)ec, x);
  PF_HIP_CHECK(hipGetLastError());
  return chebyshev<DIM, T>(L, x, 2, false, s, result);
}

template <class T>
int apply_gmg(pf_problem* pb, Hier<T>* H, const double* r, double* z, hipStream_t s) {
  const long long n = pb->geo.n_nodes;
  hipLaunchKernelGGL((k_split<T>), dim3(blocks(n)), dim3(kT), 0, s,
                     reinterpret_cast<const double2*>(r), H[0].lv[0].b, H[1].lv[0].b, n);
  PF_HIP_CHECK(hipGetLastError());
  T* x[2];
  for (int f = 0; f < 2; ++f) {
    if (pb->geo.dim == 3) PF_TRY((vcycle<3, T>(H[f], 0, s, &x[f])));
    else PF_TRY((vcycle<2, T>(H[f], 0, s, &x[f])));
  }
  hipLaunchKernelGGL((k_merge<T>), dim3(blocks(n)), dim3(kT), 0, s, (const T*)x[0], (const T*)x[1],
                     reinterpret_cast<double2*>(z), n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

template <class T>
int setup_gmg(pf_problem* pb, PcState* st, Hier<T>* H, hipStream_t s) {
  for (int f = 0; f < 2; ++f)
    if (!H[f].allocated) PF_TRY(hier_alloc<T>(pb, H[f], f == 0));
  const double idt = 1.0 / pb->params.dt;
  if (pb->geo.dim == 3) {
    PF_TRY((hier_setup<3, T>(H[0], st->coef0, idt, 1.0, s)));
    PF_TRY((hier_setup<3, T>(H[1], nullptr, idt, pb->params.D, s)));
  } else {
    PF_TRY((hier_setup<2, T>(H[0], st->coef0, idt, 1.0, s)));
    PF_TRY((hier_setup<2, T>(H[1], nullptr, idt, pb->params.D, s)));
  }
  return PF_OK;
}

}  // namespace

int pc_alloc(pf_problem* pb) {
  PcState* st = new PcState();
  pb->pc = st;
  if (hipMalloc(&st->coef0, (size_t)pb->geo.n_elems * sizeof(double)) != hipSuccess) return PF_ERR_OOM;
  if (hipMalloc(&st->jacobi_dinv, (size_t)pb->n_dof * sizeof(double)) != hipSuccess) return PF_ERR_OOM;
  return PF_OK;
}

hipError_t pc_free(pf_problem* pb) {
  PcState* st = static_cast<PcState*>(pb->pc);
  if (!st) return hipSuccess;
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess) first = e;
  };
  for (int f = 0; f < 2; ++f) {
    keep(hier_free(st->h32[f]));
    keep(hier_free(st->h64[f]));
  }
  if (st->coef0) keep(hipFree(st->coef0));
  if (st->jacobi_dinv) keep(hipFree(st->jacobi_dinv));
  delete st;
  pb->pc = nullptr;
  return first;
}

int pc_setup(pf_problem* pb, const double* U, int kind, int precision, hipStream_t s) {
  PcState* st = static_cast<PcState*>(pb->pc);
  pb->pc_kind = kind;
  pb->pc_precision = precision;
  if (kind == PF_PC_NONE) return PF_OK;
  const Geo& G = pb->geo;
  if (G.dim == 3)
    hipLaunchKernelGGL(k_cell_coef<3>, dim3(blocks(G.n_elems)), dim3(kT), 0, s, G,
                       reinterpret_cast<const double2*>(U), st->coef0);
  else
    hipLaunchKernelGGL(k_cell_coef<2>, dim3(blocks(G.n_elems)), dim3(kT), 0, s, G,
                       reinterpret_cast<const double2*>(U), st->coef0);
  PF_HIP_CHECK(hipGetLastError());
  if (kind == PF_PC_JACOBI) {
    // FP64 diagonals of both blocks on level 0 only
    Hier<double>* H = st->h64;
    PF_TRY(setup_gmg<double>(pb, st, H, s));
    hipLaunchKernelGGL((k_interleave_dinv<double>), dim3(blocks(G.n_nodes)), dim3(kT), 0, s,
                       (const double*)H[0].lv[0].dinv, (const double*)H[1].lv[0].dinv,
                       reinterpret_cast<double2*>(st->jacobi_dinv), G.n_nodes);
    PF_HIP_CHECK(hipGetLastError());
    return PF_OK;
  }
  if (precision == PF_FP32) return setup_gmg<float>(pb, st, st->h32, s);
  return setup_gmg<double>(pb, st, st->h64, s);
}

int pc_apply(pf_problem* pb, const double* r, double* z, hipStream_t s) {
  PcState* st = static_cast<PcState*>(pb->pc);
  const long long n = pb->geo.n_nodes;
  switch (pb->pc_kind) {
    case PF_PC_NONE:
      hipLaunchKernelGGL(k_copy2, dim3(blocks(n)), dim3(kT), 0, s,
                         reinterpret_cast<const double2*>(r), reinterpret_cast<double2*>(z), n);
      PF_HIP_CHECK(hipGetLastError());
      return PF_OK;
    case PF_PC_JACOBI:
      hipLaunchKernelGGL(k_jacobi, dim3(blocks(n)), dim3(kT), 0, s,
                         reinterpret_cast<const double2*>(r),
                         reinterpret_cast<const double2*>(st->jacobi_dinv),
                         reinterpret_cast<double2*>(z), n);
      PF_HIP_CHECK(hipGetLastError());
      return PF_OK;
    default:
      if (pb->pc_precision == PF_FP32) return apply_gmg<float>(pb, st->h32, r, z, s);
      return apply_gmg<double>(pb, st->h64, r, z, s);
  }
}

}  // namespace pf
