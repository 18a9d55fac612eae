// Preconditioner of the Newton-Krylov solver: M = diag(M11, M22) (the block
// Jacobi operator of the paper's Sec. 2.3.2, Eq. pre), each block of the form
//   A = sum_e c_e (sm M_e + sk K_e)
// with c_e the cell mean of a(grad phi)^2 for M11 (sm = 1/dt, sk = theta) and
// c_e = 1 for M22 (sm = 1/dt, sk = theta D) (Eqs. m11/pref2 and m22/preconc2 with
// k = 1).  Two inverses:
//   Jacobi  z = diag(A)^-1 r                                    (FP64)
//   GMG     one V-cycle per block, FP32 or FP64 arithmetic:
//           2x coarsening per axis, child-mean coarse coefficients,
//           multilinear prolongation P and restriction P^T, Jacobi-Chebyshev
//           smoothing of degree 2 on [max(lmin, lmax/4), 1.1 lmax] and
//           degree 16 on [lmin, 1.1 lmax] on the coarsest grid, with lmin,
//           lmax the exact extreme eigenvalues of D^-1 A for constant
//           coefficients (frequency corners of the Q1 symbol).
//
// Matrix-free node-centric operator: the Q1 element matrix entry between two
// corners depends only on which axes separate them, so row i of A is a
// 27-point (9-point) stencil whose weight for the neighbour at offset d is
//   Ae[p(d)] * (sum of c_e over the cells shared by node i and node i + d),
// p(d) = sum_k [d_k != 0] 2^k.  The shared-cell sums come from the 8 (4)
// cells around the node by partial sums along each axis; cells outside the
// mesh count as zero, which gives the natural-boundary rows.  The diagonal is
// the d = 0 weight; the smoothers recompute it from the cells, except the
// zero-start step, which reads the phi-block diagonal stored per node at
// set-up (the u-block diagonal is a product of cell counts).  Both blocks are
// processed by the same thread and stored as interleaved (phi, u) pairs.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pf_element.h"

namespace pf {

namespace {

constexpr int kT = 256;

// Workgroup barrier for LDS only: this wave's LDS operations have completed
// and no memory access is moved across it by the compiler, but global loads
// and stores issued before it may still be in flight.  __syncthreads() also
// waits for those (a workgroup release fence), which exposes the latency of
// every store a wave issued just before it.  Used where the threads of a
// workgroup exchange data through LDS only (the tiled sweeps and the tiled
// restriction: no thread reads another's global writes within a launch).
#ifndef PF_LDS_BARRIER
#define PF_LDS_BARRIER 1
#endif
__device__ __forceinline__ void lds_barrier() {
  if (PF_LDS_BARRIER) __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else __syncthreads();
}
constexpr int kCoarseMin = 4;
// 3-D restriction through LDS-staged fine planes (0: one thread per coarse
// node gathering its 27 fine neighbours)
#ifndef PF_RESTRICT_TILED
#define PF_RESTRICT_TILED 1
#endif
constexpr int kCoarseDegree = 16;
constexpr double kChebRatio = 4.0;
constexpr double kChebSafety = 1.1;
constexpr int kCoarseLdsNodes = 1024;  // coarsest grids up to this size are solved by one workgroup

template <class T>
struct V2;
template <>
struct V2<float> {
  using type = float2;
};
template <>
struct V2<double> {
  using type = double2;
};

// Kernel-side description of one level (both blocks).
struct LvK {
  int n[3];
  int nn[3];
  long long nnodes, ncells;
  double Ae[2][8];  // element-matrix entry by corner-difference pattern, per block
};

template <class T>
struct Level {
  LvK k;
  double h[3];
  double lmin[2], lmax[2];
  T* c;                          // phi-block cell coefficients
  typename V2<T>::type* xa;      // iterates (phi, u)
  typename V2<T>::type* xb;
  typename V2<T>::type* b;       // right-hand side
  typename V2<T>::type* r;       // residual
  typename V2<T>::type* d;       // Chebyshev direction
  T* dg;                         // phi-block diagonal per node
  int kz;                        // z-march length of the tiled 3-D stencils (0: untiled)
};

template <class T>
struct Hier {
  std::vector<Level<T>> lv;
  bool allocated = false;
  double coarse_host[4 * kCoarseDegree];  // per-step (alpha, beta) of the coarsest solve
  double* coarse_dev = nullptr;
};

// A V-cycle captured as one HIP graph: its launches (a few microseconds each on
// small grids) replay as one submission.  sig holds the block scales the
// captured kernel arguments were derived from and level0 the hierarchy they
// point into; either changing forces a new capture.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  double sig[4] = {0.0, 0.0, 0.0, 0.0};
  const void* level0 = nullptr;
};

// Meshes up to this many unknowns apply the V-cycle as a replayed graph
// (measured: a 150^2 free-growth step 20 % faster; at 2.1 M unknowns the two
// copies cost more than the launches saved).
constexpr long long kGraphMaxDof = 1LL << 20;

struct PcState {
  Hier<float> h32;
  Hier<double> h64;
  double* coef0 = nullptr;  // FP64 cell coefficient of the phi block (level 0)
  // graph path (small meshes): fixed input and output vectors of the captured
  // cycle, the stream it is captured on, one graph per precision
  bool graph_enabled = true;
  double* gin = nullptr;
  double* gout = nullptr;
  hipStream_t cap = nullptr;
  GraphCache g32, g64;
};

__host__ __device__ inline long long nidx(const LvK& g, int i, int j, int k) {
  return i + (long long)g.nn[0] * (j + (long long)g.nn[1] * k);
}

template <int DIM>
__device__ __forceinline__ void node_ijk(const LvK& g, long long i, int& ix, int& iy, int& iz) {
  ix = (int)(i % g.nn[0]);
  const long long r = i / g.nn[0];
  iy = DIM == 2 ? (int)r : (int)(r % g.nn[1]);
  iz = DIM == 2 ? 0 : (int)(r / g.nn[1]);
}

// Node-wise kernels run on a 2-D grid: blockIdx.y is the node plane (z; 0 in
// 2-D) and blockIdx.x * kT + threadIdx.x the node within the plane, so that the
// coordinates come from 32-bit arithmetic.  Returns false past the plane's end.
__device__ __forceinline__ bool plane_node(const LvK& g, int& ix, int& iy, int& iz, long long& i) {
  const int pn = g.nn[0] * g.nn[1];
  const int q = (int)blockIdx.x * kT + (int)threadIdx.x;
  if (q >= pn) return false;
  iy = q / g.nn[0];
  ix = q - iy * g.nn[0];
  iz = (int)blockIdx.y;
  i = (long long)iz * pn + q;
  return true;
}

inline dim3 plane_grid(const LvK& k) {
  return dim3((unsigned)(((long long)k.nn[0] * k.nn[1] + kT - 1) / kT), (unsigned)k.nn[2]);
}

// Stencil of node (ix, iy, iz) for both blocks: w[b][t] for the 3^DIM offsets t
// (t = tx + 3 ty + 9 tz, offset t_k - 1).  Block 0 weights cells by c, block 1
// by 1 (cells outside the mesh weigh 0).
// Weights from the block-0 cell coefficients around the node (cc, zero for
// cells outside the mesh) and the per-axis existence flags of those cells.
template <int DIM, class T>
__device__ __forceinline__ void stencil_weights(const LvK& g, const T (&cc)[DIM == 3 ? 2 : 1][2][2],
                                                const bool (&ex)[2], const bool (&ey)[2],
                                                const bool (&ez)[2], T (&w0)[DIM == 3 ? 27 : 9],
                                                T (&w1)[DIM == 3 ? 27 : 9]) {
  constexpr int NZ = DIM == 3 ? 2 : 1;
  // partial sums over the shared cells: offset -1 -> side 0, +1 -> side 1, 0 -> both
  T sx[3][NZ][2];
#pragma unroll
  for (int bz = 0; bz < NZ; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      sx[0][bz][by] = cc[bz][by][0];
      sx[2][bz][by] = cc[bz][by][1];
      sx[1][bz][by] = cc[bz][by][0] + cc[bz][by][1];
    }
  T sxy[3][3][NZ];
#pragma unroll
  for (int tx = 0; tx < 3; ++tx)
#pragma unroll
    for (int bz = 0; bz < NZ; ++bz) {
      sxy[tx][0][bz] = sx[tx][bz][0];
      sxy[tx][2][bz] = sx[tx][bz][1];
      sxy[tx][1][bz] = sx[tx][bz][0] + sx[tx][bz][1];
    }
  // block-1 counts factor per axis
  T cxn[3], cyn[3], czn[3];
  cxn[0] = ex[0] ? 1 : 0;
  cxn[2] = ex[1] ? 1 : 0;
  cxn[1] = cxn[0] + cxn[2];
  cyn[0] = ey[0] ? 1 : 0;
  cyn[2] = ey[1] ? 1 : 0;
  cyn[1] = cyn[0] + cyn[2];
  czn[0] = ez[0] ? 1 : 0;
  czn[2] = ez[1] ? 1 : 0;
  czn[1] = czn[0] + czn[2];
#pragma unroll
  for (int tz = 0; tz < (DIM == 3 ? 3 : 1); ++tz)
#pragma unroll
    for (int ty = 0; ty < 3; ++ty)
#pragma unroll
      for (int tx = 0; tx < 3; ++tx) {
        T s;
        if (DIM == 3) {
          const int a = tz == 0 ? 0 : (tz == 2 ? 1 : 2);
          s = a == 0 ? sxy[tx][ty][0] : (a == 1 ? sxy[tx][ty][NZ - 1] : sxy[tx][ty][0] + sxy[tx][ty][NZ - 1]);
        } else {
          s = sxy[tx][ty][0];
        }
        const int p = (tx != 1 ? 1 : 0) + (ty != 1 ? 2 : 0) + (tz != 1 && DIM == 3 ? 4 : 0);
        const int t = tx + 3 * ty + 9 * tz;
        const T n1 = cxn[tx] * cyn[ty] * (DIM == 3 ? czn[tz] : (T)1);
        w0[t] = (T)g.Ae[0][p] * s;
        w1[t] = (T)g.Ae[1][p] * n1;
      }
}


template <int DIM, class T>
__device__ __forceinline__ void stencil(const LvK& g, const T* __restrict__ c, int ix, int iy,
                                        int iz, T (&w0)[DIM == 3 ? 27 : 9],
                                        T (&w1)[DIM == 3 ? 27 : 9]) {
  constexpr int NZ = DIM == 3 ? 2 : 1;
  T cc[NZ][2][2];  // [bz][by][bx]
  bool ex[2], ey[2], ez[2];
  ex[0] = ix - 1 >= 0;
  ex[1] = ix < g.n[0];
  ey[0] = iy - 1 >= 0;
  ey[1] = iy < g.n[1];
  ez[0] = DIM == 2 ? true : iz - 1 >= 0;
  ez[1] = DIM == 2 ? true : iz < g.n[2];
#pragma unroll
  for (int bz = 0; bz < NZ; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const bool e = ex[bx] && ey[by] && (DIM == 2 || ez[bz]);
        const int cx = ix - 1 + bx, cy = iy - 1 + by, cz = DIM == 3 ? iz - 1 + bz : 0;
        T v = 0;
        if (e) v = c ? c[cx + (long long)g.n[0] * (cy + (long long)g.n[1] * cz)] : (T)1;
        cc[bz][by][bx] = v;
      }
  stencil_weights<DIM, T>(g, cc, ex, ey, ez, w0, w1);
}

// (A x)_i for both blocks and the two diagonals.
template <int DIM, class T>
__device__ __forceinline__ void apply_A(const LvK& g, const T* __restrict__ c,
                                        const typename V2<T>::type* __restrict__ x, int ix, int iy,
                                        int iz, T& y0, T& y1, T& d0, T& d1) {
  T w0[DIM == 3 ? 27 : 9], w1[DIM == 3 ? 27 : 9];
  stencil<DIM, T>(g, c, ix, iy, iz, w0, w1);
  y0 = 0;
  y1 = 0;
#pragma unroll
  for (int tz = 0; tz < (DIM == 3 ? 3 : 1); ++tz) {
    const int jz = DIM == 3 ? min(max(iz + tz - 1, 0), g.nn[2] - 1) : 0;
#pragma unroll
    for (int ty = 0; ty < 3; ++ty) {
      const int jy = min(max(iy + ty - 1, 0), g.nn[1] - 1);
#pragma unroll
      for (int tx = 0; tx < 3; ++tx) {
        const int jx = min(max(ix + tx - 1, 0), g.nn[0] - 1);
        const int t = tx + 3 * ty + 9 * tz;
        const auto xv = x[nidx(g, jx, jy, jz)];
        y0 += w0[t] * xv.x;
        y1 += w1[t] * xv.y;
      }
    }
  }
  const int tc = DIM == 3 ? 13 : 4;
  d0 = w0[tc];
  d1 = w1[tc];
}

template <int DIM, class T>
__device__ __forceinline__ void diag_only(const LvK& g, const T* __restrict__ c, int ix, int iy,
                                          int iz, T& d0, T& d1) {
  constexpr int NZ = DIM == 3 ? 2 : 1;
  T s = 0, n = 0;
#pragma unroll
  for (int bz = 0; bz < NZ; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int cx = ix - 1 + bx, cy = iy - 1 + by, cz = DIM == 3 ? iz - 1 + bz : 0;
        const bool e = cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1] &&
                       (DIM == 2 || (cz >= 0 && cz < g.n[2]));
        if (e) {
          s += c ? c[cx + (long long)g.n[0] * (cy + (long long)g.n[1] * cz)] : (T)1;
          n += (T)1;
        }
      }
  d0 = (T)g.Ae[0][0] * s;
  d1 = (T)g.Ae[1][0] * n;
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
        A.flux(g, G);
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

// coarse cell = mean of its 2^dim children
template <int DIM, class T>
__global__ void k_coarsen(LvK fg, LvK cg, const T* __restrict__ cf, T* __restrict__ cc) {
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

// dg[i] = phi-block diagonal of node i (the sum of the coefficients of its
// cells times the element-matrix diagonal entry)
template <int DIM, class T>
__global__ void __launch_bounds__(kT) k_diag(LvK g, const T* __restrict__ c, T* __restrict__ dg) {
  int ix, iy, iz;
  long long i;
  if (!plane_node(g, ix, iy, iz, i)) return;
  T d0, d1;
  diag_only<DIM, T>(g, c, ix, iy, iz, d0, d1);
  dg[i] = d0;
}

// num / d for a Jacobi diagonal d: times the hardware reciprocal estimate
// (1 ulp) in FP32, the IEEE quotient in FP64.
__device__ __forceinline__ float div_diag(float num, float d) { return num * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double div_diag(double num, double d) { return num / d; }

// Chebyshev step flags.  kWriteD: store the step's direction d (only a next
// step that reads it needs it).  kReadD: read the previous direction from d
// (a step whose alpha is 0, the first one, needs none).  kDIsX: the previous
// step started from x = 0, so its direction equals its iterate x_in.
constexpr int kWriteD = 1, kReadD = 2, kDIsX = 4;

// One Jacobi-Chebyshev step for both blocks:
//   d = alpha d + beta D^-1 (b - A x_in),  x_out = x_in + d.
// IN: 0 zero start (x_in = 0, b from the level array); 1 zero start with b
// read from the FP64 interleaved r64 and stored into b; 2 general step.
// OUT: 0 writes x_out; 1 writes the FP64 interleaved z64 (last step).
template <int DIM, class T, int IN, int OUT, int FL>
__global__ void __launch_bounds__(kT)
    k_smooth(LvK g, const T* __restrict__ c, typename V2<T>::type* __restrict__ b,
             const typename V2<T>::type* __restrict__ x_in, typename V2<T>::type* __restrict__ x_out,
             typename V2<T>::type* __restrict__ d, T al0, T al1, T be0, T be1,
             const double2* __restrict__ r64, double2* __restrict__ z64,
             const T* __restrict__ dgp) {
  int ix, iy, iz;
  long long i;
  if (!plane_node(g, ix, iy, iz, i)) return;
  typename V2<T>::type bb;
  if (IN == 1) {
    const double2 rv = r64[i];
    bb.x = (T)rv.x;
    bb.y = (T)rv.y;
    b[i] = bb;
  } else {
    bb = b[i];
  }
  T r0, r1, dg0, dg1, xi0 = 0, xi1 = 0, dn0, dn1;
  if (IN == 2) {
    T y0, y1;
    apply_A<DIM, T>(g, c, x_in, ix, iy, iz, y0, y1, dg0, dg1);
    r0 = bb.x - y0;
    r1 = bb.y - y1;
    const auto xv = x_in[i];
    xi0 = xv.x;
    xi1 = xv.y;
    typename V2<T>::type dv = xv;
    if (FL & kReadD) dv = d[i];
    if (!(FL & (kReadD | kDIsX))) dv.x = dv.y = 0;
    dn0 = (al0 == (T)0 ? (T)0 : al0 * dv.x) + div_diag(be0 * r0, dg0);
    dn1 = (al1 == (T)0 ? (T)0 : al1 * dv.y) + div_diag(be1 * r1, dg1);
  } else {
    // zero start: the diagonal only (phi block stored at set-up)
    dg0 = dgp[i];
    T n = (T)((ix - 1 >= 0 ? 1 : 0) + (ix < g.n[0] ? 1 : 0)) *
          (T)((iy - 1 >= 0 ? 1 : 0) + (iy < g.n[1] ? 1 : 0));
    if (DIM == 3) n *= (T)((iz - 1 >= 0 ? 1 : 0) + (iz < g.n[2] ? 1 : 0));
    dg1 = (T)g.Ae[1][0] * n;
    dn0 = div_diag(be0 * bb.x, dg0);
    dn1 = div_diag(be1 * bb.y, dg1);
  }
  typename V2<T>::type dn;
  dn.x = dn0;
  dn.y = dn1;
  if (OUT == 1) {
    z64[i] = make_double2((double)(xi0 + dn0), (double)(xi1 + dn1));
  } else {
    if (FL & kWriteD) d[i] = dn;
    typename V2<T>::type xo;
    xo.x = xi0 + dn0;
    xo.y = xi1 + dn1;
    x_out[i] = xo;
  }
}

template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_resid(LvK g, const T* __restrict__ c, const typename V2<T>::type* __restrict__ b,
            const typename V2<T>::type* __restrict__ x, typename V2<T>::type* __restrict__ r) {
  int ix, iy, iz;
  long long i;
  if (!plane_node(g, ix, iy, iz, i)) return;
  T y0, y1, d0, d1;
  apply_A<DIM, T>(g, c, x, ix, iy, iz, y0, y1, d0, d1);
  const auto bv = b[i];
  typename V2<T>::type o;
  o.x = bv.x - y0;
  o.y = bv.y - y1;
  r[i] = o;
}

// b_c[I] = sum_i P[i, I] r_f[i]: fine neighbours 2I-1, 2I, 2I+1 per axis with
// weights 1/2, 1, 1/2.
template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_restrict(LvK fg, LvK cg, const typename V2<T>::type* __restrict__ rf,
               typename V2<T>::type* __restrict__ bc) {
  int cx, cy, cz;
  long long I;
  if (!plane_node(cg, cx, cy, cz, I)) return;
  T a0 = 0, a1 = 0;
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
        const T w = (dx == 0 ? (T)1 : (T)0.5) * wy * wz;
        const auto v = rf[nidx(fg, fx, fy, fz)];
        a0 += w * v.x;
        a1 += w * v.y;
      }
    }
  }
  typename V2<T>::type o;
  o.x = a0;
  o.y = a1;
  bc[I] = o;
}

// The same restriction on 3-D levels by coarse tiles: a workgroup owns RCX x
// RCY coarse node columns and a chunk of kz coarse planes.  Each fine plane of
// the tile's footprint ((2 RCX + 1) x (2 RCY + 1) fine nodes, zero outside the
// mesh) is staged in LDS once and restricted along x and y there (weights 1/2,
// 1, 1/2); coarse plane Z then combines the fine planes 2Z - 1, 2Z, 2Z + 1
// with the z weights, the plane 2Z + 1 being carried to Z + 1.  Fine rows are
// read once, coalesced, instead of by up to 8 coarse threads each, and the
// next fine plane's loads are in flight while the current one is summed.
constexpr int RCX = 32, RCY = 8;

template <class T>
__global__ void __launch_bounds__(RCX * RCY)
    k_restrict3t(LvK fg, LvK cg, const typename V2<T>::type* __restrict__ rf,
                 typename V2<T>::type* __restrict__ bc, int kz) {
  using T2 = typename V2<T>::type;
  constexpr int FX = 2 * RCX + 1, FY = 2 * RCY + 1;
  const int tid = threadIdx.x;
  const int cx = tid % RCX, cy = tid / RCX;
  const int ntx = (cg.nn[0] + RCX - 1) / RCX, nty = (cg.nn[1] + RCY - 1) / RCY;
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int X0 = (tile % ntx) * RCX, Y0 = ((tile / ntx) % nty) * RCY;
  const int Z0 = (tile / (ntx * nty)) * kz;
  const int X = X0 + cx, Y = Y0 + cy;
  const bool inside = X < cg.nn[0] && Y < cg.nn[1];
  const int zend = min(Z0 + kz, cg.nn[2]);
  const long long fplane = (long long)fg.nn[0] * fg.nn[1];
  // The fine planes 2 Z0 - 1 .. 2 zend - 1 are streamed in order, each staged
  // in one of two LDS buffers from registers loaded while the previous plane
  // was restricted (the node offsets of a thread's slots do not change with z).
  constexpr int NQ = FX * FY, NR = (NQ + RCX * RCY - 1) / (RCX * RCY);
  __shared__ T2 fsd[2][FY][FX];
  int off[NR];
  bool okq[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int q = tid + j * RCX * RCY;
    const int fx = 2 * X0 - 1 + q % FX, fy = 2 * Y0 - 1 + q / FX;
    okq[j] = q < NQ && fx >= 0 && fx < fg.nn[0] && fy >= 0 && fy < fg.nn[1];
    off[j] = okq[j] ? fx + fg.nn[0] * fy : 0;
  }
  T2 pf[NR];
  auto fetch = [&](int z) {
    const bool zin = z >= 0 && z < fg.nn[2];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      pf[j].x = 0;
      pf[j].y = 0;
      if (zin && okq[j]) pf[j] = rf[off[j] + fplane * z];
    }
  };
  const int zlast = 2 * (zend - 1) + 1;  // last fine plane this chunk reads
  int buf = 0;
  // x-y restriction of fine plane z (0 for a plane outside the mesh), whose
  // values are in pf; the next plane's loads are issued before the sums
  auto plane = [&](int z) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int q = tid + j * RCX * RCY;
      if (q < NQ) fsd[buf][q / FX][q % FX] = pf[j];
    }
    lds_barrier();
    if (z + 1 <= zlast) fetch(z + 1);
    T2 p;
    p.x = 0;
    p.y = 0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const T wy = dy == 1 ? (T)1 : (T)0.5;
      T ax = 0, ay = 0;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const T wx = dx == 1 ? (T)1 : (T)0.5;
        const T2 v = fsd[buf][2 * cy + dy][2 * cx + dx];
        ax += wx * v.x;
        ay += wx * v.y;
      }
      p.x += wy * ax;
      p.y += wy * ay;
    }
    buf ^= 1;
    return p;
  };
  fetch(2 * Z0 - 1);
  T2 lo = plane(2 * Z0 - 1);
  for (int Z = Z0; Z < zend; ++Z) {
    const T2 mid = plane(2 * Z);
    const T2 hi = plane(2 * Z + 1);
    if (inside) {
      T2 o;
      o.x = (T)0.5 * lo.x + mid.x + (T)0.5 * hi.x;
      o.y = (T)0.5 * lo.y + mid.y + (T)0.5 * hi.y;
      bc[X + cg.nn[0] * (long long)Y + (long long)cg.nn[0] * cg.nn[1] * Z] = o;
    }
    lo = hi;
  }
}

// x_f[i] += sum_I P[i, I] e_c[I], by coarse node: the thread of coarse node
// (cx, cy, cz) updates the fine nodes 2c + o, o in {0, 1}^DIM, that exist.  A
// fine node with odd coordinates along m axes takes the sum of its 2^m coarse
// neighbours times 2^-m.  Neighbouring threads touch neighbouring fine pairs,
// so the fine rows are read and written once, coalesced.
template <int DIM, class T>
__global__ void __launch_bounds__(kT)
    k_prolong_add(LvK fg, LvK cg, const typename V2<T>::type* __restrict__ ec,
                  typename V2<T>::type* __restrict__ xf) {
  using T2 = typename V2<T>::type;
  int cx, cy, cz;
  long long I;
  if (!plane_node(cg, cx, cy, cz, I)) return;
  const bool hx = cx + 1 < cg.nn[0], hy = cy + 1 < cg.nn[1];
  const bool hz = DIM == 3 && cz + 1 < cg.nn[2];
  const long long sy = cg.nn[0], sz = (long long)cg.nn[0] * cg.nn[1];
  // coarse corner values e[dz][dy][dx]; absent corners are never used
  T2 e[2][2][2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const bool ok = (dx == 0 || hx) && (dy == 0 || hy) && (dz == 0 || hz);
        e[dz][dy][dx] = ok ? ec[I + dx + dy * sy + dz * sz] : ec[I];
      }
  const long long fsy = fg.nn[0], fsz = (long long)fg.nn[0] * fg.nn[1];
  const long long f0 = 2LL * cx + fsy * (2LL * cy) + (DIM == 3 ? fsz * (2LL * cz) : 0LL);
#pragma unroll
  for (int oz = 0; oz < (DIM == 3 ? 2 : 1); ++oz) {
    if (oz == 1 && !hz) continue;
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
      if (oy == 1 && !hy) continue;
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        if (ox == 1 && !hx) continue;
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int kz = 0; kz <= oz; ++kz)
#pragma unroll
          for (int ky = 0; ky <= oy; ++ky)
#pragma unroll
            for (int kx = 0; kx <= ox; ++kx) {
              a0 += e[kz][ky][kx].x;
              a1 += e[kz][ky][kx].y;
            }
        const T w = (ox ? (T)0.5 : (T)1) * (oy ? (T)0.5 : (T)1) * (oz ? (T)0.5 : (T)1);
        const long long i = f0 + ox + fsy * oy + fsz * oz;
        T2 x = xf[i];
        x.x += w * a0;
        x.y += w * a1;
        xf[i] = x;
      }
    }
  }
}


// ----------------------------------------------------------------- 2.5-D stencil kernels (3-D)
// A workgroup owns a 32 x 8 tile of node columns and marches through kz node
// planes in z.  The iterate x (tile plus a one-node halo) is staged plane by
// plane in a 3-plane LDS ring and the cell coefficients in a 2-plane ring, so
// each value is fetched from memory about once per sweep instead of once per
// stencil use.  kz is chosen per level: long marches on the finest level, short
// ones on coarse levels, whose few tiles would otherwise leave most compute
// units idle while a handful of workgroups step through their planes.
#ifndef PF_SBX
#define PF_SBX 32
#endif
#ifndef PF_SBY
#define PF_SBY 8
#endif
constexpr int SBX = PF_SBX, SBY = PF_SBY, SKZ = 32;
#ifndef PF_TILED_MIN_GROUPS
#define PF_TILED_MIN_GROUPS 4096
#endif
constexpr long long kTiledMinGroups = PF_TILED_MIN_GROUPS;

inline bool use_tiled(const LvK& k, int dim) { return dim == 3 && k.nn[0] >= SBX && k.nn[1] >= SBY; }

// z-march length: the longest power of two up to SKZ that still gives at
// least min_groups workgroups
inline int tiled_kz(const LvK& k, long long min_groups) {
  const long long tiles = (long long)((k.nn[0] + SBX - 1) / SBX) * ((k.nn[1] + SBY - 1) / SBY);
  int kz = SKZ;
  while (kz > 1 && tiles * ((k.nn[2] + kz - 1) / kz) < min_groups) kz /= 2;
  return kz;
}

// The workgroup target of the z-march choice; the environment variable
// PF_GMG_TILE_GROUPS (a positive integer, read when the hierarchy is built)
// overrides it, which lets small meshes exercise long z-marches.
inline long long tiled_min_groups() {
  const char* e = std::getenv("PF_GMG_TILE_GROUPS");
  if (e && *e) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end && *end == '\0' && v > 0) return v;
  }
  return kTiledMinGroups;
}

// Arguments of the tiled kernel.  al, be: the step's Chebyshev coefficients
// per block.  OP 3/4 also take the first (zero-start) step's betas zb, the
// stored phi-block diagonal dg and, for OP 3, the FP64 right-hand side r64
// whose FP32 copy they write to bout.
template <class T>
struct StArgs {
  using T2 = typename V2<T>::type;
  const T* c;
  const T2* b;
  const T2* x;
  T2* out;
  T2* d;
  T al0, al1, be0, be1;
  double2* z64;
  int kz;
  T zb0, zb1;
  const double2* r64;
  T2* bout;
  const T* dg;
};

// OP 0: r = b - A x.  OP 1: Chebyshev step (x_out, d).  OP 2: Chebyshev step
// writing the FP64 interleaved z64 (last step of the V-cycle).  OP 3/4: the
// first two steps from x = 0 in one sweep: the zero-start iterate
// x1 = zb D^-1 b is formed while the halo planes are staged (from the FP64 r64,
// OP 3, or from b, OP 4) and the second step is taken on it; its direction is
// x1 itself.
template <class T, int OP, int FL>
__global__ void __launch_bounds__(SBX * SBY) k_stencil3(LvK g, StArgs<T> A) {
  using T2 = typename V2<T>::type;
  const T* __restrict__ c = A.c;
  const T2* __restrict__ b = A.b;
  const T2* __restrict__ x = A.x;
  T2* __restrict__ out = A.out;
  T2* __restrict__ d = A.d;
  const T al0 = A.al0, al1 = A.al1, be0 = A.be0, be1 = A.be1;
  double2* __restrict__ z64 = A.z64;
  const int kz = A.kz;
  constexpr bool ZS = OP >= 3;  // fused zero start
  __shared__ T2 xs[3][SBY + 2][SBX + 2];
  __shared__ T cs[2][SBY + 1][SBX + 1];
  // zero start in FP32: the right-hand side of the staged planes is kept in
  // LDS, so that the centre value needs no second global read (1 % faster
  // cycle; in FP64 the extra registers cost more than the read)
  constexpr bool ZSB = OP >= 3 && sizeof(T) == 4;
  __shared__ T2 bs[ZSB ? 3 : 1][ZSB ? SBY + 2 : 1][ZSB ? SBX + 2 : 1];
  const int tid = threadIdx.x;
  const int tx = tid % SBX, ty = tid / SBX;
  // 1-D grid of tiles (x fastest), dealt to the XCDs in contiguous runs
  const int ntx = (g.nn[0] + SBX - 1) / SBX, nty = (g.nn[1] + SBY - 1) / SBY;
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * SBX, y0 = ((tile / ntx) % nty) * SBY, z0 = (tile / (ntx * nty)) * kz;
  const int ix = x0 + tx, iy = y0 + ty;
  const bool inside = ix < g.nn[0] && iy < g.nn[1];
  const int zend = min(z0 + kz, g.nn[2]);

  // Software pipeline: the halo values of the next planes are fetched into
  // registers (at most 2 per thread each) while the current plane is computed,
  // and stored to the LDS ring at the top of the next iteration.  Each thread's
  // halo slots q = tid + j * 256 and their in-plane offsets do not change with z.
  constexpr int NQX = (SBX + 2) * (SBY + 2), NQC = (SBX + 1) * (SBY + 1);
  constexpr int NX = (NQX + SBX * SBY - 1) / (SBX * SBY);
  constexpr int NC = (NQC + SBX * SBY - 1) / (SBX * SBY);
  const long long plane_n = (long long)g.nn[0] * g.nn[1];
  const long long plane_c = (long long)g.n[0] * g.n[1];
  int offx[NX], offc[NC];
  bool okx[NX], okc[NC];
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const int q = tid + j * SBX * SBY;
    const int gx = x0 - 1 + q % (SBX + 2), gy = y0 - 1 + q / (SBX + 2);
    okx[j] = q < NQX && gx >= 0 && gx < g.nn[0] && gy >= 0 && gy < g.nn[1];
    offx[j] = okx[j] ? gx + g.nn[0] * gy : 0;
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int q = tid + j * SBX * SBY;
    const int cx = x0 - 1 + q % (SBX + 1), cy = y0 - 1 + q / (SBX + 1);
    okc[j] = q < NQC && cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1];
    offc[j] = okc[j] ? cx + g.n[0] * cy : 0;
  }
  // a fetched halo node plane, held in registers until stored to the ring;
  // zero start: also the raw right-hand side and diagonal of its nodes and
  // whether they are in the mesh
  struct XPlane {
    T2 rx[NX];
    double2 rr[OP == 3 ? NX : 1];
    T rdg[ZS ? NX : 1];
    bool rin[ZS ? NX : 1];
    int fz;
  };
  XPlane xa, xb;  // xb: the prologue's second plane only
  T rc[NC];
  // zero start: the in-plane cell counts of the halo nodes (u-block diagonal)
  T cxy[ZS ? NX : 1];
  if constexpr (ZS) {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int q = tid + j * SBX * SBY;
      const int gx = x0 - 1 + q % (SBX + 2), gy = y0 - 1 + q / (SBX + 2);
      cxy[j] = (T)((gx - 1 >= 0 ? 1 : 0) + (gx < g.n[0] ? 1 : 0)) *
               (T)((gy - 1 >= 0 ? 1 : 0) + (gy < g.n[1] ? 1 : 0));
    }
  }
  auto fetch_x = [&](XPlane& f, int z) {
    const bool zin = z >= 0 && z < g.nn[2];
    const long long po = plane_n * (zin ? z : 0);
    f.fz = z;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      f.rx[j].x = 0;
      f.rx[j].y = 0;
      if constexpr (ZS) {
        f.rin[j] = zin && okx[j];
        f.rdg[j] = 1;
        if constexpr (OP == 3) f.rr[j] = make_double2(0.0, 0.0);
        if (f.rin[j]) {
          f.rdg[j] = A.dg[po + offx[j]];
          if constexpr (OP == 3) f.rr[j] = A.r64[po + offx[j]];
          else f.rx[j] = b[po + offx[j]];
        }
      } else {
        if (zin && okx[j]) f.rx[j] = x[po + offx[j]];
      }
    }
  };
  auto store_x = [&](const XPlane& f, int slot) {
    T czf = 1;
    if constexpr (ZS) czf = (T)((f.fz - 1 >= 0 ? 1 : 0) + (f.fz < g.n[2] ? 1 : 0));
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int q = tid + j * SBX * SBY;
      T2 v = f.rx[j];
      if constexpr (ZS) {
        // x1 = zb D^-1 b at the halo node (0 outside the mesh)
        T2 bv = f.rx[j];
        if constexpr (OP == 3) {
          bv.x = (T)f.rr[j].x;
          bv.y = (T)f.rr[j].y;
        }
        const T dg1 = (T)g.Ae[1][0] * (cxy[j] * czf);
        v.x = f.rin[j] ? div_diag(A.zb0 * bv.x, f.rdg[j]) : (T)0;
        v.y = f.rin[j] ? div_diag(A.zb1 * bv.y, dg1) : (T)0;
        if (ZSB && q < NQX) (&bs[slot][0][0])[q] = bv;
      }
      if (q < NQX) (&xs[slot][0][0])[q] = v;
    }
  };
  auto fetch_c = [&](int zc) {
    const bool zin = zc >= 0 && zc < g.n[2];
    const T* cpl = c + plane_c * (zin ? zc : 0);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      rc[j] = 0;
      if (zin && okc[j]) rc[j] = cpl[offc[j]];
    }
  };
  auto store_c = [&](int slot) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int q = tid + j * SBX * SBY;
      if (q < NQC) (&cs[slot][0][0])[q] = rc[j];
    }
  };
  // ring slots: node plane z lives in slot (z - z0 + 1) % 3, cell plane zc in
  // (zc - z0 + 1) & 1.  The prologue's three planes are loaded together.
  fetch_x(xa, z0 - 1);
  fetch_x(xb, z0);
  fetch_c(z0 - 1);
  store_x(xa, 0);
  store_x(xb, 1);
  store_c(0);
  fetch_x(xa, z0 + 1);
  fetch_c(z0);
  const long long ibase = ix + (long long)g.nn[0] * iy;
  // FP32 residual and Chebyshev steps: the node's own right-hand side one
  // plane ahead in registers, so that the compute phase waits on one global
  // read fewer (measured: the last step, which also reads d and writes FP64,
  // and the FP64 sweeps are slower with it; steps that both read and write d
  // would lose a wave per SIMD to the two extra registers)
  constexpr bool kPreB = sizeof(T) == 4 && OP <= 1 && FL != (kReadD | kWriteD);
  T2 nb{};
  auto fetch_b = [&](int z) {
    if constexpr (kPreB) {
      if (inside) nb = b[ibase + plane_n * z];
    }
  };
  fetch_b(z0);
  for (int z = z0; z < zend; ++z) {
    const int k = z - z0;
    const int sm = k % 3, s0 = (k + 1) % 3, sp = (k + 2) % 3;
    const int cm = k & 1, cp = cm ^ 1;
    store_x(xa, sp);  // plane z + 1
    store_c(cp);      // cell plane z
    lds_barrier();
    const T2 cur_b = nb;
    if (z + 1 < zend) {
      fetch_x(xa, z + 2);
      fetch_c(z + 1);
      fetch_b(z + 1);
    }
    (void)cur_b;
    if (inside) {
      // y = A x for both blocks, grouped by the corner-difference pattern p
      // of the stencil offset (bit 0: x offset, 1: y, 2: z):
      //   y0 = sum_p Ae0[p] sum_{t in p} s_t x0_t, s_t the sum of the cell
      //        coefficients shared by the node and node t (cells outside the
      //        mesh are staged as 0, so missing neighbours drop out);
      //   y1 = sum_p Ae1[p] f_p sum_{t in p} x1_t, f_p the product over the
      //        axes not in p of the number of cells along that axis (1 or 2);
      //        along the axes in p the count is 0 or 1 and the neighbour value
      //        is staged as 0 exactly when it is 0.
      T cc[2][2][2];  // [bz][by][bx]
#pragma unroll
      for (int by = 0; by < 2; ++by)
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
          cc[0][by][bx] = cs[cm][ty + by][tx + bx];
          cc[1][by][bx] = cs[cp][ty + by][tx + bx];
        }
      T Sz[2][2], Sy[2][2], Sx[2][2];  // pair sums along z, y, x
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          Sz[u][v] = cc[0][u][v] + cc[1][u][v];  // [by][bx]
          Sy[u][v] = cc[u][0][v] + cc[u][1][v];  // [bz][bx]
          Sx[u][v] = cc[u][v][0] + cc[u][v][1];  // [bz][by]
        }
      T Syz[2], Sxz[2], Sxy[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        Syz[u] = Sz[0][u] + Sz[1][u];  // [bx]
        Sxz[u] = Sz[u][0] + Sz[u][1];  // [by]
        Sxy[u] = Sx[u][0] + Sx[u][1];  // [bz]
      }
      const T Sall = Syz[0] + Syz[1];
      const int sl[3] = {sm, s0, sp};
      auto X = [&](int dx, int dy, int dz) { return xs[sl[dz]][ty + dy][tx + dx]; };
      // phi block, per pattern
      T P0[8];
      P0[0] = Sall * X(1, 1, 1).x;
      P0[1] = Syz[0] * X(0, 1, 1).x + Syz[1] * X(2, 1, 1).x;
      P0[2] = Sxz[0] * X(1, 0, 1).x + Sxz[1] * X(1, 2, 1).x;
      P0[4] = Sxy[0] * X(1, 1, 0).x + Sxy[1] * X(1, 1, 2).x;
      P0[3] = 0;
      P0[5] = 0;
      P0[6] = 0;
      P0[7] = 0;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          P0[3] += Sz[u][v] * X(2 * v, 2 * u, 1).x;  // [by][bx]
          P0[5] += Sy[u][v] * X(2 * v, 1, 2 * u).x;  // [bz][bx]
          P0[6] += Sx[u][v] * X(1, 2 * v, 2 * u).x;  // [bz][by]
#pragma unroll
          for (int w = 0; w < 2; ++w) P0[7] += cc[u][v][w] * X(2 * w, 2 * v, 2 * u).x;
        }
      // u block: sums over x first, then y, then z
      T Xo[3][3], Xc[3][3];  // [dy][dz]
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          Xo[dy][dz] = X(0, dy, dz).y + X(2, dy, dz).y;
          Xc[dy][dz] = X(1, dy, dz).y;
        }
      T G1[8];
      {
        T Yoo[3], Yoc[3], Yco[3], Ycc[3];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
          Yoo[dz] = Xo[0][dz] + Xo[2][dz];
          Yoc[dz] = Xo[1][dz];
          Yco[dz] = Xc[0][dz] + Xc[2][dz];
          Ycc[dz] = Xc[1][dz];
        }
        G1[0] = Ycc[1];
        G1[1] = Yoc[1];
        G1[2] = Yco[1];
        G1[3] = Yoo[1];
        G1[4] = Ycc[0] + Ycc[2];
        G1[5] = Yoc[0] + Yoc[2];
        G1[6] = Yco[0] + Yco[2];
        G1[7] = Yoo[0] + Yoo[2];
      }
      const T cx = (T)((ix - 1 >= 0 ? 1 : 0) + (ix < g.n[0] ? 1 : 0));
      const T cy = (T)((iy - 1 >= 0 ? 1 : 0) + (iy < g.n[1] ? 1 : 0));
      const T cz = (T)((z - 1 >= 0 ? 1 : 0) + (z < g.n[2] ? 1 : 0));
      const T cxy = cx * cy;
      T f[8];
      f[0] = cxy * cz;
      f[1] = cy * cz;
      f[2] = cx * cz;
      f[3] = cz;
      f[4] = cxy;
      f[5] = cy;
      f[6] = cx;
      f[7] = 1;
      T y0 = 0, y1 = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        y0 += (T)g.Ae[0][q] * P0[q];
        y1 += ((T)g.Ae[1][q] * f[q]) * G1[q];
      }
      const T dg0 = (T)g.Ae[0][0] * Sall, dg1 = (T)g.Ae[1][0] * f[0];
      const long long i = ibase + plane_n * z;
      T2 bb;
      if constexpr (ZSB) {
        bb = bs[s0][ty + 1][tx + 1];
        if constexpr (OP == 3) A.bout[i] = bb;
      } else if constexpr (OP == 3) {
        const double2 rv = A.r64[i];
        bb.x = (T)rv.x;
        bb.y = (T)rv.y;
        A.bout[i] = bb;
      } else {
        bb = kPreB ? cur_b : b[i];
      }
      const T r0 = bb.x - y0, r1 = bb.y - y1;
      if (OP == 0) {
        T2 o;
        o.x = r0;
        o.y = r1;
        out[i] = o;
      } else {
        const T2 xi = xs[s0][ty + 1][tx + 1];
        T2 dv = xi;
        if (FL & kReadD) dv = d[i];
        if (!ZS && !(FL & (kReadD | kDIsX))) dv.x = dv.y = 0;
        const T dn0 = (al0 == (T)0 ? (T)0 : al0 * dv.x) + div_diag(be0 * r0, dg0);
        const T dn1 = (al1 == (T)0 ? (T)0 : al1 * dv.y) + div_diag(be1 * r1, dg1);
        if (OP == 2) {
          z64[i] = make_double2((double)(xi.x + dn0), (double)(xi.y + dn1));
        } else {
          T2 dn, xo;
          dn.x = dn0;
          dn.y = dn1;
          xo.x = xi.x + dn0;
          xo.y = xi.y + dn1;
          if (FL & kWriteD) d[i] = dn;
          out[i] = xo;
        }
      }
    }
    // this plane's LDS reads done before the next plane is staged; its global
    // stores are left in flight (no thread reads another's outputs here)
    lds_barrier();
  }
}

// Coarsest level: COARSE_DEGREE Chebyshev steps for both blocks by one
// workgroup, iterates in LDS.  al/be: per-step coefficients, [step][block].
template <int DIM, class T>
__global__ void __launch_bounds__(1024)
    k_coarse(LvK g, const T* __restrict__ c, const typename V2<T>::type* __restrict__ b,
             typename V2<T>::type* __restrict__ x_res, const double* __restrict__ coef) {
  using T2 = typename V2<T>::type;
  __shared__ T2 xs[2][kCoarseLdsNodes];
  __shared__ T2 ds[kCoarseLdsNodes];
  // the right-hand side and the cell coefficients are read from memory once:
  // every step then touches LDS only (a grid of n nodes has fewer than n cells)
  __shared__ T2 bs[kCoarseLdsNodes];
  __shared__ T cs[kCoarseLdsNodes];
  const int n = (int)g.nnodes;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    bs[i] = b[i];
    if (i < g.ncells) cs[i] = c[i];
  }
  __syncthreads();
  for (int k = 0; k < kCoarseDegree; ++k) {
    const int src = k & 1, dst = src ^ 1;
    const T al0 = (T)coef[4 * k + 0], al1 = (T)coef[4 * k + 1];
    const T be0 = (T)coef[4 * k + 2], be1 = (T)coef[4 * k + 3];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      int ix, iy, iz;
      node_ijk<DIM>(g, i, ix, iy, iz);
      const T2 bb = bs[i];
      T dn0, dn1, x0 = 0, x1 = 0;
      if (k == 0) {
        T dg0, dg1;
        diag_only<DIM, T>(g, cs, ix, iy, iz, dg0, dg1);
        dn0 = div_diag(be0 * bb.x, dg0);
        dn1 = div_diag(be1 * bb.y, dg1);
      } else {
        T w0[DIM == 3 ? 27 : 9], w1[DIM == 3 ? 27 : 9];
        stencil<DIM, T>(g, cs, ix, iy, iz, w0, w1);
        T y0 = 0, y1 = 0;
#pragma unroll
        for (int tz = 0; tz < (DIM == 3 ? 3 : 1); ++tz) {
          const int jz = DIM == 3 ? min(max(iz + tz - 1, 0), g.nn[2] - 1) : 0;
#pragma unroll
          for (int ty = 0; ty < 3; ++ty) {
            const int jy = min(max(iy + ty - 1, 0), g.nn[1] - 1);
#pragma unroll
            for (int tx = 0; tx < 3; ++tx) {
              const int jx = min(max(ix + tx - 1, 0), g.nn[0] - 1);
              const int t = tx + 3 * ty + 9 * tz;
              const T2 xv = xs[src][(int)nidx(g, jx, jy, jz)];
              y0 += w0[t] * xv.x;
              y1 += w1[t] * xv.y;
            }
          }
        }
        const int tc = DIM == 3 ? 13 : 4;
        const T2 xv = xs[src][i];
        x0 = xv.x;
        x1 = xv.y;
        const T2 dv = ds[i];
        dn0 = al0 * dv.x + be0 * (bb.x - y0) / w0[tc];
        dn1 = al1 * dv.y + be1 * (bb.y - y1) / w1[tc];
      }
      T2 dn, xo;
      dn.x = dn0;
      dn.y = dn1;
      xo.x = x0 + dn0;
      xo.y = x1 + dn1;
      ds[i] = dn;
      xs[dst][i] = xo;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) x_res[i] = xs[kCoarseDegree & 1][i];
}

// The same solve for coarsest grids of at most kCoarseSmall nodes: one node
// per thread, whose 27 (9) stencil weights and neighbour indices are formed
// once instead of at every step.  Same operations on the same values in the
// same order as k_coarse: same bits.
constexpr int kCoarseSmall = 256;
template <int DIM, class T>
__global__ void __launch_bounds__(kCoarseSmall)
    k_coarse_small(LvK g, const T* __restrict__ c, const typename V2<T>::type* __restrict__ b,
                   typename V2<T>::type* __restrict__ x_res, const double* __restrict__ coef) {
  using T2 = typename V2<T>::type;
  constexpr int NW = DIM == 3 ? 27 : 9;
  __shared__ T2 xs[2][kCoarseSmall];
  __shared__ T cs[kCoarseSmall];
  const int n = (int)g.nnodes;
  const int i = threadIdx.x;
  const bool own = i < n;
  if (i < g.ncells) cs[i] = c[i];
  __syncthreads();
  T2 bb{};
  T w0[NW], w1[NW], dg0 = 1, dg1 = 1;
  int nb[NW];
  if (own) {
    bb = b[i];
    int ix, iy, iz;
    node_ijk<DIM>(g, i, ix, iy, iz);
    diag_only<DIM, T>(g, cs, ix, iy, iz, dg0, dg1);
    stencil<DIM, T>(g, cs, ix, iy, iz, w0, w1);
#pragma unroll
    for (int tz = 0; tz < (DIM == 3 ? 3 : 1); ++tz) {
      const int jz = DIM == 3 ? min(max(iz + tz - 1, 0), g.nn[2] - 1) : 0;
#pragma unroll
      for (int ty = 0; ty < 3; ++ty) {
        const int jy = min(max(iy + ty - 1, 0), g.nn[1] - 1);
#pragma unroll
        for (int tx = 0; tx < 3; ++tx) {
          const int jx = min(max(ix + tx - 1, 0), g.nn[0] - 1);
          nb[tx + 3 * ty + 9 * tz] = (int)nidx(g, jx, jy, jz);
        }
      }
    }
  }
  T2 dv{}, xv{};  // this node's direction and iterate
  for (int k = 0; k < kCoarseDegree; ++k) {
    const int src = k & 1, dst = src ^ 1;
    const T al0 = (T)coef[4 * k + 0], al1 = (T)coef[4 * k + 1];
    const T be0 = (T)coef[4 * k + 2], be1 = (T)coef[4 * k + 3];
    if (own) {
      T dn0, dn1, x0 = 0, x1 = 0;
      if (k == 0) {
        dn0 = div_diag(be0 * bb.x, dg0);
        dn1 = div_diag(be1 * bb.y, dg1);
      } else {
        T y0 = 0, y1 = 0;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
          const T2 xn = xs[src][nb[t]];
          y0 += w0[t] * xn.x;
          y1 += w1[t] * xn.y;
        }
        const int tc = DIM == 3 ? 13 : 4;
        x0 = xv.x;
        x1 = xv.y;
        dn0 = al0 * dv.x + be0 * (bb.x - y0) / w0[tc];
        dn1 = al1 * dv.y + be1 * (bb.y - y1) / w1[tc];
      }
      dv.x = dn0;
      dv.y = dn1;
      xv.x = x0 + dn0;
      xv.y = x1 + dn1;
      xs[dst][i] = xv;
    }
    __syncthreads();
  }
  if (own) x_res[i] = xv;
}

__global__ void k_jacobi(Geo G, const double* __restrict__ c, const double2* __restrict__ r,
                         double2* __restrict__ z, double ae0, double ae1) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= G.n_nodes) return;
  LvK g{};
  for (int k = 0; k < 3; ++k) {
    g.n[k] = G.n[k];
    g.nn[k] = G.nn[k];
  }
  g.Ae[0][0] = ae0;
  g.Ae[1][0] = ae1;
  int ix, iy, iz;
  double d0, d1;
  if (G.dim == 3) {
    node_ijk<3>(g, i, ix, iy, iz);
    diag_only<3, double>(g, c, ix, iy, iz, d0, d1);
  } else {
    node_ijk<2>(g, i, ix, iy, iz);
    diag_only<2, double>(g, c, ix, iy, iz, d0, d1);
  }
  const double2 a = r[i];
  z[i] = make_double2(a.x / d0, a.y / d1);
}

template <class T>
__global__ void k_split(const double2* __restrict__ r, typename V2<T>::type* __restrict__ b,
                        long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double2 v = r[i];
  typename V2<T>::type o;
  o.x = (T)v.x;
  o.y = (T)v.y;
  b[i] = o;
}

template <class T>
__global__ void k_merge(const typename V2<T>::type* __restrict__ x, double2* __restrict__ z,
                        long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const auto v = x[i];
  z[i] = make_double2((double)v.x, (double)v.y);
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

// Chebyshev step coefficients (alpha_k, beta_k), k = 0 .. degree-1, for the
// iteration d_k = alpha_k d_{k-1} + beta_k D^-1 r_k on [lo, hi].
void cheb_coefs(double lo, double hi, int degree, double* al, double* be) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int k = 0; k < degree; ++k) {
    if (k == 0) {
      al[k] = 0.0;
      be[k] = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      al[k] = rn * rho;
      be[k] = 2.0 * rn / delta;
      rho = rn;
    }
  }
}

template <class T>
int hier_alloc(pf_problem* pb, Hier<T>& H) {
  const Geo& G = pb->geo;
  int n[3] = {G.n[0], G.n[1], G.dim == 3 ? G.n[2] : 1};
  double h[3] = {G.h[0], G.h[1], G.h[2]};
  const long long min_groups = tiled_min_groups();
  H.lv.clear();
  while (true) {
    Level<T> L{};
    for (int k = 0; k < 3; ++k) {
      L.k.n[k] = (k < G.dim) ? n[k] : 1;
      L.k.nn[k] = (k < G.dim) ? n[k] + 1 : 1;
      L.h[k] = h[k];
    }
    L.k.nnodes = (long long)L.k.nn[0] * L.k.nn[1] * L.k.nn[2];
    L.k.ncells = (long long)L.k.n[0] * L.k.n[1] * L.k.n[2];
    // coarser levels march further, for half the workgroups: their chunks are
    // short, and the halo planes every chunk re-reads cost more there than
    // the compute units left idle (the 129^3 level of 256^3: 2 -> 4 planes)
    L.kz = use_tiled(L.k, G.dim) ? tiled_kz(L.k, H.lv.empty() ? min_groups : (min_groups + 1) / 2) : 0;
    const size_t nb = (size_t)L.k.nnodes * sizeof(typename V2<T>::type);
    // registered before allocating, so that hier_free releases a partial level
    H.lv.push_back(L);
    Level<T>& M = H.lv.back();
    if (hipMalloc(&M.c, (size_t)M.k.ncells * sizeof(T)) != hipSuccess) return PF_ERR_OOM;
    typename V2<T>::type** bufs[] = {&M.xa, &M.xb, &M.b, &M.r, &M.d};
    for (auto p : bufs)
      if (hipMalloc(p, nb) != hipSuccess) return PF_ERR_OOM;
    if (hipMalloc(&M.dg, (size_t)M.k.nnodes * sizeof(T)) != hipSuccess) return PF_ERR_OOM;
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
  if (hipMalloc(&H.coarse_dev, sizeof(H.coarse_host)) != hipSuccess) return PF_ERR_OOM;
  H.allocated = true;
  return PF_OK;
}

template <class T>
hipError_t hier_free(Hier<T>& H) {
  hipError_t first = hipSuccess;
  for (auto& L : H.lv) {
    void* bufs[] = {L.c, L.xa, L.xb, L.b, L.r, L.d, L.dg};
    for (void* p : bufs) {
      if (!p) continue;
      const hipError_t e = hipFree(p);
      if (first == hipSuccess) first = e;
    }
  }
  if (H.coarse_dev) {
    const hipError_t e = hipFree(H.coarse_dev);
    if (first == hipSuccess) first = e;
    H.coarse_dev = nullptr;
  }
  H.lv.clear();
  H.allocated = false;
  return first;
}

// Mass and stiffness scales of the two blocks: phi block (1/dt) M_c +
// theta K_c; u block (1/dt) M + theta D K (thermal) or (1+k)/(2 dt) M +
// theta D K (alloy, the one-sided mobility at its liquid value).  Free
// growth: (1/dt) M_c + theta beta Gamma K_c and (1/dt) M + theta alpha K.
void block_scales(const pf_problem* pb, double* sm, double* sk) {
  const double idt = 1.0 / pb->params.dt, th = pb->params.theta;
  sm[0] = idt;
  sk[0] = th;
  sm[1] = pb->model == 1 ? 0.5 * (1.0 + pb->alloy.k) * idt : idt;
  sk[1] = th * pb->params.D;
  if (pb->model == 2) {
    sk[0] = th * pb->fg.beta * pb->fg.Gamma;
    sk[1] = th * pb->fg.alpha;
  }
}

template <int DIM, class T>
int hier_setup(pf_problem* pb, Hier<T>& H, const double* c0_dev, hipStream_t s) {
  double sm[2], sk[2];
  block_scales(pb, sm, sk);
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level<T>& L = H.lv[l];
    for (int f = 0; f < 2; ++f) {
      element_table(DIM, L.h, sm[f], sk[f], L.k.Ae[f]);
      symbol_extremes(DIM, L.h, sm[f], sk[f], &L.lmin[f], &L.lmax[f]);
    }
    if (l == 0) {
      hipLaunchKernelGGL((k_convert<T>), dim3(blocks(L.k.ncells)), dim3(kT), 0, s, c0_dev, L.c,
                         L.k.ncells);
    } else {
      hipLaunchKernelGGL((k_coarsen<DIM, T>), dim3(blocks(L.k.ncells)), dim3(kT), 0, s,
                         H.lv[l - 1].k, L.k, (const T*)H.lv[l - 1].c, L.c);
    }
    PF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_diag<DIM, T>), plane_grid(L.k), dim3(kT), 0, s, L.k, (const T*)L.c, L.dg);
    PF_HIP_CHECK(hipGetLastError());
  }
  // per-step coefficients of the coarsest solve, [step][alpha0, alpha1, beta0, beta1]
  const Level<T>& C = H.lv.back();
  for (int f = 0; f < 2; ++f) {
    double a[kCoarseDegree], b[kCoarseDegree];
    cheb_coefs(C.lmin[f], kChebSafety * C.lmax[f], kCoarseDegree, a, b);
    for (int k = 0; k < kCoarseDegree; ++k) {
      H.coarse_host[4 * k + f] = a[k];
      H.coarse_host[4 * k + 2 + f] = b[k];
    }
  }
  PF_HIP_CHECK(hipMemcpy(H.coarse_dev, H.coarse_host, sizeof(H.coarse_host), hipMemcpyHostToDevice));
  return PF_OK;
}

// Levels whose x rows span at least one tile use the 2.5-D kernels.
template <class T>
inline dim3 tiled_grid(const Level<T>& L) {
  const LvK& k = L.k;
  return dim3((unsigned)(((k.nn[0] + SBX - 1) / SBX) * ((k.nn[1] + SBY - 1) / SBY) *
                         ((k.nn[2] + L.kz - 1) / L.kz)));
}

template <int DIM, class T, int IN, int OUT, int FL>
int smooth_step(Level<T>& L, const typename V2<T>::type* x_in, typename V2<T>::type* x_out,
                const double* al, const double* be, int k, const double* r64, double* z64,
                hipStream_t s) {
  if (IN == 2 && L.kz > 0) {
    constexpr int OP = OUT == 1 ? 2 : 1;
    StArgs<T> A{};
    A.c = L.c;
    A.b = L.b;
    A.x = x_in;
    A.out = x_out;
    A.d = L.d;
    A.al0 = (T)al[2 * k];
    A.al1 = (T)al[2 * k + 1];
    A.be0 = (T)be[2 * k];
    A.be1 = (T)be[2 * k + 1];
    A.z64 = reinterpret_cast<double2*>(z64);
    A.kz = L.kz;
    hipLaunchKernelGGL((k_stencil3<T, OP, FL>), tiled_grid(L), dim3(SBX * SBY), 0, s, L.k, A);
    PF_HIP_CHECK(hipGetLastError());
    return PF_OK;
  }
  hipLaunchKernelGGL((k_smooth<DIM, T, IN, OUT, FL>), plane_grid(L.k), dim3(kT), 0, s, L.k,
                     (const T*)L.c, L.b, x_in, x_out, L.d, (T)al[2 * k], (T)al[2 * k + 1],
                     (T)be[2 * k], (T)be[2 * k + 1], reinterpret_cast<const double2*>(r64),
                     reinterpret_cast<double2*>(z64), (const T*)L.dg);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

// coefficients of the level's degree-2 smoother, [k][block]
template <class T>
void smoother_coefs(const Level<T>& L, double* al, double* be) {
  for (int f = 0; f < 2; ++f) {
    const double hi = kChebSafety * L.lmax[f];
    double lo = L.lmax[f] / kChebRatio;
    if (L.lmin[f] > lo) lo = L.lmin[f];
    double a[2], b[2];
    cheb_coefs(lo, hi, 2, a, b);
    for (int k = 0; k < 2; ++k) {
      al[2 * k + f] = a[k];
      be[2 * k + f] = b[k];
    }
  }
}

// V-cycle from level l on the right-hand side in lv[l].b (or r64 at level 0);
// the result is left in lv[l].xb (or written to z64 at level 0).
template <int DIM, class T>
int vcycle(pf_problem* pb, Hier<T>& H, size_t l, const double* r64, double* z64, hipStream_t s) {
  Level<T>& L = H.lv[l];
  const bool top = l == 0;
  if (l + 1 == H.lv.size()) {
    // coarsest grid: Chebyshev of degree kCoarseDegree on [lmin, 1.1 lmax]
    if (top) {
      hipLaunchKernelGGL((k_split<T>), dim3(blocks(L.k.nnodes)), dim3(kT), 0, s,
                         reinterpret_cast<const double2*>(r64), L.b, L.k.nnodes);
      PF_HIP_CHECK(hipGetLastError());
    }
    if (L.k.nnodes <= kCoarseSmall) {
      hipLaunchKernelGGL((k_coarse_small<DIM, T>), dim3(1), dim3(kCoarseSmall), 0, s, L.k,
                         (const T*)L.c, (const typename V2<T>::type*)L.b, L.xb,
                         (const double*)H.coarse_dev);
      PF_HIP_CHECK(hipGetLastError());
    } else if (L.k.nnodes <= kCoarseLdsNodes) {
      hipLaunchKernelGGL((k_coarse<DIM, T>), dim3(1), dim3(1024), 0, s, L.k, (const T*)L.c,
                         (const typename V2<T>::type*)L.b, L.xb, (const double*)H.coarse_dev);
      PF_HIP_CHECK(hipGetLastError());
    } else {
      const double* co = H.coarse_host;
      double al[2 * kCoarseDegree], be[2 * kCoarseDegree];
      for (int k = 0; k < kCoarseDegree; ++k) {
        al[2 * k] = co[4 * k];
        al[2 * k + 1] = co[4 * k + 1];
        be[2 * k] = co[4 * k + 2];
        be[2 * k + 1] = co[4 * k + 3];
      }
      // ping-pong ending in xb (kCoarseDegree is even)
      PF_TRY((smooth_step<DIM, T, 0, 0, kWriteD>(L, nullptr, L.xa, al, be, 0, nullptr, nullptr, s)));
      for (int k = 1; k < kCoarseDegree; ++k) {
        auto* in = (k & 1) ? L.xa : L.xb;
        auto* out = (k & 1) ? L.xb : L.xa;
        PF_TRY((smooth_step<DIM, T, 2, 0, kReadD | kWriteD>(L, in, out, al, be, k, nullptr, nullptr,
                                                            s)));
      }
    }
    if (top) {
      hipLaunchKernelGGL((k_merge<T>), dim3(blocks(L.k.nnodes)), dim3(kT), 0, s,
                         (const typename V2<T>::type*)L.xb, reinterpret_cast<double2*>(z64),
                         L.k.nnodes);
      PF_HIP_CHECK(hipGetLastError());
    }
    return PF_OK;
  }
  double al[4], be[4];
  smoother_coefs(L, al, be);
  // pre-smoothing from zero: xa, then xb.  The first direction equals xa, and
  // the post-smoothing restarts with alpha = 0: neither step stores d.  Tiled
  // levels take both steps in one sweep.
  if (L.kz > 0) {
    StArgs<T> A{};
    A.c = L.c;
    A.b = L.b;
    A.out = L.xb;
    A.al0 = (T)al[2];
    A.al1 = (T)al[3];
    A.be0 = (T)be[2];
    A.be1 = (T)be[3];
    A.kz = L.kz;
    A.zb0 = (T)be[0];
    A.zb1 = (T)be[1];
    A.r64 = reinterpret_cast<const double2*>(r64);
    A.bout = L.b;
    A.dg = L.dg;
    if (top)
      hipLaunchKernelGGL((k_stencil3<T, 3, 0>), tiled_grid(L), dim3(SBX * SBY), 0, s, L.k, A);
    else
      hipLaunchKernelGGL((k_stencil3<T, 4, 0>), tiled_grid(L), dim3(SBX * SBY), 0, s, L.k, A);
    PF_HIP_CHECK(hipGetLastError());
  } else {
    if (top) PF_TRY((smooth_step<DIM, T, 1, 0, 0>(L, nullptr, L.xa, al, be, 0, r64, nullptr, s)));
    else PF_TRY((smooth_step<DIM, T, 0, 0, 0>(L, nullptr, L.xa, al, be, 0, nullptr, nullptr, s)));
    PF_TRY((smooth_step<DIM, T, 2, 0, kDIsX>(L, L.xa, L.xb, al, be, 1, nullptr, nullptr, s)));
  }
  if (L.kz > 0) {
    StArgs<T> A{};
    A.c = L.c;
    A.b = L.b;
    A.x = L.xb;
    A.out = L.r;
    A.kz = L.kz;
    hipLaunchKernelGGL((k_stencil3<T, 0, 0>), tiled_grid(L), dim3(SBX * SBY), 0, s, L.k, A);
  } else {
    hipLaunchKernelGGL((k_resid<DIM, T>), plane_grid(L.k), dim3(kT), 0, s, L.k,
                       (const T*)L.c, (const typename V2<T>::type*)L.b,
                       (const typename V2<T>::type*)L.xb, L.r);
  }
  PF_HIP_CHECK(hipGetLastError());
  Level<T>& C = H.lv[l + 1];
  if (DIM == 3 && PF_RESTRICT_TILED) {
    // coarse z-chunks: the longest power of two up to 16 planes that still
    // gives half the stencils' workgroup target (PF_GMG_TILE_GROUPS overrides
    // it as for the stencils)
    const long long tiles = (long long)((C.k.nn[0] + RCX - 1) / RCX) * ((C.k.nn[1] + RCY - 1) / RCY);
    const long long target = (tiled_min_groups() + 1) / 2;
    int kz = 16;
    while (kz > 1 && tiles * ((C.k.nn[2] + kz - 1) / kz) < target) kz /= 2;
    const unsigned nb = (unsigned)(tiles * ((C.k.nn[2] + kz - 1) / kz));
    hipLaunchKernelGGL((k_restrict3t<T>), dim3(nb), dim3(RCX * RCY), 0, s, L.k, C.k,
                       (const typename V2<T>::type*)L.r, C.b, kz);
  } else {
    hipLaunchKernelGGL((k_restrict<DIM, T>), plane_grid(C.k), dim3(kT), 0, s, L.k, C.k,
                       (const typename V2<T>::type*)L.r, C.b);
  }
  PF_HIP_CHECK(hipGetLastError());
  PF_TRY((vcycle<DIM, T>(pb, H, l + 1, nullptr, nullptr, s)));
  hipLaunchKernelGGL((k_prolong_add<DIM, T>), plane_grid(C.k), dim3(kT), 0, s, L.k, C.k,
                     (const typename V2<T>::type*)C.xb, L.xb);
  PF_HIP_CHECK(hipGetLastError());
  // post-smoothing from the corrected iterate: xb -> xa -> xb (or z64); only
  // the first step's direction is read again
  PF_TRY((smooth_step<DIM, T, 2, 0, kWriteD>(L, L.xb, L.xa, al, be, 0, nullptr, nullptr, s)));
  if (top) PF_TRY((smooth_step<DIM, T, 2, 1, kReadD>(L, L.xa, nullptr, al, be, 1, nullptr, z64, s)));
  else PF_TRY((smooth_step<DIM, T, 2, 0, kReadD>(L, L.xa, L.xb, al, be, 1, nullptr, nullptr, s)));
  return PF_OK;
}

template <class T>
int setup_gmg(pf_problem* pb, PcState* st, Hier<T>& H, hipStream_t s) {
  if (!H.allocated) PF_TRY(hier_alloc<T>(pb, H));
  if (pb->geo.dim == 3) return hier_setup<3, T>(pb, H, st->coef0, s);
  return hier_setup<2, T>(pb, H, st->coef0, s);
}

template <class T>
int apply_gmg(pf_problem* pb, Hier<T>& H, const double* r, double* z, hipStream_t s) {
  if (pb->geo.dim == 3) return vcycle<3, T>(pb, H, 0, r, z, s);
  return vcycle<2, T>(pb, H, 0, r, z, s);
}

// The V-cycle on small meshes: r is copied into the fixed input vector, the
// cycle captured from gin to gout replays on the caller's stream, and gout is
// copied to z.  The capture (on the library's own stream, so that the
// caller's stream may be the null stream) happens on the first apply and again
// whenever the block scales or the hierarchy change; set-up only rewrites
// device buffers the graph reads.  The result equals the eager cycle's bit for
// bit.
template <class T>
int apply_gmg_graph(pf_problem* pb, PcState* st, Hier<T>& H, GraphCache& gc, const double* r,
                    double* z, hipStream_t s) {
  const long long n = pb->geo.n_nodes;
  if (!st->gin) {
    if (hipMalloc(&st->gin, (size_t)2 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&st->gout, (size_t)2 * n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("out of device memory for the V-cycle graph vectors");
      return PF_ERR_OOM;
    }
  }
  if (!st->cap) PF_HIP_CHECK(hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
  double sm[2], sk[2];
  block_scales(pb, sm, sk);
  const double sig[4] = {sm[0], sm[1], sk[0], sk[1]};
  const void* level0 = H.lv.empty() ? nullptr : (const void*)H.lv[0].c;
  bool same = gc.exec != nullptr && gc.level0 == level0;
  for (int i = 0; i < 4 && same; ++i) same = gc.sig[i] == sig[i];
  if (!same) {
    if (gc.exec) {
      PF_HIP_CHECK(hipGraphExecDestroy(gc.exec));
      gc.exec = nullptr;
    }
    PF_HIP_CHECK(hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal));
    const int rc = apply_gmg<T>(pb, H, st->gin, st->gout, st->cap);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st->cap, &graph);
    if (rc != PF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    PF_HIP_CHECK(ec);
    const hipError_t ei = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) gc.exec = nullptr;
    PF_HIP_CHECK(ei);
    for (int i = 0; i < 4; ++i) gc.sig[i] = sig[i];
    gc.level0 = level0;
  }
  hipLaunchKernelGGL(k_copy2, dim3(blocks(n)), dim3(kT), 0, s, reinterpret_cast<const double2*>(r),
                     reinterpret_cast<double2*>(st->gin), n);
  PF_HIP_CHECK(hipGetLastError());
  PF_HIP_CHECK(hipGraphLaunch(gc.exec, s));
  hipLaunchKernelGGL(k_copy2, dim3(blocks(n)), dim3(kT), 0, s,
                     reinterpret_cast<const double2*>(st->gout), reinterpret_cast<double2*>(z), n);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace

int pc_alloc(pf_problem* pb) {
  PcState* st = new PcState();
  pb->pc = st;
  // PF_GMG_GRAPH=0 keeps every V-cycle on eager launches (read at creation)
  const char* e = std::getenv("PF_GMG_GRAPH");
  if (e && e[0] == '0' && e[1] == '\0') st->graph_enabled = false;
  if (hipMalloc(&st->coef0, (size_t)pb->geo.n_elems * sizeof(double)) != hipSuccess) return PF_ERR_OOM;
  return PF_OK;
}

hipError_t pc_free(pf_problem* pb) {
  PcState* st = static_cast<PcState*>(pb->pc);
  if (!st) return hipSuccess;
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess) first = e;
  };
  for (GraphCache* gc : {&st->g32, &st->g64})
    if (gc->exec) keep(hipGraphExecDestroy(gc->exec));
  if (st->cap) keep(hipStreamDestroy(st->cap));
  if (st->gin) keep(hipFree(st->gin));
  if (st->gout) keep(hipFree(st->gout));
  keep(hier_free(st->h32));
  keep(hier_free(st->h64));
  if (st->coef0) keep(hipFree(st->coef0));
  delete st;
  pb->pc = nullptr;
  return first;
}

double* pc_coef_buffer(pf_problem* pb) { return static_cast<PcState*>(pb->pc)->coef0; }

int pc_setup_prepared(pf_problem* pb, int kind, int precision, hipStream_t s) {
  PcState* st = static_cast<PcState*>(pb->pc);
  pb->pc_kind = kind;
  pb->pc_precision = precision;
  if (kind == PF_PC_NONE || kind == PF_PC_JACOBI) return PF_OK;
  if (precision == PF_FP32) return setup_gmg<float>(pb, st, st->h32, s);
  return setup_gmg<double>(pb, st, st->h64, s);
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
  if (kind == PF_PC_JACOBI) return PF_OK;
  if (precision == PF_FP32) return setup_gmg<float>(pb, st, st->h32, s);
  return setup_gmg<double>(pb, st, st->h64, s);
}

int pc_apply(pf_problem* pb, const double* r, double* z, hipStream_t s) {
  PcState* st = static_cast<PcState*>(pb->pc);
  const Geo& G = pb->geo;
  const long long n = G.n_nodes;
  switch (pb->pc_kind) {
    case PF_PC_NONE:
      hipLaunchKernelGGL(k_copy2, dim3(blocks(n)), dim3(kT), 0, s,
                         reinterpret_cast<const double2*>(r), reinterpret_cast<double2*>(z), n);
      PF_HIP_CHECK(hipGetLastError());
      return PF_OK;
    case PF_PC_JACOBI: {
      double Ae0[8], Ae1[8];
      double sm[2], sk[2];
      block_scales(pb, sm, sk);
      element_table(G.dim, G.h, sm[0], sk[0], Ae0);
      element_table(G.dim, G.h, sm[1], sk[1], Ae1);
      hipLaunchKernelGGL(k_jacobi, dim3(blocks(n)), dim3(kT), 0, s, G, (const double*)st->coef0,
                         reinterpret_cast<const double2*>(r), reinterpret_cast<double2*>(z),
                         Ae0[0], Ae1[0]);
      PF_HIP_CHECK(hipGetLastError());
      return PF_OK;
    }
    default:
      if (st->graph_enabled && pb->n_dof <= kGraphMaxDof) {
        if (pb->pc_precision == PF_FP32)
          return apply_gmg_graph<float>(pb, st, st->h32, st->g32, r, z, s);
        return apply_gmg_graph<double>(pb, st, st->h64, st->g64, r, z, s);
      }
      if (pb->pc_precision == PF_FP32) return apply_gmg<float>(pb, st->h32, r, z, s);
      return apply_gmg<double>(pb, st->h64, r, z, s);
  }
}

}  // namespace pf
