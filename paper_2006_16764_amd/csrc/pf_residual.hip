// Residual-family kernels: F(U), fused finite-difference Jv, analytic Jv and
// the vector-Jacobian product, all from one element routine (pf_element.h).
//
// Two passes, both deterministic:
//   k_elem   one thread per element: gathers its 2^d corner values (16-byte
//            interleaved loads), evaluates the element vectors by sum
//            factorisation and stores them structure-of-arrays,
//            E[(o * 2^d + a) * n_elems + e];
//   k_gather one thread per node: sums the contributions of the <= 2^d
//            elements around it in a fixed order and writes the interleaved
//            result (no atomics, no colouring).
// The VJP's two parameter sums are reduced per block in a fixed tree and then
// across blocks in a fixed order.
#include "pf_element.h"

namespace pf {

namespace {

constexpr int kElemBlock = 256;

template <int DIM>
__device__ __forceinline__ void corner_nodes(const Geo& G, long long e, long long (&node)[1 << DIM]) {
  const long long n0 = G.n[0], n1 = G.n[1];
  const long long ex = e % n0;
  const long long rest = e / n0;
  const long long ey = (DIM == 2) ? rest : rest % n1;
  const long long ez = (DIM == 2) ? 0 : rest / n1;
  const long long s1 = G.nn[0], s2 = (long long)G.nn[0] * G.nn[1];
  const long long base = ex + s1 * (ey + (long long)G.nn[1] * ez);
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a)
    node[a] = base + (a & 1) + ((a >> 1) & 1) * s1 + (DIM == 3 ? ((a >> 2) & 1) * s2 : 0);
}

template <int DIM, int MODE>
__global__ void __launch_bounds__(kElemBlock)
    k_elem(Geo G, const double2* __restrict__ U, const double2* __restrict__ Up,
           const double2* __restrict__ V, const double* __restrict__ eps_dev,
           double* __restrict__ E, double* __restrict__ vjp_part, double* __restrict__ coef) {
  constexpr int NA = 1 << DIM;
  constexpr int NO = (MODE == MODE_VJP) ? 4 : 2;
  const long long e = (long long)blockIdx.x * kElemBlock + threadIdx.x;
  const bool active = e < G.n_elems;
  double ge = 0.0, gl = 0.0;
  if (active) {
    long long node[NA];
    corner_nodes<DIM>(G, e, node);
    double u0[NA], u1[NA], p0[NA], p1[NA], v0[NA], v1[NA];
    double eps = 0.0;
    if (MODE == MODE_FD) eps = *eps_dev;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      double2 u = U[node[a]];
      const double2 up = Up[node[a]];
      double2 v = make_double2(0.0, 0.0);
      if (MODE != MODE_RES) v = V[node[a]];
      if (MODE == MODE_FD) {
        u.x = fma(eps, v.x, u.x);
        u.y = fma(eps, v.y, u.y);
      }
      u0[a] = u.x;
      u1[a] = u.y;
      p0[a] = up.x;
      p1[a] = up.y;
      v0[a] = v.x;
      v1[a] = v.y;
    }
    double out[NO][NA];
    Element<DIM, MODE>::run(G, u0, u1, p0, p1, v0, v1, out, ge, gl);
    if (MODE == MODE_RES && coef) coef[e] = ge / ((double)NA * G.jac);
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int a = 0; a < NA; ++a) E[(long long)(o * NA + a) * G.n_elems + e] = out[o][a];
  }
  if (MODE == MODE_VJP) {
    // fixed-order block reduction of the two parameter sums
    __shared__ double red[2][kElemBlock];
    red[0][threadIdx.x] = ge;
    red[1][threadIdx.x] = gl;
    __syncthreads();
    for (int w = kElemBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        red[0][threadIdx.x] += red[0][threadIdx.x + w];
        red[1][threadIdx.x] += red[1][threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      vjp_part[blockIdx.x] = red[0][0];
      vjp_part[gridDim.x + blockIdx.x] = red[1][0];
    }
  }
}

// Sum the element contributions around every node.  NO = 2 (one output
// vector) or 4 (VJP: gU then gUprev).  mode FD: out0 = (sum - F0)/eps.
template <int DIM, int NO>
__global__ void __launch_bounds__(256)
    k_gather(Geo G, const double* __restrict__ E, double2* __restrict__ out0,
             double2* __restrict__ out1, const double2* __restrict__ F0,
             const double* __restrict__ eps_dev, int fd) {
  constexpr int NA = 1 << DIM;
  // blockIdx.y is the node plane (0 in 2-D): coordinates from 32-bit arithmetic
  const int pn = G.nn[0] * G.nn[1];
  const int q = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  if (q >= pn) return;
  const int iy = q / G.nn[0];
  const int ix = q - iy * G.nn[0];
  const int iz = (int)blockIdx.y;
  const long long i = (long long)iz * pn + q;
  double acc[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) acc[o] = 0.0;
#pragma unroll
  for (int bz = 0; bz < (DIM == 3 ? 2 : 1); ++bz) {
    const int ez = iz - 1 + bz + (DIM == 3 ? 0 : 1);
    if (DIM == 3 && (ez < 0 || ez >= G.n[2])) continue;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int ey = iy - 1 + by;
      if (ey < 0 || ey >= G.n[1]) continue;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int ex = ix - 1 + bx;
        if (ex < 0 || ex >= G.n[0]) continue;
        const long long e = ex + (long long)G.n[0] * (ey + (long long)G.n[1] * (DIM == 3 ? ez : 0));
        const int a = (1 - bx) + 2 * (1 - by) + (DIM == 3 ? 4 * (1 - bz) : 0);
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] += E[(long long)(o * NA + a) * G.n_elems + e];
      }
    }
  }
  if (fd) {
    const double eps = *eps_dev;
    const double2 f0 = F0[i];
    double2 o;
    if (eps == 0.0) {
      o.x = 0.0;
      o.y = 0.0;
    } else {
      const double ie = 1.0 / eps;
      o.x = (acc[0] - f0.x) * ie;
      o.y = (acc[1] - f0.y) * ie;
    }
    out0[i] = o;
    return;
  }
  if (out0) out0[i] = make_double2(acc[0], acc[1]);
  if (NO == 4 && out1) out1[i] = make_double2(acc[2 % NO], acc[3 % NO]);
}

template <int DIM>
int launch_dim(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
               const double* F0, const double* eps_dev, double* out0, double* out1,
               double* vjp_part, double* coef, hipStream_t s) {
  const Geo& G = pb->geo;
  const unsigned eb = (unsigned)((G.n_elems + kElemBlock - 1) / kElemBlock);
  const dim3 nb((unsigned)(((long long)G.nn[0] * G.nn[1] + 255) / 256), (unsigned)G.nn[2]);
  auto U2 = reinterpret_cast<const double2*>(U);
  auto P2 = reinterpret_cast<const double2*>(Uprev);
  auto V2 = reinterpret_cast<const double2*>(v);
  switch (mode) {
    case MODE_RES:
      hipLaunchKernelGGL((k_elem<DIM, MODE_RES>), dim3(eb), dim3(kElemBlock), 0, s, G, U2, P2,
                         nullptr, nullptr, pb->elem_buf, nullptr, coef);
      break;
    case MODE_FD:
      hipLaunchKernelGGL((k_elem<DIM, MODE_FD>), dim3(eb), dim3(kElemBlock), 0, s, G, U2, P2, V2,
                         eps_dev, pb->elem_buf, nullptr, nullptr);
      break;
    case MODE_JVP:
      hipLaunchKernelGGL((k_elem<DIM, MODE_JVP>), dim3(eb), dim3(kElemBlock), 0, s, G, U2, P2, V2,
                         nullptr, pb->elem_buf, nullptr, nullptr);
      break;
    case MODE_VJPU:
      hipLaunchKernelGGL((k_elem<DIM, MODE_VJPU>), dim3(eb), dim3(kElemBlock), 0, s, G, U2, P2, V2,
                         nullptr, pb->elem_buf, nullptr, nullptr);
      break;
    default:
      hipLaunchKernelGGL((k_elem<DIM, MODE_VJP>), dim3(eb), dim3(kElemBlock), 0, s, G, U2, P2, V2,
                         nullptr, pb->elem_buf, vjp_part, nullptr);
      break;
  }
  PF_HIP_CHECK(hipGetLastError());
  if (mode == MODE_VJP) {
    hipLaunchKernelGGL((k_gather<DIM, 4>), dim3(nb), dim3(256), 0, s, G, pb->elem_buf,
                       reinterpret_cast<double2*>(out0), reinterpret_cast<double2*>(out1),
                       nullptr, nullptr, 0);
  } else {
    hipLaunchKernelGGL((k_gather<DIM, 2>), dim3(nb), dim3(256), 0, s, G, pb->elem_buf,
                       reinterpret_cast<double2*>(out0), nullptr,
                       reinterpret_cast<const double2*>(F0), eps_dev, mode == MODE_FD ? 1 : 0);
  }
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace

long long residual2_elem_len(const Geo& G) { return (long long)2 * 4 * G.n_elems; }

int launch_residual2(const Geo& G, double* elem, const double* U, const double* Uprev, double* F,
                     hipStream_t s) {
  const unsigned eb = (unsigned)((G.n_elems + kElemBlock - 1) / kElemBlock);
  const dim3 nb((unsigned)(((long long)G.nn[0] * G.nn[1] + 255) / 256), (unsigned)G.nn[2]);
  hipLaunchKernelGGL((k_elem<2, MODE_RES>), dim3(eb), dim3(kElemBlock), 0, s, G,
                     reinterpret_cast<const double2*>(U), reinterpret_cast<const double2*>(Uprev),
                     nullptr, nullptr, elem, nullptr, nullptr);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_gather<2, 2>), dim3(nb), dim3(256), 0, s, G, elem,
                     reinterpret_cast<double2*>(F), nullptr, nullptr, nullptr, 0);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int launch_gather2(pf_problem* pb, double* out0, const double* F0, const double* eps_dev, int fd,
                   hipStream_t s) {
  const Geo& G = pb->geo;
  const dim3 nb((unsigned)(((long long)G.nn[0] * G.nn[1] + 255) / 256), (unsigned)G.nn[2]);
  if (G.dim == 3)
    hipLaunchKernelGGL((k_gather<3, 2>), dim3(nb), dim3(256), 0, s, G, pb->elem_buf,
                       reinterpret_cast<double2*>(out0), nullptr,
                       reinterpret_cast<const double2*>(F0), eps_dev, fd);
  else
    hipLaunchKernelGGL((k_gather<2, 2>), dim3(nb), dim3(256), 0, s, G, pb->elem_buf,
                       reinterpret_cast<double2*>(out0), nullptr,
                       reinterpret_cast<const double2*>(F0), eps_dev, fd);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int launch_residual_family(pf_problem* pb, int mode, const double* U, const double* Uprev,
                           const double* v, const double* F0, const double* eps_dev,
                           double* out0, double* out1, double* vjp_part, hipStream_t s,
                           double* coef) {
  if (pb->model == 1) return launch_alloy(pb, mode, U, Uprev, v, F0, eps_dev, out0, coef, s);
  if (pb->model == 2) return launch_fg(pb, mode, U, Uprev, v, F0, eps_dev, out0, coef, s);
  if (mode == MODE_VJPP) {
    // out1 receives (dF/dUprev)^T w; the fused 3-D kernel writes its one
    // output through out0, the 2-D path runs the full adjoint without gU
    if (pb->geo.dim == 3)
      return launch_fused3(pb, MODE_VJPP, U, Uprev, v, F0, eps_dev, out1, nullptr, vjp_part, coef, s);
    return launch_dim<2>(pb, MODE_VJP, U, Uprev, v, F0, eps_dev, nullptr, out1, vjp_part, coef, s);
  }
  if (pb->geo.dim == 3)
    return launch_fused3(pb, mode, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, coef, s);
  return launch_dim<2>(pb, mode, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, coef, s);
}

// Number of per-block partial sums the VJP writes (one per workgroup).
int elem_blocks(const pf_problem* pb) {
  if (pb->geo.dim == 3) return fused3_tiles(pb->geo);
  return (int)((pb->geo.n_elems + kElemBlock - 1) / kElemBlock);
}

}  // namespace pf
