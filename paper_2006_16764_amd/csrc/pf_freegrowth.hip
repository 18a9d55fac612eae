// Free-growth model (pure melt, phi in [0, 1], temperature T; Sec. 4.1):
// residual, FD Jv and analytic Jv of the part of the theta step that depends
// on the new state, and the explicit part fixed by the previous state, on
// order-1 elements (2-D and 3-D, through quad2/quad3 of pf_element.h) and on
// order-2 (biquadratic, 9-node) elements in 2-D.
//
// Two passes as for the alloy model: one thread per element evaluates the
// element vectors into the element buffer, then a fixed-order gather forms
// the node sums (the order-1 gather of pf_residual.hip, or the order-2 gather
// below, which sums the 1, 2 or 4 elements sharing a node).  The analytic
// tangent runs the pointwise template on dual numbers.
#include "pf_dual.h"

namespace pf {

namespace {

constexpr int kFgBlock = 128;

// Pointwise terms: s1, f1 (phi rows), s3, f3 (T rows); a2 receives a^2.
template <int DIM, class T>
__device__ __forceinline__ void fg_point(const Geo& G, const FgConst& C, const T& phi,
                                         const T (&g)[3], const T& tem, const T (&gT)[3],
                                         const T& dphi, const T& dT, double hist, T& s1,
                                         T (&f1)[3], T& s3, T (&f3)[3], double& a2) {
  T g2[3], q = g[0] * g[0], S;
  g2[0] = q;
  S = g2[0] * g2[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    g2[k] = g[k] * g[k];
    q = q + g2[k];
    S = S + g2[k] * g2[k];
  }
  const T iQ = rcp_t(q + G.delta2);
  const T iQ2 = iQ * iQ;
  const T a = G.a0 + G.e4x4 * (S * iQ2);
  const T SQ = S * iQ;
  const T aa = a * a;
  const T aqc = a * q * (G.e16 * iQ2);
  const T om = 1.0 - phi;
  const T pom = phi * om;
  // G2 = bg phi (1-phi)(1-2phi)/W^2 - 5 beta (Tm - T) phi^2 (1-phi)^2 / W
  const T G2 = pom * (C.c_dw * (1.0 - 2.0 * phi) - C.c_drv * ((C.Tm - tem) * pom));
  s1 = aa * dphi * G.idt + C.theta * G2;
  const T ph = (C.theta * G.idt) * dphi + hist;
  s3 = G.idt * dT - C.Lcp * ph;
  const double tb = C.theta * C.bg, ta = C.theta * C.alpha;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < DIM) {
      f1[k] = tb * (g[k] * (aa + aqc * (g2[k] - SQ)));
      f3[k] = ta * gT[k];
    } else {
      f1[k] = T{};
      f3[k] = T{};
    }
  }
  a2 = val(aa);
}

// Order 1.  Residual: gradient fields {phi, T}; value fields {dphi, dT, hist}.
template <int DIM>
struct PhysFgRes {
  static constexpr int kGxUnroll = 1;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  const FgConst& C;
  double ca, car, a2;
  __device__ PhysFgRes(const Geo& g, const FgConst& c) : G(g), C(c), ca(0.0), car(0.0), a2(0.0) {}
  __device__ __forceinline__ void weight(double wx) { car = fma(wx, a2, car); }
  __device__ __forceinline__ void row(double wrow) {
    ca = fma(wrow, car, ca);
    car = 0.0;
  }
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const double g[3] = {gg[0][0], gg[0][1], gg[0][2]};
    const double gT[3] = {gg[1][0], gg[1][1], gg[1][2]};
    fg_point<DIM, double>(G, C, gv[0], g, gv[1], gT, vv[0], vv[1], vv[2], s[0], f[0], s[1], f[1],
                          a2);
  }
};

// Order 1.  Tangent: gradient fields {phi, T, v_phi, v_T}; value fields as above.
template <int DIM>
struct PhysFgJvp {
  static constexpr int kGxUnroll = 1;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  const FgConst& C;
  __device__ PhysFgJvp(const Geo& g, const FgConst& c) : G(g), C(c) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void row(double) {}
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const Dual phi{gv[0], gv[2]}, tem{gv[1], gv[3]};
    Dual g[3], gT[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g[k] = Dual{gg[0][k], gg[2][k]};
      gT[k] = Dual{gg[1][k], gg[3][k]};
    }
    const Dual dphi{vv[0], gv[2]}, dT{vv[1], gv[3]};
    Dual s1, s3, f1[3], f3[3];
    double a2;
    fg_point<DIM, Dual>(G, C, phi, g, tem, gT, dphi, dT, vv[2], s1, f1, s3, f3, a2);
    s[0] = s1.d;
    s[1] = s3.d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[0][k] = f1[k].d;
      f[1][k] = f3[k].d;
    }
  }
};

template <int DIM, int MODE>
__global__ void __launch_bounds__(kFgBlock)
    k_fg_elem(Geo G, FgConst C, const double2* __restrict__ U, const double2* __restrict__ Up,
              const double2* __restrict__ V, const double* __restrict__ eps_dev,
              const double* __restrict__ hist, double* __restrict__ E, double* __restrict__ coef) {
  constexpr int NA = 1 << DIM;
  const long long e = (long long)blockIdx.x * kFgBlock + threadIdx.x;
  if (e >= G.n_elems) return;
  const long long n0 = G.n[0], n1 = G.n[1];
  const long long ex = e % n0;
  const long long rest = e / n0;
  const long long ey = (DIM == 2) ? rest : rest % n1;
  const long long ez = (DIM == 2) ? 0 : rest / n1;
  const long long s1 = G.nn[0], s2 = (long long)G.nn[0] * G.nn[1];
  const long long base = ex + s1 * (ey + (long long)G.nn[1] * ez);
  const double eps = (MODE == MODE_FD) ? *eps_dev : 0.0;
  double ng[4][NA], nv[3][NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const long long node = base + (a & 1) + ((a >> 1) & 1) * s1 + (DIM == 3 ? ((a >> 2) & 1) * s2 : 0);
    double2 u = U[node];
    const double2 up = Up[node];
    double2 v = make_double2(0.0, 0.0);
    if (MODE != MODE_RES) v = V[node];
    if (MODE == MODE_FD) {
      u.x = fma(eps, v.x, u.x);
      u.y = fma(eps, v.y, u.y);
    }
    ng[0][a] = u.x;
    ng[1][a] = u.y;
    ng[2][a] = v.x;
    ng[3][a] = v.y;
    nv[0][a] = u.x - up.x;
    nv[1][a] = u.y - up.y;
    nv[2][a] = C.use_hist ? hist[node] : 0.0;
  }
  double out[2][NA], dummy[1][NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) out[0][a] = out[1][a] = 0.0;
  if constexpr (MODE == MODE_JVP) {
    PhysFgJvp<DIM> ph(G, C);
    if constexpr (DIM == 3) quad3<4, 3, 2, 0>(G, ng, nv, out, dummy, ph);
    else quad2<4, 3, 2, 0>(G, ng, nv, out, dummy, ph);
  } else {
    double ng2[2][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      ng2[0][a] = ng[0][a];
      ng2[1][a] = ng[1][a];
    }
    PhysFgRes<DIM> ph(G, C);
    if constexpr (DIM == 3) quad3<2, 3, 2, 0>(G, ng2, nv, out, dummy, ph);
    else quad2<2, 3, 2, 0>(G, ng2, nv, out, dummy, ph);
    if (MODE == MODE_RES && coef) coef[e] = ph.ca / ((double)NA * G.jac);
  }
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int a = 0; a < NA; ++a) E[(long long)(o * NA + a) * G.n_elems + e] = out[o][a];
}

// ----------------------------------------------------------------- order 2 (2-D)
// 1-D quadratic Lagrange basis (nodes -1, 0, 1) at the 3 Gauss points.
struct P2 {
  static constexpr double s = 0.77459666924148337704;  // sqrt(3/5)
  __host__ __device__ static constexpr double xi(int q) { return q == 0 ? -s : (q == 1 ? 0.0 : s); }
  __host__ __device__ static constexpr double b(int a, int q) {
    return a == 0 ? 0.5 * xi(q) * (xi(q) - 1.0) : (a == 1 ? 1.0 - xi(q) * xi(q) : 0.5 * xi(q) * (xi(q) + 1.0));
  }
  __host__ __device__ static constexpr double d(int a, int q) {
    return a == 0 ? xi(q) - 0.5 : (a == 1 ? -2.0 * xi(q) : xi(q) + 0.5);
  }
};

// One thread per 9-node element.  Node (lx, ly) of element (ex, ey) is grid
// node (2 ex + lx, 2 ey + ly); the grid spacing G.h is half the element size,
// so d/dx = G.ih[0] d/dxi and the Jacobian of the reference map is G.h0 G.h1.
template <int MODE>
__global__ void __launch_bounds__(kFgBlock)
    k_fg_q2(Geo G, FgConst C, const double2* __restrict__ U, const double2* __restrict__ Up,
            const double2* __restrict__ V, const double* __restrict__ eps_dev,
            const double* __restrict__ hist, double* __restrict__ E, double* __restrict__ coef) {
  const long long ne = (long long)C.n_macro[0] * C.n_macro[1];
  const long long e = (long long)blockIdx.x * kFgBlock + threadIdx.x;
  if (e >= ne) return;
  const int ex = (int)(e % C.n_macro[0]), ey = (int)(e / C.n_macro[0]);
  const long long nn0 = G.nn[0];
  const double eps = (MODE == MODE_FD) ? *eps_dev : 0.0;
  // fields: 0 phi, 1 T, 2 dphi, 3 dT, 4 hist, 5 v_phi, 6 v_T
  constexpr int NF = MODE == MODE_JVP ? 7 : 5;
  double u[NF][3][3];
#pragma unroll
  for (int ly = 0; ly < 3; ++ly)
#pragma unroll
    for (int lx = 0; lx < 3; ++lx) {
      const long long node = (2 * ex + lx) + nn0 * (long long)(2 * ey + ly);
      double2 w = U[node];
      const double2 up = Up[node];
      double2 v = make_double2(0.0, 0.0);
      if (MODE != MODE_RES) v = V[node];
      if (MODE == MODE_FD) {
        w.x = fma(eps, v.x, w.x);
        w.y = fma(eps, v.y, w.y);
      }
      u[0][ly][lx] = w.x;
      u[1][ly][lx] = w.y;
      u[2][ly][lx] = w.x - up.x;
      u[3][ly][lx] = w.y - up.y;
      u[4][ly][lx] = C.use_hist ? hist[node] : 0.0;
      if constexpr (MODE == MODE_JVP) {
        u[5][ly][lx] = v.x;
        u[6][ly][lx] = v.y;
      }
    }
  double out[2][3][3];
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int ly = 0; ly < 3; ++ly)
#pragma unroll
      for (int lx = 0; lx < 3; ++lx) out[o][ly][lx] = 0.0;
  const double ih0 = G.ih[0], ih1 = G.ih[1], jac = G.h[0] * G.h[1];
  double ca = 0.0;
#pragma unroll 1
  for (int qy = 0; qy < 3; ++qy) {
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
      // values and derivatives of every field at the point, row by row
      double val[NF], dx[NF], dy[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
        for (int ly = 0; ly < 3; ++ly) {
          const double rv = P2::b(0, qx) * u[f][ly][0] + P2::b(1, qx) * u[f][ly][1] +
                            P2::b(2, qx) * u[f][ly][2];
          const double rd = P2::d(0, qx) * u[f][ly][0] + P2::d(1, qx) * u[f][ly][1] +
                            P2::d(2, qx) * u[f][ly][2];
          v0 = fma(P2::b(ly, qy), rv, v0);
          v1 = fma(P2::b(ly, qy), rd, v1);
          v2 = fma(P2::d(ly, qy), rv, v2);
        }
        val[f] = v0;
        dx[f] = v1 * ih0;
        dy[f] = v2 * ih1;
      }
      double s[2], fl[2][3], a2 = 0.0;
      if constexpr (MODE == MODE_JVP) {
        const Dual phi{val[0], val[5]}, tem{val[1], val[6]};
        const Dual g[3] = {Dual{dx[0], dx[5]}, Dual{dy[0], dy[5]}, Dual{0.0, 0.0}};
        const Dual gT[3] = {Dual{dx[1], dx[6]}, Dual{dy[1], dy[6]}, Dual{0.0, 0.0}};
        const Dual dphi{val[2], val[5]}, dT{val[3], val[6]};
        Dual s1, s3, f1[3], f3[3];
        fg_point<2, Dual>(G, C, phi, g, tem, gT, dphi, dT, val[4], s1, f1, s3, f3, a2);
        s[0] = s1.d;
        s[1] = s3.d;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          fl[0][k] = f1[k].d;
          fl[1][k] = f3[k].d;
        }
      } else {
        const double g[3] = {dx[0], dy[0], 0.0};
        const double gT[3] = {dx[1], dy[1], 0.0};
        fg_point<2, double>(G, C, val[0], g, val[1], gT, val[2], val[3], val[4], s[0], fl[0], s[1],
                            fl[1], a2);
      }
      const double wq = Q1::w(qx) * Q1::w(qy) * jac;
      ca = fma(wq, a2, ca);
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const double ws = wq * s[o], wfx = wq * fl[o][0] * ih0, wfy = wq * fl[o][1] * ih1;
#pragma unroll
        for (int ly = 0; ly < 3; ++ly) {
          const double cy = ws * P2::b(ly, qy), cx = wfx * P2::b(ly, qy), cd = wfy * P2::d(ly, qy);
#pragma unroll
          for (int lx = 0; lx < 3; ++lx)
            out[o][ly][lx] += cy * P2::b(lx, qx) + cx * P2::d(lx, qx) + cd * P2::b(lx, qx);
        }
      }
    }
  }
  if (MODE == MODE_RES && coef) {
    // element mean of a^2 on its four grid cells (the preconditioner's grid)
    const double c = ca / (4.0 * jac);
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx)
        coef[(2 * ex + sx) + (long long)G.n[0] * (2 * ey + sy)] = c;
  }
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int ly = 0; ly < 3; ++ly)
#pragma unroll
      for (int lx = 0; lx < 3; ++lx) E[(long long)(o * 9 + lx + 3 * ly) * ne + e] = out[o][ly][lx];
}

// Node sums of the 9-node element buffer: grid node (gx, gy) belongs to the
// elements whose index range covers it (1, 2 or 4), summed in a fixed order.
__global__ void __launch_bounds__(256)
    k_fg_q2_gather(Geo G, FgConst C, const double* __restrict__ E, double2* __restrict__ out,
                   const double2* __restrict__ F0, const double* __restrict__ eps_dev, int fd) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.n_nodes) return;
  const long long ne = (long long)C.n_macro[0] * C.n_macro[1];
  const int gx = (int)(i % G.nn[0]), gy = (int)(i / G.nn[0]);
  int exs[2], lxs[2], nx = 0, eys[2], lys[2], ny = 0;
  if (gx & 1) {
    exs[0] = gx >> 1;
    lxs[0] = 1;
    nx = 1;
  } else {
    if (gx > 0) {
      exs[nx] = (gx >> 1) - 1;
      lxs[nx++] = 2;
    }
    if ((gx >> 1) < C.n_macro[0]) {
      exs[nx] = gx >> 1;
      lxs[nx++] = 0;
    }
  }
  if (gy & 1) {
    eys[0] = gy >> 1;
    lys[0] = 1;
    ny = 1;
  } else {
    if (gy > 0) {
      eys[ny] = (gy >> 1) - 1;
      lys[ny++] = 2;
    }
    if ((gy >> 1) < C.n_macro[1]) {
      eys[ny] = gy >> 1;
      lys[ny++] = 0;
    }
  }
  double a0 = 0.0, a1 = 0.0;
  for (int jy = 0; jy < ny; ++jy)
    for (int jx = 0; jx < nx; ++jx) {
      const long long e = exs[jx] + (long long)C.n_macro[0] * eys[jy];
      const int a = lxs[jx] + 3 * lys[jy];
      a0 += E[(long long)a * ne + e];
      a1 += E[(long long)(9 + a) * ne + e];
    }
  if (fd) {
    const double eps = *eps_dev;
    const double2 f0 = F0[i];
    out[i] = eps == 0.0 ? make_double2(0.0, 0.0)
                        : make_double2((a0 - f0.x) / eps, (a1 - f0.y) / eps);
    return;
  }
  out[i] = make_double2(a0, a1);
}

FgConst fg_const(const pf_problem* pb, double theta, int use_hist) {
  const pf_freegrowth_params& f = pb->fg;
  FgConst C{};
  C.bg = f.beta * f.Gamma;
  C.c_dw = f.beta * f.Gamma / (f.W * f.W);
  C.c_drv = 5.0 * f.beta / f.W;
  C.Tm = f.Tm;
  C.alpha = f.alpha;
  C.Lcp = f.Lcp;
  C.theta = theta;
  C.use_hist = use_hist;
  C.n_macro[0] = pb->params.n[0];
  C.n_macro[1] = pb->params.n[1];
  return C;
}

int launch_elem(pf_problem* pb, const FgConst& C, int mode, const double* U, const double* Uprev,
                const double* v, const double* eps_dev, double* coef, hipStream_t s) {
  const Geo& G = pb->geo;
  auto U2 = reinterpret_cast<const double2*>(U);
  auto P2p = reinterpret_cast<const double2*>(Uprev);
  auto V2 = reinterpret_cast<const double2*>(v);
  if (pb->params.order == 2) {
    const long long ne = (long long)C.n_macro[0] * C.n_macro[1];
    const unsigned eb = (unsigned)((ne + kFgBlock - 1) / kFgBlock);
    if (mode == MODE_RES)
      hipLaunchKernelGGL(k_fg_q2<MODE_RES>, dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p, nullptr,
                         nullptr, pb->hist, pb->elem_buf, coef);
    else if (mode == MODE_FD)
      hipLaunchKernelGGL(k_fg_q2<MODE_FD>, dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p, V2,
                         eps_dev, pb->hist, pb->elem_buf, nullptr);
    else
      hipLaunchKernelGGL(k_fg_q2<MODE_JVP>, dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p, V2,
                         nullptr, pb->hist, pb->elem_buf, nullptr);
  } else {
    const unsigned eb = (unsigned)((G.n_elems + kFgBlock - 1) / kFgBlock);
    if (G.dim == 3) {
      if (mode == MODE_RES)
        hipLaunchKernelGGL((k_fg_elem<3, MODE_RES>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           nullptr, nullptr, pb->hist, pb->elem_buf, coef);
      else if (mode == MODE_FD)
        hipLaunchKernelGGL((k_fg_elem<3, MODE_FD>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           V2, eps_dev, pb->hist, pb->elem_buf, nullptr);
      else
        hipLaunchKernelGGL((k_fg_elem<3, MODE_JVP>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           V2, nullptr, pb->hist, pb->elem_buf, nullptr);
    } else {
      if (mode == MODE_RES)
        hipLaunchKernelGGL((k_fg_elem<2, MODE_RES>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           nullptr, nullptr, pb->hist, pb->elem_buf, coef);
      else if (mode == MODE_FD)
        hipLaunchKernelGGL((k_fg_elem<2, MODE_FD>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           V2, eps_dev, pb->hist, pb->elem_buf, nullptr);
      else
        hipLaunchKernelGGL((k_fg_elem<2, MODE_JVP>), dim3(eb), dim3(kFgBlock), 0, s, G, C, U2, P2p,
                           V2, nullptr, pb->hist, pb->elem_buf, nullptr);
    }
  }
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int gather(pf_problem* pb, const FgConst& C, double* out0, const double* F0, const double* eps_dev,
           int fd, hipStream_t s) {
  if (pb->params.order != 2) return launch_gather2(pb, out0, F0, eps_dev, fd, s);
  const unsigned nb = (unsigned)((pb->geo.n_nodes + 255) / 256);
  hipLaunchKernelGGL(k_fg_q2_gather, dim3(nb), dim3(256), 0, s, pb->geo, C, pb->elem_buf,
                     reinterpret_cast<double2*>(out0), reinterpret_cast<const double2*>(F0),
                     eps_dev, fd);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace

long long fg_elem_buf_len(const pf_problem* pb) {
  if (pb->params.order == 2) return (long long)2 * 9 * pb->params.n[0] * pb->params.n[1];
  return (long long)2 * (1 << pb->geo.dim) * pb->geo.n_elems;
}

int launch_fg(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
              const double* F0, const double* eps_dev, double* out0, double* coef, hipStream_t s) {
  if (mode != MODE_RES && mode != MODE_FD && mode != MODE_JVP) {
    set_error("the free-growth model has no VJP");
    return PF_ERR_INVALID_ARG;
  }
  const FgConst C = fg_const(pb, pb->params.theta, 1);
  PF_TRY(launch_elem(pb, C, mode, U, Uprev, v, eps_dev, coef, s));
  return gather(pb, C, out0, F0, eps_dev, mode == MODE_FD ? 1 : 0, s);
}

int fg_explicit(pf_problem* pb, const double* Un, double* E, hipStream_t s) {
  const double th = pb->params.theta;
  if (th == 1.0) {
    PF_HIP_CHECK(hipMemsetAsync(E, 0, pb->n_dof * sizeof(double), s));
    return PF_OK;
  }
  // the residual at (U^n; U^n) with weight 1 and no history is the spatial
  // operator at U^n: the time and rate terms vanish
  const FgConst C = fg_const(pb, 1.0, 0);
  PF_TRY(launch_elem(pb, C, MODE_RES, Un, Un, nullptr, nullptr, nullptr, s));
  PF_TRY(gather(pb, C, E, nullptr, nullptr, 0, s));
  return blas_axpby(1.0 - th, E, 0.0, E, E, pb->n_dof, s);
}

}  // namespace pf
