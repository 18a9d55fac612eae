// Alloy model (directional solidification, Sec. 4.3): residual, FD Jv and
// analytic Jv of the part of the theta step that depends on the new state,
// and the explicit part fixed by the previous state.
//
// Two passes as for the 2-D thermal kernels: k_alloy_elem evaluates every
// element once (one thread per element; Gauss rule by the sum-factorised
// quad3/quad2 of pf_element.h) into the element buffer, then the shared
// gather kernel forms the node sums in a fixed order.  Unlike the thermal u
// equation the solute equation is nonlinear (one-sided mobility,
// anti-trapping current, cu phihat source), so both fields go through the
// Gauss rule.  The analytic tangent evaluates the same pointwise function on
// dual numbers (value, directional derivative): forward-mode differentiation
// of exactly the residual's arithmetic.
#include "pf_dual.h"

namespace pf {

namespace {

constexpr int kAlloyBlock = 128;
constexpr double kInv2Sqrt2 = 0.35355339059327376220;  // 1/(2 sqrt 2)

// Pointwise terms of the alloy residual: s1, f1 (phi rows: value and flux
// parts), s2, f2 (u rows).  hist = (1 - theta)(phi^n - phi^(n-1))/dt, x the
// point's coordinate along axis 0.  a2 receives cu a^2, the mobility factor of
// the time term (the preconditioner's phi-block coefficient).
template <int DIM, class T>
__device__ __forceinline__ void alloy_point(const Geo& G, const AlloyConst& C, const T& phi,
                                            const T (&g)[3], const T& u, const T (&gu)[3],
                                            const T& dphi, const T& du, double hist, double x,
                                            T& s1, T (&f1)[3], T& s2, T (&f2)[3], double& a2) {
  T g2[3], q = g[0] * g[0], S;
  g2[0] = q;
  S = g2[0] * g2[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    g2[k] = g[k] * g[k];
    q = q + g2[k];
    S = S + g2[k] * g2[k];
  }
  const T Q = q + G.delta2;
  const T iQ = rcp_t(Q);
  const T iQ2 = iQ * iQ;
  const T a = G.a0 + G.e4x4 * (S * iQ2);
  const T SQ = S * iQ;
  const T aa = a * a;
  const T aqc = a * q * (G.e16 * iQ2);
  const T cu = 1.0 + C.omk * u;
  const T om = 1.0 - phi * phi;
  const double G4 = fma(x, C.g4a, C.g4b);
  const T R = om * (phi - G.lam * (om * (u + G4)));
  s1 = cu * aa * dphi * G.idt - C.theta * R;
  const T ph = (C.theta * G.idt) * dphi + hist;
  s2 = (C.hopk * G.idt) * du - 0.5 * (ph * cu);
  const T mob = (C.theta * G.D * 0.5) * (1.0 - phi);
  const T at = kInv2Sqrt2 * (cu * ph * rsqrt_t(Q));
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < DIM) {
      const T J = g[k] * (aa + aqc * (g2[k] - SQ));
      f1[k] = C.theta * J;
      f2[k] = mob * gu[k] + at * g[k];
    } else {
      f1[k] = T{};
      f2[k] = T{};
    }
  }
  a2 = val(cu * aa);
}

// Residual: gradient fields {phi, u}; value fields {phi - phi^n, u - u^n, hist, x}.
template <int DIM>
struct PhysAlloyRes {
  // unroll choices measured at 1024 x 256 x 256 (points and rows unrolled)
  static constexpr int kGxUnroll = 3;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  const AlloyConst& C;
  double ca, car, a2;
  __device__ PhysAlloyRes(const Geo& g, const AlloyConst& c)
      : G(g), C(c), ca(0.0), car(0.0), a2(0.0) {}
  __device__ __forceinline__ void weight(double wx) { car = fma(wx, a2, car); }
  __device__ __forceinline__ void row(double wrow) {
    ca = fma(wrow, car, ca);
    car = 0.0;
  }
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const double g[3] = {gg[0][0], gg[0][1], gg[0][2]};
    const double gu[3] = {gg[1][0], gg[1][1], gg[1][2]};
    alloy_point<DIM, double>(G, C, gv[0], g, gv[1], gu, vv[0], vv[1], vv[2], vv[3], s[0], f[0], s[1],
                             f[1], a2);
  }
};

// Tangent: gradient fields {phi, u, v_phi, v_u}; value fields as the residual.
template <int DIM>
struct PhysAlloyJvp {
  // points unrolled, rows one at a time (measured at 1024 x 256 x 256)
  static constexpr int kGxUnroll = 3;
  static constexpr int kGyUnroll = 1;
  const Geo& G;
  const AlloyConst& C;
  __device__ PhysAlloyJvp(const Geo& g, const AlloyConst& c) : G(g), C(c) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void row(double) {}
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const Dual phi{gv[0], gv[2]}, u{gv[1], gv[3]};
    Dual g[3], gu[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g[k] = Dual{gg[0][k], gg[2][k]};
      gu[k] = Dual{gg[1][k], gg[3][k]};
    }
    const Dual dphi{vv[0], gv[2]}, du{vv[1], gv[3]};
    Dual s1, s2, f1[3], f2[3];
    double a2;
    alloy_point<DIM, Dual>(G, C, phi, g, u, gu, dphi, du, vv[2], vv[3], s1, f1, s2, f2, a2);
    s[0] = s1.d;
    s[1] = s2.d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[0][k] = f1[k].d;
      f[1][k] = f2[k].d;
    }
  }
};

template <int DIM, int MODE>
struct AlloyElement {
  static constexpr int NA = 1 << DIM;
  template <int NG, int NV, class Phys>
  __device__ __forceinline__ static void quad(const Geo& G, const double (&ng)[NG][NA],
                                              const double (&nv)[NV][NA], double (&os)[2][NA],
                                              Phys& ph) {
    double dummy[1][NA];
    if constexpr (DIM == 3) quad3<NG, NV, 2, 0>(G, ng, nv, os, dummy, ph);
    else quad2<NG, NV, 2, 0>(G, ng, nv, os, dummy, ph);
  }
  // u0/u1: (phi, u) of the state (the perturbed state for FD), p0/p1 of the
  // previous state, hs: history rate, xc: x coordinates, v0/v1: direction.
  __device__ __forceinline__ static void run(const Geo& G, const AlloyConst& C,
                                             const double (&u0)[NA], const double (&u1)[NA],
                                             const double (&p0)[NA], const double (&p1)[NA],
                                             const double (&hs)[NA], const double (&xc)[NA],
                                             const double (&v0)[NA], const double (&v1)[NA],
                                             double (&out)[2][NA], double& ge) {
#pragma unroll
    for (int a = 0; a < NA; ++a) out[0][a] = out[1][a] = 0.0;
    double nv[4][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      nv[0][a] = u0[a] - p0[a];
      nv[1][a] = u1[a] - p1[a];
      nv[2][a] = hs[a];
      nv[3][a] = xc[a];
    }
    if constexpr (MODE == MODE_JVP) {
      double ng[4][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ng[0][a] = u0[a];
        ng[1][a] = u1[a];
        ng[2][a] = v0[a];
        ng[3][a] = v1[a];
      }
      PhysAlloyJvp<DIM> ph(G, C);
      quad<4, 4>(G, ng, nv, out, ph);
      ge = 0.0;
    } else {
      double ng[2][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ng[0][a] = u0[a];
        ng[1][a] = u1[a];
      }
      PhysAlloyRes<DIM> ph(G, C);
      quad<2, 4>(G, ng, nv, out, ph);
      ge = ph.ca;
    }
  }
};

template <int DIM, int MODE>
__global__ void __launch_bounds__(kAlloyBlock)
    k_alloy_elem(Geo G, AlloyConst C, const double2* __restrict__ U, const double2* __restrict__ Up,
                 const double2* __restrict__ V, const double* __restrict__ eps_dev,
                 const double* __restrict__ hist, double* __restrict__ E, double* __restrict__ coef) {
  constexpr int NA = 1 << DIM;
  // blockIdx.y is the element layer (0 in 2-D): coordinates from 32-bit arithmetic
  const int pe = G.n[0] * G.n[1];
  const int q = (int)blockIdx.x * kAlloyBlock + (int)threadIdx.x;
  if (q >= pe) return;
  const int ey = q / G.n[0];
  const int ex = q - ey * G.n[0];
  const int ez = (int)blockIdx.y;
  const long long e = (long long)ez * pe + q;
  const long long s1 = G.nn[0], s2 = (long long)G.nn[0] * G.nn[1];
  const long long base = ex + s1 * (ey + (long long)G.nn[1] * ez);
  const double eps = (MODE == MODE_FD) ? *eps_dev : 0.0;
  double u0[NA], u1[NA], p0[NA], p1[NA], hs[NA], xc[NA], v0[NA], v1[NA];
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
    u0[a] = u.x;
    u1[a] = u.y;
    p0[a] = up.x;
    p1[a] = up.y;
    v0[a] = v.x;
    v1[a] = v.y;
    hs[a] = C.use_hist ? hist[node] : 0.0;
    xc[a] = fma((double)(ex + (a & 1)), C.h0, C.x0);
  }
  double out[2][NA];
  double ge = 0.0;
  AlloyElement<DIM, MODE == MODE_FD ? MODE_RES : MODE>::run(G, C, u0, u1, p0, p1, hs, xc, v0, v1,
                                                            out, ge);
  if (MODE == MODE_RES && coef) coef[e] = ge / ((double)NA * G.jac);
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int a = 0; a < NA; ++a) E[(long long)(o * NA + a) * G.n_elems + e] = out[o][a];
}

__global__ void k_history(long long n, const double2* __restrict__ Un,
                             const double2* __restrict__ Unm1, double c, double* __restrict__ hist) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    hist[i] = c * (Un[i].x - Unm1[i].x);
}

template <int DIM>
int launch_elem(pf_problem* pb, const AlloyConst& C, int mode, const double* U, const double* Uprev,
                const double* v, const double* eps_dev, double* coef, hipStream_t s) {
  const Geo& G = pb->geo;
  const dim3 eb((unsigned)(((long long)G.n[0] * G.n[1] + kAlloyBlock - 1) / kAlloyBlock),
                (unsigned)G.n[2]);
  auto U2 = reinterpret_cast<const double2*>(U);
  auto P2 = reinterpret_cast<const double2*>(Uprev);
  auto V2 = reinterpret_cast<const double2*>(v);
  switch (mode) {
    case MODE_RES:
      hipLaunchKernelGGL((k_alloy_elem<DIM, MODE_RES>), dim3(eb), dim3(kAlloyBlock), 0, s, G, C, U2,
                         P2, nullptr, nullptr, pb->hist, pb->elem_buf, coef);
      break;
    case MODE_FD:
      hipLaunchKernelGGL((k_alloy_elem<DIM, MODE_FD>), dim3(eb), dim3(kAlloyBlock), 0, s, G, C, U2,
                         P2, V2, eps_dev, pb->hist, pb->elem_buf, nullptr);
      break;
    default:
      hipLaunchKernelGGL((k_alloy_elem<DIM, MODE_JVP>), dim3(eb), dim3(kAlloyBlock), 0, s, G, C,
                         U2, P2, V2, nullptr, pb->hist, pb->elem_buf, nullptr);
      break;
  }
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

int launch_elem_dim(pf_problem* pb, const AlloyConst& C, int mode, const double* U,
                    const double* Uprev, const double* v, const double* eps_dev, double* coef,
                    hipStream_t s) {
  if (pb->geo.dim == 3) return launch_elem<3>(pb, C, mode, U, Uprev, v, eps_dev, coef, s);
  return launch_elem<2>(pb, C, mode, U, Uprev, v, eps_dev, coef, s);
}

}  // namespace

AlloyConst alloy_const(const pf_problem* pb, double t, double theta, int use_hist) {
  const pf_alloy_params& a = pb->alloy;
  AlloyConst C{};
  C.omk = 1.0 - a.k;
  C.hopk = 0.5 * (1.0 + a.k);
  C.g4a = 1.0 / a.l_T;
  C.g4b = -(a.x_iso + a.v_pull * t) / a.l_T;
  C.x0 = -pb->params.half_width[0];
  C.h0 = pb->geo.h[0];
  C.theta = theta;
  C.use_hist = use_hist;
  return C;
}

int launch_alloy(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
                 const double* F0, const double* eps_dev, double* out0, double* coef,
                 hipStream_t s) {
  if (mode != MODE_RES && mode != MODE_FD && mode != MODE_JVP) {
    set_error("the alloy model has no VJP");
    return PF_ERR_INVALID_ARG;
  }
  const AlloyConst C = alloy_const(pb, pb->t_new, pb->params.theta, 1);
  PF_TRY(launch_elem_dim(pb, C, mode, U, Uprev, v, eps_dev, coef, s));
  return launch_gather2(pb, out0, F0, eps_dev, mode == MODE_FD ? 1 : 0, s);
}

int alloy_explicit(pf_problem* pb, const double* Un, double t_n, double* E, hipStream_t s) {
  const double th = pb->params.theta;
  if (th == 1.0) {
    PF_HIP_CHECK(hipMemsetAsync(E, 0, pb->n_dof * sizeof(double), s));
    return PF_OK;
  }
  // the residual at (U^n; U^n) with weight 1 and no history is the spatial
  // operator at U^n: the time and rate terms vanish
  const AlloyConst C = alloy_const(pb, t_n, 1.0, 0);
  PF_TRY(launch_elem_dim(pb, C, MODE_RES, Un, Un, nullptr, nullptr, nullptr, s));
  PF_TRY(launch_gather2(pb, E, nullptr, nullptr, 0, s));
  return blas_axpby(1.0 - th, E, 0.0, E, E, pb->n_dof, s);
}

int history_rate(pf_problem* pb, const double* Un, const double* Unm1, hipStream_t s) {
  const long long n = pb->geo.n_nodes;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  const unsigned nb = (unsigned)blocks;
  hipLaunchKernelGGL(k_history, dim3(nb), dim3(256), 0, s, n,
                     reinterpret_cast<const double2*>(Un), reinterpret_cast<const double2*>(Unm1),
                     (1.0 - pb->params.theta) / pb->params.dt, pb->hist);
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace pf
