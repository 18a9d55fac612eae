// Q1 element evaluation by sum factorisation and the pointwise physics of the
// coupled phase-field residual, its tangent and its adjoint.
//
// Reference element [-1,1]^d, corners a = ax + 2 ay (+ 4 az) at xi_k = -1 for
// bit k = 0 and +1 for bit k = 1; 3 Gauss points per axis at -s, 0, s with
// s = sqrt(3/5), weights 5/9, 8/9, 5/9 (the 9- and 27-point rules of the
// paper, Secs. 4.1 and 4.2).  1-D basis values at the Gauss points:
//   B[g][0] = (1 - xi_g)/2,  B[g][1] = (1 + xi_g)/2,
// and physical derivatives -1/h, +1/h (constant along the axis).
//
// element_eval interpolates NF nodal fields (value and gradient) to every
// Gauss point plane by plane (z outermost, then y rows, then x points), calls
// the pointwise functor, and contracts its NO outputs (s, f) with the test
// functions:  out[o][a] += w_q (s_o N_a + f_o . grad N_a).
#pragma once

#include "pf_internal.h"

namespace pf {

struct Q1 {
  static constexpr double s = 0.77459666924148337704;  // sqrt(3/5)
  // B[g][0] and B[g][1]: 1-D basis values at Gauss point g
  __host__ __device__ static constexpr double b0(int g) {
    return g == 0 ? 0.5 * (1.0 + s) : (g == 1 ? 0.5 : 0.5 * (1.0 - s));
  }
  __host__ __device__ static constexpr double b1(int g) {
    return g == 0 ? 0.5 * (1.0 - s) : (g == 1 ? 0.5 : 0.5 * (1.0 + s));
  }
  __host__ __device__ static constexpr double w(int g) { return g == 1 ? 8.0 / 9.0 : 5.0 / 9.0; }
};

// ----------------------------------------------------------------- 3-D element
template <int NF, int NO, class Phys>
__device__ __forceinline__ void element_eval3(const double (&nod)[NF][8], double (&out)[NO][8],
                                              const Geo& G, Phys& phys) {
  const double ihx = G.ih[0], ihy = G.ih[1], ihz = G.ih[2];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int a = 0; a < 8; ++a) out[o][a] = 0.0;

  // z-derivatives of the nodal fields on the 4 (ax, ay) lines
  double dz[NF][4];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int a = 0; a < 4; ++a) dz[f][a] = (nod[f][a + 4] - nod[f][a]) * ihz;

#pragma unroll 1
  for (int gz = 0; gz < 3; ++gz) {
    const double bz0 = Q1::b0(gz), bz1 = Q1::b1(gz);
    double pz[NF][4];  // field interpolated to the plane, at the 4 (ax, ay) corners
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int a = 0; a < 4; ++a) pz[f][a] = bz0 * nod[f][a] + bz1 * nod[f][a + 4];
    double S[NO][4], Zc[NO][4];  // plane contraction accumulators
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int a = 0; a < 4; ++a) { S[o][a] = 0.0; Zc[o][a] = 0.0; }

#pragma unroll
    for (int gy = 0; gy < 3; ++gy) {
      const double by0 = Q1::b0(gy), by1 = Q1::b1(gy);
      double qv[NF][2], qy[NF][2], qz[NF][2];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
          qv[f][ax] = by0 * pz[f][ax] + by1 * pz[f][ax + 2];
          qy[f][ax] = (pz[f][ax + 2] - pz[f][ax]) * ihy;
          qz[f][ax] = by0 * dz[f][ax] + by1 * dz[f][ax + 2];
        }
      double rs[NO][2], rx[NO], ry[NO][2], rz[NO][2];  // row accumulators
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        rx[o] = 0.0;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) { rs[o][ax] = 0.0; ry[o][ax] = 0.0; rz[o][ax] = 0.0; }
      }
#pragma unroll
      for (int gx = 0; gx < 3; ++gx) {
        const double bx0 = Q1::b0(gx), bx1 = Q1::b1(gx);
        double v[NF], g[NF][3];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          v[f] = bx0 * qv[f][0] + bx1 * qv[f][1];
          g[f][0] = (qv[f][1] - qv[f][0]) * ihx;
          g[f][1] = bx0 * qy[f][0] + bx1 * qy[f][1];
          g[f][2] = bx0 * qz[f][0] + bx1 * qz[f][1];
        }
        double s[NO], fl[NO][3];
        phys(v, g, s, fl);
        const double wq = Q1::w(gx) * Q1::w(gy) * Q1::w(gz) * G.jac;
        phys.weight(wq);
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const double ws = wq * s[o], wx = wq * fl[o][0], wy = wq * fl[o][1], wz = wq * fl[o][2];
          rs[o][0] += ws * bx0;
          rs[o][1] += ws * bx1;
          rx[o] += wx;
          ry[o][0] += wy * bx0;
          ry[o][1] += wy * bx1;
          rz[o][0] += wz * bx0;
          rz[o][1] += wz * bx1;
        }
      }
      // contract the row in y: corners (ax, ay) -> index ax + 2 ay
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        const double sx0 = rs[o][0] - rx[o] * ihx;  // s N + f_x dN/dx for ax = 0
        const double sx1 = rs[o][1] + rx[o] * ihx;  // ax = 1
        S[o][0] += by0 * sx0 - ry[o][0] * ihy;
        S[o][1] += by0 * sx1 - ry[o][1] * ihy;
        S[o][2] += by1 * sx0 + ry[o][0] * ihy;
        S[o][3] += by1 * sx1 + ry[o][1] * ihy;
        Zc[o][0] += by0 * rz[o][0];
        Zc[o][1] += by0 * rz[o][1];
        Zc[o][2] += by1 * rz[o][0];
        Zc[o][3] += by1 * rz[o][1];
      }
    }
    // contract the plane in z
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        out[o][a] += bz0 * S[o][a] - Zc[o][a] * ihz;
        out[o][a + 4] += bz1 * S[o][a] + Zc[o][a] * ihz;
      }
  }
}

// ----------------------------------------------------------------- 2-D element
template <int NF, int NO, class Phys>
__device__ __forceinline__ void element_eval2(const double (&nod)[NF][4], double (&out)[NO][4],
                                              const Geo& G, Phys& phys) {
  const double ihx = G.ih[0], ihy = G.ih[1];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int a = 0; a < 4; ++a) out[o][a] = 0.0;
#pragma unroll
  for (int gy = 0; gy < 3; ++gy) {
    const double by0 = Q1::b0(gy), by1 = Q1::b1(gy);
    double qv[NF][2], qy[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        qv[f][ax] = by0 * nod[f][ax] + by1 * nod[f][ax + 2];
        qy[f][ax] = (nod[f][ax + 2] - nod[f][ax]) * ihy;
      }
    double rs[NO][2], rx[NO], ry[NO][2];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      rx[o] = 0.0;
      rs[o][0] = rs[o][1] = ry[o][0] = ry[o][1] = 0.0;
    }
#pragma unroll
    for (int gx = 0; gx < 3; ++gx) {
      const double bx0 = Q1::b0(gx), bx1 = Q1::b1(gx);
      double v[NF], g[NF][3];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        v[f] = bx0 * qv[f][0] + bx1 * qv[f][1];
        g[f][0] = (qv[f][1] - qv[f][0]) * ihx;
        g[f][1] = bx0 * qy[f][0] + bx1 * qy[f][1];
        g[f][2] = 0.0;
      }
      double s[NO], fl[NO][3];
      phys(v, g, s, fl);
      const double wq = Q1::w(gx) * Q1::w(gy) * G.jac;
      phys.weight(wq);
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        const double ws = wq * s[o], wx = wq * fl[o][0], wy = wq * fl[o][1];
        rs[o][0] += ws * bx0;
        rs[o][1] += ws * bx1;
        rx[o] += wx;
        ry[o][0] += wy * bx0;
        ry[o][1] += wy * bx1;
      }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const double sx0 = rs[o][0] - rx[o] * ihx;
      const double sx1 = rs[o][1] + rx[o] * ihx;
      out[o][0] += by0 * sx0 - ry[o][0] * ihy;
      out[o][1] += by0 * sx1 - ry[o][1] * ihy;
      out[o][2] += by1 * sx0 + ry[o][0] * ihy;
      out[o][3] += by1 * sx1 + ry[o][1] * ihy;
    }
  }
}

// ----------------------------------------------------------------- pointwise physics
// Anisotropy a(g) = 1 - 3 eps4 + 4 eps4 S/Q^2, Q = |g|^2 + delta2, S = sum g^4,
// its gradient da/dg_k = 16 eps4 g_k (g_k^2 - S/Q)/Q^2 and the flux
// J = a^2 g + a |g|^2 da/dg (gradient of a^2 |g|^2 / 2).
template <int DIM>
struct Aniso {
  double q, S, iQ, a, da[3], J[3];
  __device__ __forceinline__ void eval(const double* g, double eps4, double delta2) {
    double g2[3];
    q = 0.0;
    S = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      g2[k] = g[k] * g[k];
      q += g2[k];
      S += g2[k] * g2[k];
    }
    const double Q = q + delta2;
    iQ = 1.0 / Q;
    const double iQ2 = iQ * iQ;
    a = 1.0 - 3.0 * eps4 + 4.0 * eps4 * S * iQ2;
    const double SQ = S * iQ;
    const double c = 16.0 * eps4 * iQ2;
    const double a2 = a * a, aq = a * q;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      da[k] = c * g[k] * (g2[k] - SQ);
      J[k] = a2 * g[k] + aq * da[k];
    }
  }
  // H v with H the Hessian of a^2 |g|^2 / 2:
  // H v = a^2 v + 2a (g (da.v) + da (g.v)) + q da (da.v) + a q 4 eps4 T v,
  // T v = 12 g^2 v/Q^2 - 16 (g^3 (g.v) + g (g^3.v))/Q^3 - 4 S v/Q^3 + 24 S g (g.v)/Q^4.
  __device__ __forceinline__ void hess(const double* g, const double* v, double eps4,
                                       double* Hv) const {
    double gv = 0.0, dav = 0.0, g3v = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      gv += g[k] * v[k];
      dav += da[k] * v[k];
      g3v += g[k] * g[k] * g[k] * v[k];
    }
    const double iQ2 = iQ * iQ, iQ3 = iQ2 * iQ, iQ4 = iQ2 * iQ2;
    const double a2 = a * a;
    const double c4 = 4.0 * eps4 * a * q;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double gk = g[k];
      const double Tv = 12.0 * gk * gk * v[k] * iQ2 - 16.0 * (gk * gk * gk * gv + gk * g3v) * iQ3 -
                        4.0 * S * v[k] * iQ3 + 24.0 * S * gk * gv * iQ4;
      Hv[k] = a2 * v[k] + 2.0 * a * (gk * dav + da[k] * gv) + q * da[k] * dav + c4 * Tv;
    }
  }
};

// Residual: fields {phi, u, phi - phi^n, u - u^n}; outputs {F1, F2}.
template <int DIM>
struct PhysResidual {
  const Geo& G;
  __device__ PhysResidual(const Geo& g) : G(g) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void operator()(const double* v, const double (*g)[3], double* s,
                                             double (*f)[3]) {
    const double phi = v[0], u = v[1], dphi = v[2], du = v[3];
    Aniso<DIM> A;
    A.eval(g[0], G.eps4, G.delta2);
    const double p2 = phi * phi;
    const double om = 1.0 - p2;
    const double R = phi - p2 * phi - G.lam * om * om * u;
    s[0] = A.a * A.a * dphi * G.idt - R;
    s[1] = (du - 0.5 * dphi) * G.idt;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[0][k] = (k < DIM) ? A.J[k] : 0.0;
      f[1][k] = (k < DIM) ? G.D * g[1][k] : 0.0;
    }
  }
};

// Tangent: fields {phi, u, phi - phi^n, dphi_tan, du_tan}; outputs {J1 v, J2 v}.
template <int DIM>
struct PhysJvp {
  const Geo& G;
  __device__ PhysJvp(const Geo& g) : G(g) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void operator()(const double* v, const double (*g)[3], double* s,
                                             double (*f)[3]) {
    const double phi = v[0], u = v[1], dphi = v[2], tp = v[3], tu = v[4];
    Aniso<DIM> A;
    A.eval(g[0], G.eps4, G.delta2);
    double dav = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dav += A.da[k] * g[3][k];
    const double p2 = phi * phi;
    const double om = 1.0 - p2;
    const double Rp = 1.0 - 3.0 * p2 + 4.0 * G.lam * phi * om * u;  // dR/dphi
    const double Ru = -G.lam * om * om;                              // dR/du
    s[0] = (2.0 * A.a * dav * dphi + A.a * A.a * tp) * G.idt - (Rp * tp + Ru * tu);
    s[1] = (tu - 0.5 * tp) * G.idt;
    double Hv[3] = {0.0, 0.0, 0.0};
    A.hess(g[0], g[3], G.eps4, Hv);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[0][k] = (k < DIM) ? Hv[k] : 0.0;
      f[1][k] = (k < DIM) ? G.D * g[4][k] : 0.0;
    }
  }
};

// Adjoint: fields {phi, u, phi - phi^n, w1, w2}; outputs {gU_phi, gU_u,
// gUprev_phi, gUprev_u}; accumulates w . dF/d eps4 and w . dF/d lambda.
template <int DIM>
struct PhysVjp {
  const Geo& G;
  double ge, gl;      // element accumulators
  double pe, pl;      // pointwise values (weighted in weight())
  __device__ PhysVjp(const Geo& g) : G(g), ge(0.0), gl(0.0), pe(0.0), pl(0.0) {}
  __device__ __forceinline__ void weight(double wq) {
    ge += wq * pe;
    gl += wq * pl;
  }
  __device__ __forceinline__ void operator()(const double* v, const double (*g)[3], double* s,
                                             double (*f)[3]) {
    const double phi = v[0], u = v[1], dphi = v[2], w1 = v[3], w2 = v[4];
    Aniso<DIM> A;
    A.eval(g[0], G.eps4, G.delta2);
    const double p2 = phi * phi;
    const double om = 1.0 - p2;
    const double Rp = 1.0 - 3.0 * p2 + 4.0 * G.lam * phi * om * u;
    const double a2 = A.a * A.a;
    double Hw[3] = {0.0, 0.0, 0.0};
    A.hess(g[0], g[3], G.eps4, Hw);
    const double m = 2.0 * A.a * dphi * G.idt * w1;  // d(a^2 dphi/dt w1)/da
    s[0] = w1 * (a2 * G.idt - Rp) - 0.5 * w2 * G.idt;
    s[1] = w1 * G.lam * om * om + w2 * G.idt;
    s[2] = -w1 * a2 * G.idt + 0.5 * w2 * G.idt;
    s[3] = -w2 * G.idt;
    // parameter derivatives: da/deps4 = -3 + 4 S/Q^2, d(da)/deps4 = da/eps4
    const double iQ2 = A.iQ * A.iQ;
    const double ae = -3.0 + 4.0 * A.S * iQ2;
    const double SQ = A.S * A.iQ;
    double Je_w = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double gk = g[0][k];
      const double dae = 16.0 * iQ2 * gk * (gk * gk - SQ);
      const double Je = 2.0 * A.a * ae * gk + ae * A.q * A.da[k] + A.a * A.q * dae;
      Je_w += Je * g[3][k];
    }
    pe = m * ae + Je_w;
    pl = w1 * om * om * u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[0][k] = (k < DIM) ? Hw[k] + m * A.da[k] : 0.0;
      f[1][k] = (k < DIM) ? G.D * g[4][k] : 0.0;
      f[2][k] = 0.0;
      f[3][k] = 0.0;
    }
  }
};

}  // namespace pf
