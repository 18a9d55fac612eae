// Q1 element evaluation for the coupled phase-field residual, its tangent and
// its adjoint.
//
// Reference element [-1,1]^d, corners a = ax + 2 ay (+ 4 az) at xi_k = -1 for
// bit k = 0 and +1 for bit k = 1; 3 Gauss points per axis at -s, 0, s with
// s = sqrt(3/5), weights 5/9, 8/9, 5/9 (the 9- and 27-point rules of the
// paper, Secs. 4.1 and 4.2).  1-D basis values at the Gauss points:
//   B[g][0] = (1 - xi_g)/2,  B[g][1] = (1 + xi_g)/2,
// and physical derivatives -1/h, +1/h (constant along the axis).
//
// Split of the work:
//  * nonlinear terms (anisotropic flux, a^2-weighted time term, lambda
//    coupling) are integrated with the Gauss rule: quad3/quad2 interpolate the
//    fields plane by plane (z outermost, then y rows, then x points), call the
//    pointwise functor and contract its outputs with the test functions,
//      out[o][a] += w_q (s_o N_a + f_o . grad N_a);
//  * linear constant-coefficient terms (u equation, latent heat) are applied
//    as the exact element mass and stiffness matrices in tensor-product form,
//    M_e = M1 x M1 (x M1), K_e = sum over axes of K1 on that axis and M1 on
//    the others, with M1 = h/6 [2 1; 1 2] and K1 = 1/h [1 -1; -1 1].  The
//    3-point rule integrates these exactly, so both routes give the same
//    discrete residual.
#pragma once

#include "pf_internal.h"

// Unroll factor of the y-row loop of the 3-D Gauss rule (the z-plane loop is
// not unrolled; the x-point and y-row loops are unrolled or not per physics
// functor, kGxUnroll and kGyUnroll, the latter taking this factor when not 1):
// a register-pressure / ILP trade-off.
#ifndef PF_GY_UNROLL
#define PF_GY_UNROLL 3
#endif
// The x-point loop of the tangent and adjoint functors: 3 unrolls it, 1 keeps
// it rolled.
#ifndef PF_TAN_GX_UNROLL
#define PF_TAN_GX_UNROLL 3
#endif
#define PF_PRAGMA(x) _Pragma(#x)
#define PF_UNROLL(n) PF_PRAGMA(unroll n)

namespace pf {

struct Q1 {
  static constexpr double s = 0.77459666924148337704;  // sqrt(3/5)
  __host__ __device__ static constexpr double b0(int g) {
    return g == 0 ? 0.5 * (1.0 + s) : (g == 1 ? 0.5 : 0.5 * (1.0 - s));
  }
  __host__ __device__ static constexpr double b1(int g) {
    return g == 0 ? 0.5 * (1.0 - s) : (g == 1 ? 0.5 : 0.5 * (1.0 + s));
  }
  __host__ __device__ static constexpr double w(int g) { return g == 1 ? 8.0 / 9.0 : 5.0 / 9.0; }
  // w(g) b0(g) and w(g) b1(g): the point weights of the two test-function halves
  __host__ __device__ static constexpr double c0(int g) { return w(g) * b0(g); }
  __host__ __device__ static constexpr double c1(int g) { return w(g) * b1(g); }
};

// ----------------------------------------------------------------- exact linear part
// y += cm M_e xm + ck K_e xk, 3-D, corners a = ax + 2 ay + 4 az.
__device__ __forceinline__ void mass_stiff3(const Geo& G, const double (&xm)[8], double cm,
                                            const double (&xk)[8], double ck, double (&y)[8]) {
  const double hx6 = G.h[0] / 6.0, hy6 = G.h[1] / 6.0, hz6 = G.h[2] / 6.0;
  double t[8], c[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) t[a] = hx6 * (2.0 * xm[a] + xm[a ^ 1]);
#pragma unroll
  for (int a = 0; a < 8; ++a) c[a] = hy6 * (2.0 * t[a] + t[a ^ 2]);
#pragma unroll
  for (int a = 0; a < 8; ++a) y[a] += cm * (hz6 * (2.0 * c[a] + c[a ^ 4]));
  // stiffness: Kx My Mz + Mx Ky Mz + Mx My Kz
  double mx[8], kx[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    mx[a] = hx6 * (2.0 * xk[a] + xk[a ^ 1]);
    kx[a] = (xk[a] - xk[a ^ 1]) * G.ih[0];
  }
  double mm[8], s2[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    mm[a] = hy6 * (2.0 * mx[a] + mx[a ^ 2]);                                 // Mx My
    s2[a] = hy6 * (2.0 * kx[a] + kx[a ^ 2]) + (mx[a] - mx[a ^ 2]) * G.ih[1];  // Kx My + Mx Ky
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
    y[a] += ck * (hz6 * (2.0 * s2[a] + s2[a ^ 4]) + (mm[a] - mm[a ^ 4]) * G.ih[2]);
}

__device__ __forceinline__ void mass_stiff2(const Geo& G, const double (&xm)[4], double cm,
                                            const double (&xk)[4], double ck, double (&y)[4]) {
  const double hx6 = G.h[0] / 6.0, hy6 = G.h[1] / 6.0;
  double t[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) t[a] = hx6 * (2.0 * xm[a] + xm[a ^ 1]);
#pragma unroll
  for (int a = 0; a < 4; ++a) y[a] += cm * (hy6 * (2.0 * t[a] + t[a ^ 2]));
  double mx[4], kx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    mx[a] = hx6 * (2.0 * xk[a] + xk[a ^ 1]);
    kx[a] = (xk[a] - xk[a ^ 1]) * G.ih[0];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
    y[a] += ck * (hy6 * (2.0 * kx[a] + kx[a ^ 2]) + (mx[a] - mx[a ^ 2]) * G.ih[1]);
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (each step squares the relative error), used instead of the IEEE division
// sequence in the pointwise physics.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// The same with one Newton step.  Measured on gfx950 over 4M positive values
// spanning 60 binades: the estimate is within 4.6e-8 relative, one step within
// 2.2e-15 (about 10 ulp), two steps correctly rounded in every case.  Used for
// the anisotropy's 1/Q, where 2.2e-15 is far below every tolerance the
// results are held to.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// ----------------------------------------------------------------- Gauss-rule part, 3-D
// NG fields interpolated with value and gradient (ng), NV fields with value
// only (nv); NS outputs with value and flux parts (os), NP value-only outputs
// (op).  The functor is called as phys(gv, gg, vv, s, f, p) at every point,
// phys.weight(w_x) right after with the point's x weight, and phys.row(w_row)
// at the end of each row of points with the row's weight (y, z weights and
// the Jacobian): point weight = w_x w_row.  Row sums are accumulated with the
// x weights only and scaled once per row.
//
// quad3g takes the corner values from load(gz, ng, nv), called at the start of
// every Gauss plane gz: a loader that reads them from memory each time keeps
// them out of registers between planes (quad3 passes register arrays).
//
// The element outputs are accumulated through acc: acc.s(o, a, c1, v1, c2, v2)
// adds c1 v1 + c2 v2 (two FMAs) to value-and-flux output o at corner a,
// acc.p(o, a, c, v) adds c v to value-only output o (RegAcc: register arrays;
// StridedAcc: a lane's slots in memory).
template <int NS, int NP>
struct RegAcc {
  double (&os)[NS > 0 ? NS : 1][8];
  double (&op)[NP > 0 ? NP : 1][8];
  __device__ __forceinline__ void s(int o, int a, double c1, double v1, double c2, double v2) {
    os[o][a] = fma(c2, v2, fma(c1, v1, os[o][a]));
  }
  __device__ __forceinline__ void p(int o, int a, double c, double v) { op[o][a] = fma(c, v, op[o][a]); }
};
// Output o, corner a at base_s[(o * 8 + a) * stride] (value-only outputs at
// base_p likewise).
struct StridedAcc {
  double* base_s;
  double* base_p;
  int stride;
  __device__ __forceinline__ void s(int o, int a, double c1, double v1, double c2, double v2) {
    double& x = base_s[(o * 8 + a) * stride];
    x = fma(c2, v2, fma(c1, v1, x));
  }
  __device__ __forceinline__ void p(int o, int a, double c, double v) {
    double& x = base_p[(o * 8 + a) * stride];
    x = fma(c, v, x);
  }
};

template <int NG, int NV, int NS, int NP, class Phys, class Load, class Acc>
__device__ __forceinline__ void quad3g(const Geo& G, Load& load, Acc& acc, Phys& phys) {
  const double ihx = G.ih[0], ihy = G.ih[1], ihz = G.ih[2];
#pragma unroll 1
  for (int gz = 0; gz < 3; ++gz) {
    const double bz0 = Q1::b0(gz), bz1 = Q1::b1(gz);
    double ng[NG][8], nv[NV > 0 ? NV : 1][8];
    load(gz, ng, nv);
    double pg[NG][4], dz[NG][4], pv[NV > 0 ? NV : 1][4];
    // b0 + b1 = 1: value = q0 + b1 (q1 - q0), and the difference also gives
    // the derivative along the axis
#pragma unroll
    for (int f = 0; f < NG; ++f)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double d = ng[f][a + 4] - ng[f][a];
        pg[f][a] = fma(bz1, d, ng[f][a]);
        dz[f][a] = d * ihz;
      }
#pragma unroll
    for (int f = 0; f < NV; ++f)
#pragma unroll
      for (int a = 0; a < 4; ++a) pv[f][a] = fma(bz1, nv[f][a + 4] - nv[f][a], nv[f][a]);
    double S[NS > 0 ? NS : 1][4], Zc[NS > 0 ? NS : 1][4], P[NP > 0 ? NP : 1][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int o = 0; o < NS; ++o) S[o][a] = Zc[o][a] = 0.0;
#pragma unroll
      for (int o = 0; o < NP; ++o) P[o][a] = 0.0;
    }
    auto row_of_points = [&](int gy) {
      const double by0 = Q1::b0(gy), by1 = Q1::b1(gy);
      const double wrow = Q1::w(gy) * Q1::w(gz) * G.jac;
      const double wb0 = wrow * by0, wb1 = wrow * by1, wih = wrow * ihy;
      double qv[NG][2], qy[NG][2], qz[NG][2], qw[NV > 0 ? NV : 1][2];
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          const double d = pg[f][ax + 2] - pg[f][ax];
          qv[f][ax] = fma(by1, d, pg[f][ax]);
          qy[f][ax] = d * ihy;
          qz[f][ax] = fma(by1, dz[f][ax + 2] - dz[f][ax], dz[f][ax]);
        }
#pragma unroll
        for (int f = 0; f < NV; ++f) qw[f][ax] = fma(by1, pv[f][ax + 2] - pv[f][ax], pv[f][ax]);
      }
      // differences along x, shared by the row's three points; the x
      // derivative is constant along a row of a Q1 element
      double dqv[NG], gxr[NG], dqy[NG], dqz[NG], dqw[NV > 0 ? NV : 1];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        dqv[f] = qv[f][1] - qv[f][0];
        gxr[f] = dqv[f] * ihx;
        dqy[f] = qy[f][1] - qy[f][0];
        dqz[f] = qz[f][1] - qz[f][0];
      }
#pragma unroll
      for (int f = 0; f < NV; ++f) dqw[f] = qw[f][1] - qw[f][0];
      double rs[NS > 0 ? NS : 1][2], rx[NS > 0 ? NS : 1], ry[NS > 0 ? NS : 1][2], rz[NS > 0 ? NS : 1][2], rp[NP > 0 ? NP : 1][2];
#pragma unroll
      for (int o = 0; o < NS; ++o) {
        rx[o] = 0.0;
        rs[o][0] = rs[o][1] = ry[o][0] = ry[o][1] = rz[o][0] = rz[o][1] = 0.0;
      }
#pragma unroll
      for (int o = 0; o < NP; ++o) rp[o][0] = rp[o][1] = 0.0;
      auto point = [&](int gx) {
        const double bx1 = Q1::b1(gx);
        double gv[NG], gg[NG][3], vv[NV > 0 ? NV : 1];
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          gv[f] = fma(bx1, dqv[f], qv[f][0]);
          gg[f][0] = gxr[f];
          gg[f][1] = fma(bx1, dqy[f], qy[f][0]);
          gg[f][2] = fma(bx1, dqz[f], qz[f][0]);
        }
#pragma unroll
        for (int f = 0; f < NV; ++f) vv[f] = fma(bx1, dqw[f], qw[f][0]);
        double s[NS > 0 ? NS : 1], fl[NS > 0 ? NS : 1][3], p[NP > 0 ? NP : 1];
        phys(gv, gg, vv, s, fl, p);
        const double wq = Q1::w(gx), w0 = Q1::c0(gx), w1 = Q1::c1(gx);
        phys.weight(wq);
#pragma unroll
        for (int o = 0; o < NS; ++o) {
          rs[o][0] = fma(s[o], w0, rs[o][0]);
          rs[o][1] = fma(s[o], w1, rs[o][1]);
          rx[o] = fma(fl[o][0], wq, rx[o]);
          ry[o][0] = fma(fl[o][1], w0, ry[o][0]);
          ry[o][1] = fma(fl[o][1], w1, ry[o][1]);
          rz[o][0] = fma(fl[o][2], w0, rz[o][0]);
          rz[o][1] = fma(fl[o][2], w1, rz[o][1]);
        }
#pragma unroll
        for (int o = 0; o < NP; ++o) {
          rp[o][0] = fma(p[o], w0, rp[o][0]);
          rp[o][1] = fma(p[o], w1, rp[o][1]);
        }
            };
      if constexpr (Phys::kGxUnroll == 1) {
#pragma unroll 1
        for (int gx = 0; gx < 3; ++gx) point(gx);
      } else {
#pragma unroll
        for (int gx = 0; gx < 3; ++gx) point(gx);
      }
      phys.row(wrow);
#pragma unroll
      for (int o = 0; o < NS; ++o) {
        const double sx0 = rs[o][0] - rx[o] * ihx;
        const double sx1 = rs[o][1] + rx[o] * ihx;
        S[o][0] = fma(-ry[o][0], wih, fma(wb0, sx0, S[o][0]));
        S[o][1] = fma(-ry[o][1], wih, fma(wb0, sx1, S[o][1]));
        S[o][2] = fma(ry[o][0], wih, fma(wb1, sx0, S[o][2]));
        S[o][3] = fma(ry[o][1], wih, fma(wb1, sx1, S[o][3]));
        Zc[o][0] += wb0 * rz[o][0];
        Zc[o][1] += wb0 * rz[o][1];
        Zc[o][2] += wb1 * rz[o][0];
        Zc[o][3] += wb1 * rz[o][1];
      }
#pragma unroll
      for (int o = 0; o < NP; ++o) {
        P[o][0] += wb0 * rp[o][0];
        P[o][1] += wb0 * rp[o][1];
        P[o][2] += wb1 * rp[o][0];
        P[o][3] += wb1 * rp[o][1];
      }
    };
    if constexpr (Phys::kGyUnroll == 1) {
#pragma unroll 1
      for (int gy = 0; gy < 3; ++gy) row_of_points(gy);
    } else {
PF_UNROLL(PF_GY_UNROLL)
      for (int gy = 0; gy < 3; ++gy) row_of_points(gy);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int o = 0; o < NS; ++o) {
        acc.s(o, a, bz0, S[o][a], -ihz, Zc[o][a]);
        acc.s(o, a + 4, bz1, S[o][a], ihz, Zc[o][a]);
      }
#pragma unroll
      for (int o = 0; o < NP; ++o) {
        acc.p(o, a, bz0, P[o][a]);
        acc.p(o, a + 4, bz1, P[o][a]);
      }
    }
  }
}

template <int NG, int NV, int NS, int NP, class Phys>
__device__ __forceinline__ void quad3(const Geo& G, const double (&ng)[NG][8],
                                     const double (&nv)[NV > 0 ? NV : 1][8], double (&os)[NS > 0 ? NS : 1][8],
                                     double (&op)[NP > 0 ? NP : 1][8], Phys& phys) {
  auto load = [&](int, double (&g)[NG][8], double (&v)[NV > 0 ? NV : 1][8]) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int f = 0; f < NG; ++f) g[f][a] = ng[f][a];
#pragma unroll
      for (int f = 0; f < (NV > 0 ? NV : 1); ++f) v[f][a] = nv[f][a];
    }
  };
  RegAcc<NS, NP> acc{os, op};
  quad3g<NG, NV, NS, NP>(G, load, acc, phys);
}

// ----------------------------------------------------------------- Gauss-rule part, 2-D
template <int NG, int NV, int NS, int NP, class Phys>
__device__ __forceinline__ void quad2(const Geo& G, const double (&ng)[NG][4],
                                     const double (&nv)[NV > 0 ? NV : 1][4], double (&os)[NS > 0 ? NS : 1][4],
                                     double (&op)[NP > 0 ? NP : 1][4], Phys& phys) {
  const double ihx = G.ih[0], ihy = G.ih[1];
#pragma unroll
  for (int gy = 0; gy < 3; ++gy) {
    const double by0 = Q1::b0(gy), by1 = Q1::b1(gy);
    const double wrow = Q1::w(gy) * G.jac;
    const double wb0 = wrow * by0, wb1 = wrow * by1, wih = wrow * ihy;
    double qv[NG][2], qy[NG][2], qw[NV > 0 ? NV : 1][2];
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        const double d = ng[f][ax + 2] - ng[f][ax];
        qv[f][ax] = fma(by1, d, ng[f][ax]);
        qy[f][ax] = d * ihy;
      }
#pragma unroll
      for (int f = 0; f < NV; ++f) qw[f][ax] = fma(by1, nv[f][ax + 2] - nv[f][ax], nv[f][ax]);
    }
    double dqv[NG], gxr[NG], dqy[NG], dqw[NV > 0 ? NV : 1];
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      dqv[f] = qv[f][1] - qv[f][0];
      gxr[f] = dqv[f] * ihx;
      dqy[f] = qy[f][1] - qy[f][0];
    }
#pragma unroll
    for (int f = 0; f < NV; ++f) dqw[f] = qw[f][1] - qw[f][0];
    double rs[NS > 0 ? NS : 1][2], rx[NS > 0 ? NS : 1], ry[NS > 0 ? NS : 1][2], rp[NP > 0 ? NP : 1][2];
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      rx[o] = 0.0;
      rs[o][0] = rs[o][1] = ry[o][0] = ry[o][1] = 0.0;
    }
#pragma unroll
    for (int o = 0; o < NP; ++o) rp[o][0] = rp[o][1] = 0.0;
#pragma unroll
    for (int gx = 0; gx < 3; ++gx) {
      const double bx1 = Q1::b1(gx);
      double gv[NG], gg[NG][3], vv[NV > 0 ? NV : 1];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        gv[f] = fma(bx1, dqv[f], qv[f][0]);
        gg[f][0] = gxr[f];
        gg[f][1] = fma(bx1, dqy[f], qy[f][0]);
        gg[f][2] = 0.0;
      }
#pragma unroll
      for (int f = 0; f < NV; ++f) vv[f] = fma(bx1, dqw[f], qw[f][0]);
      double s[NS > 0 ? NS : 1], fl[NS > 0 ? NS : 1][3], p[NP > 0 ? NP : 1];
      phys(gv, gg, vv, s, fl, p);
      const double wq = Q1::w(gx), w0 = Q1::c0(gx), w1 = Q1::c1(gx);
      phys.weight(wq);
#pragma unroll
      for (int o = 0; o < NS; ++o) {
        rs[o][0] = fma(s[o], w0, rs[o][0]);
        rs[o][1] = fma(s[o], w1, rs[o][1]);
        rx[o] = fma(fl[o][0], wq, rx[o]);
        ry[o][0] = fma(fl[o][1], w0, ry[o][0]);
        ry[o][1] = fma(fl[o][1], w1, ry[o][1]);
      }
#pragma unroll
      for (int o = 0; o < NP; ++o) {
        rp[o][0] = fma(p[o], w0, rp[o][0]);
        rp[o][1] = fma(p[o], w1, rp[o][1]);
      }
    }
    phys.row(wrow);
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      const double sx0 = rs[o][0] - rx[o] * ihx;
      const double sx1 = rs[o][1] + rx[o] * ihx;
      os[o][0] = fma(-ry[o][0], wih, fma(wb0, sx0, os[o][0]));
      os[o][1] = fma(-ry[o][1], wih, fma(wb0, sx1, os[o][1]));
      os[o][2] = fma(ry[o][0], wih, fma(wb1, sx0, os[o][2]));
      os[o][3] = fma(ry[o][1], wih, fma(wb1, sx1, os[o][3]));
    }
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      op[o][0] += wb0 * rp[o][0];
      op[o][1] += wb0 * rp[o][1];
      op[o][2] += wb1 * rp[o][0];
      op[o][3] += wb1 * rp[o][1];
    }
  }
}

// ----------------------------------------------------------------- pointwise physics
// Anisotropy a(g) = 1 - 3 eps4 + 4 eps4 S/Q^2, Q = |g|^2 + delta2, S = sum g^4,
// its gradient da/dg_k = 16 eps4 g_k (g_k^2 - S/Q)/Q^2 and the flux
// J = a^2 g + a |g|^2 da/dg (gradient of a^2 |g|^2 / 2).
template <int DIM>
struct Aniso {
  // primal quantities kept for the tangent and adjoint: q = |g|^2, S = sum g^4,
  // iQ = 1/Q, iQ2 = 1/Q^2, a, a^2, b = 16 eps4/Q^2, aqc = a q b, SQ = S/Q,
  // g2_k = g_k^2 (da/dg_k = b g_k (g_k^2 - S/Q)); J is the flux, with
  // J_k = g_k t_k, t_k = a^2 + aqc (g_k^2 - S/Q) formed as
  // (a^2 - aqc S/Q) + aqc g_k^2 (one FMA per component).
  double q, S, iQ, iQ2, a, a2, b, aqc, SQ, g2[3], J[3];
  __device__ __forceinline__ void flux(const double* g, const Geo& G) {
    q = 0.0;
    S = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      g2[k] = g[k] * g[k];
      q += g2[k];
      S = fma(g2[k], g2[k], S);
    }
    iQ = rcp_nr1(q + G.delta2);
    iQ2 = iQ * iQ;
    a = fma(G.e4x4 * S, iQ2, G.a0);
    SQ = S * iQ;
    a2 = a * a;
    b = G.e16 * iQ2;
    aqc = (a * q) * b;
    const double K0 = fma(-aqc, SQ, a2);
#pragma unroll
    for (int k = 0; k < DIM; ++k) J[k] = g[k] * fma(aqc, g2[k], K0);
  }
  // Directional derivative along v (after flux()): out = (dJ/dg) v, the
  // Hessian of a^2 |g|^2 / 2 times v (symmetric), plus extra g_k (g_k^2 - S/Q)
  // when kExtra (the transposed product adds that multiple of da/dg), and
  // da = (da/dg) . v.  Forward-mode differentiation of flux(), with gv = g.v
  // and g3v = sum g_k^3 v_k:
  //   da = b (g3v - (S/Q) gv),  d(a^2) = 2 a da,  dq = 2 gv,
  //   d(S/Q) = (4 g3v - (S/Q) dq)/Q,
  //   d(aqc) = b (da q + a dq (1 - 2 q/Q))   (db = -2 b dq/Q),
  //   dt_k = d(a^2) + d(aqc) gm_k + 2 aqc g_k v_k - aqc d(S/Q),
  //   (Hv)_k = v_k t_k + g_k dt_k,
  // regrouped by component as
  //   out_k = v_k c_k + g_k (D g_k^2 + K1),  c_k = (a^2 - aqc S/Q) + 3 aqc g_k^2,
  //   D = d(aqc) + extra,  K1 = d(a^2) - aqc d(S/Q) - D S/Q:
  // c_k depends on the primal only: three operations per component.
  // gvo = g.v and gmv = sum g_k gm_k v_k = g3v - (S/Q) gv are returned too.
  template <bool kExtra>
  __device__ __forceinline__ void hvp_c(const double* g, const double* v, double extra,
                                        double* out, double& da, double& gvo, double& gmv) const {
    double gv = 0.0, g3v = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double gvk = g[k] * v[k];
      gv += gvk;
      g3v = fma(g2[k], gvk, g3v);
    }
    gvo = gv;
    gmv = fma(-SQ, gv, g3v);
    da = b * gmv;
    const double dq = gv + gv;
    const double da2 = (a + a) * da;
    const double dSQ = iQ * fma(4.0, g3v, -SQ * dq);
    const double daqc = b * fma(da, q, (a * dq) * fma(-2.0 * q, iQ, 1.0));
    const double D = kExtra ? daqc + extra : daqc;
    const double K1 = fma(-D, SQ, fma(-aqc, dSQ, da2));
    const double K0 = fma(-aqc, SQ, a2);
    const double aqc3 = 3.0 * aqc;
#pragma unroll
    for (int k = 0; k < DIM; ++k) out[k] = fma(v[k], fma(aqc3, g2[k], K0), g[k] * fma(D, g2[k], K1));
  }
};

// Residual F1 (Gauss part): gradient field {phi}; value fields {u, phi - phi^n};
// output s = a^2 (phi - phi^n)/dt - (phi - phi^3 - lambda (1 - phi^2)^2 u), f = J.
template <int DIM>
struct PhysResidual {
  // all three points of a row unrolled, rows one at a time: more independent
  // work per row within the two-waves-per-SIMD register budget
  static constexpr int kGxUnroll = 3;
  static constexpr int kGyUnroll = 1;
  const Geo& G;
  double ca;   // sum of w_q a^2 over the element (preconditioner coefficient)
  double car;  // the current row's sum of w_x a^2
  double a2;
  __device__ PhysResidual(const Geo& g) : G(g), ca(0.0), car(0.0), a2(0.0) {}
  __device__ __forceinline__ void weight(double wx) { car = fma(wx, a2, car); }
  __device__ __forceinline__ void row(double wrow) {
    ca = fma(wrow, car, ca);
    car = 0.0;
  }
  // vv[1] holds (phi - phi^n)/dt
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const double phi = gv[0], u = vv[0], dphi_dt = vv[1];
    Aniso<DIM> A;
    A.flux(gg[0], G);
    a2 = A.a * A.a;
    const double om = fma(-phi, phi, 1.0);
    const double R = om * fma(-G.lam * om, u, phi);  // phi - phi^3 - lambda (1-phi^2)^2 u
    s[0] = fma(a2, dphi_dt, -R);
#pragma unroll
    for (int k = 0; k < 3; ++k) f[0][k] = (k < DIM) ? A.J[k] : 0.0;
  }
};

// Tangent of F1 (Gauss part): gradient fields {phi, v_phi}; value fields
// {u, phi - phi^n, v_u}.
template <int DIM>
struct PhysJvp {
  static constexpr int kGxUnroll = PF_TAN_GX_UNROLL;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  __device__ PhysJvp(const Geo& g) : G(g) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void row(double) {}
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double*) {
    const double phi = gv[0], tp = gv[1], u = vv[0], dphi = vv[1], tu = vv[2];
    Aniso<DIM> A;
    A.flux(gg[0], G);
    double Hv[3] = {0.0, 0.0, 0.0};
    double dav, gtv, gmv;
    A.template hvp_c<false>(gg[0], gg[1], 0.0, Hv, dav, gtv, gmv);
    // dR/dphi = 1 - 3 phi^2 + 4 lambda phi (1 - phi^2) u = (1 - phi^2)(3 + 4 lambda phi u) - 2,
    // dR/du = -lambda (1 - phi^2)^2
    const double om = fma(-phi, phi, 1.0);
    const double Rp = fma(om, fma(4.0 * G.lam * phi, u, 3.0), -2.0);
    const double Rv = fma(Rp, tp, (-G.lam * om) * (om * tu));  // dR/dphi tp + dR/du tu
    s[0] = fma(fma((A.a + A.a) * dav, dphi, A.a2 * tp), G.idtm, -Rv);
#pragma unroll
    for (int k = 0; k < 3; ++k) f[0][k] = (k < DIM) ? Hv[k] : 0.0;
  }
};

// Adjoint of F1 (Gauss part): gradient fields {phi, w1}; value fields
// {u, phi - phi^n}; outputs: gU_phi (value + flux), value-only gU_u (lambda
// term) and gUprev_phi (time term); accumulates w1 . dF1/d eps4 and
// w1 . dF1/d lambda (F2 does not depend on the parameters).
template <int DIM>
struct PhysVjp {
  static constexpr int kGxUnroll = PF_TAN_GX_UNROLL;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  double ge, gl;    // element accumulators
  double ger, glr;  // the current row's sums with the x weights
  double pe, pl;    // pointwise values (weighted in weight())
  __device__ PhysVjp(const Geo& g)
      : G(g), ge(0.0), gl(0.0), ger(0.0), glr(0.0), pe(0.0), pl(0.0) {}
  __device__ __forceinline__ void weight(double wx) {
    ger = fma(wx, pe, ger);
    glr = fma(wx, pl, glr);
  }
  __device__ __forceinline__ void row(double wrow) {
    ge = fma(wrow, ger, ge);
    gl = fma(wrow, glr, gl);
    ger = glr = 0.0;
  }
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double* p) {
    const double phi = gv[0], w1 = gv[1], u = vv[0], dphi = vv[1];
    Aniso<DIM> A;
    A.flux(gg[0], G);
    const double p2 = phi * phi;
    const double om = 1.0 - p2;
    const double Rp = 1.0 - 3.0 * p2 + 4.0 * G.lam * phi * om * u;
    const double m = 2.0 * A.a * dphi * G.idtm * w1;  // d(a^2 dphi idtm w1)/da
    s[0] = w1 * (A.a2 * G.idtm - Rp);
    p[0] = w1 * G.lam * om * om;
    p[1] = -w1 * A.a2 * G.idtm;
    // flux part: H w + m da/dg, da/dg_k = b g_k gm_k
    double fw[3] = {0.0, 0.0, 0.0};
    double daw, gw, gmw;
    A.template hvp_c<true>(gg[0], gg[1], m * A.b, fw, daw, gw, gmw);
#pragma unroll
    for (int k = 0; k < 3; ++k) f[0][k] = (k < DIM) ? fw[k] : 0.0;
    // parameter derivatives: da/deps4 = ae = -3 + 4 S/Q^2; d(da/dg_k)/deps4 = dae_k =
    // 16 g_k gm_k/Q^2, and da/dg_k = eps4 dae_k; J_k = a^2 g_k + a q da/dg_k, so
    // dJ_k/deps4 = 2 a ae g_k + (ae q eps4 + a q) dae_k and, summed against w,
    // w . dJ/deps4 = 2 a ae (g.w) + (ae q eps4 + a q) 16/Q^2 sum_k g_k gm_k w_k
    const double ae = fma(4.0 * A.S, A.iQ2, -3.0);
    const double C16 = fma(ae * A.q, G.eps4, A.a * A.q) * (16.0 * A.iQ2);
    const double Je_w = fma((A.a + A.a) * ae, gw, C16 * gmw);
    pe = m * ae + Je_w;
    pl = w1 * om * om * u;
  }
};

// Adjoint of F1 restricted to (dF1/dU)^T w1: gradient fields {phi, w1}; value
// fields {u, phi - phi^n}; outputs gU_phi (value + flux) and value-only gU_u.
template <int DIM>
struct PhysVjpU {
  static constexpr int kGxUnroll = PF_TAN_GX_UNROLL;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  __device__ PhysVjpU(const Geo& g) : G(g) {}
  __device__ __forceinline__ void weight(double) {}
  __device__ __forceinline__ void row(double) {}
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double* s, double (*f)[3],
                                             double* p) {
    const double phi = gv[0], w1 = gv[1], u = vv[0], dphi = vv[1];
    Aniso<DIM> A;
    A.flux(gg[0], G);
    const double om = fma(-phi, phi, 1.0);
    const double Rp = fma(om, fma(4.0 * G.lam * phi, u, 3.0), -2.0);  // as in PhysJvp
    const double m = (A.a * dphi) * ((G.idtm + G.idtm) * w1);
    s[0] = w1 * fma(A.a2, G.idtm, -Rp);
    p[0] = (w1 * G.lam) * (om * om);
    // H w + m da/dg = H w + m b g_k gm_k
    double fw[3] = {0.0, 0.0, 0.0};
    double daw, gw, gmw;
    A.template hvp_c<true>(gg[0], gg[1], m * A.b, fw, daw, gw, gmw);
#pragma unroll
    for (int k = 0; k < 3; ++k) f[0][k] = (k < DIM) ? fw[k] : 0.0;
  }
};

// Adjoint of F1 with respect to the previous state and the parameters only:
// gradient fields {phi, w1}; value fields {u, phi - phi^n}; one value-only
// output, gUprev_phi (time term); the parameter sums as PhysVjp.  No
// (dF1/dU)^T w1 part, so no Hessian-vector product.
template <int DIM>
struct PhysVjpPrev {
  static constexpr int kGxUnroll = PF_TAN_GX_UNROLL;
  static constexpr int kGyUnroll = PF_GY_UNROLL;
  const Geo& G;
  double ge, gl;
  double ger, glr;
  double pe, pl;
  __device__ PhysVjpPrev(const Geo& g)
      : G(g), ge(0.0), gl(0.0), ger(0.0), glr(0.0), pe(0.0), pl(0.0) {}
  __device__ __forceinline__ void weight(double wx) {
    ger = fma(wx, pe, ger);
    glr = fma(wx, pl, glr);
  }
  __device__ __forceinline__ void row(double wrow) {
    ge = fma(wrow, ger, ge);
    gl = fma(wrow, glr, gl);
    ger = glr = 0.0;
  }
  __device__ __forceinline__ void operator()(const double* gv, const double (*gg)[3],
                                             const double* vv, double*, double (*)[3],
                                             double* p) {
    const double phi = gv[0], w1 = gv[1], u = vv[0], dphi = vv[1];
    Aniso<DIM> A;
    A.flux(gg[0], G);
    const double om = 1.0 - phi * phi;
    const double m = 2.0 * A.a * dphi * G.idtm * w1;
    p[0] = -w1 * A.a2 * G.idtm;
    // w . dJ/deps4 as in PhysVjp: 2 a ae (g.w) + (ae q eps4 + a q) 16/Q^2 sum_k g_k gm_k w_k
    double gw = 0.0, g3w = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double gwk = gg[0][k] * gg[1][k];
      gw += gwk;
      g3w = fma(A.g2[k], gwk, g3w);
    }
    const double ae = fma(4.0 * A.S, A.iQ2, -3.0);
    const double C16 = fma(ae * A.q, G.eps4, A.a * A.q) * (16.0 * A.iQ2);
    const double Je_w = fma((A.a + A.a) * ae, gw, C16 * fma(-A.SQ, gw, g3w));
    pe = m * ae + Je_w;
    pl = w1 * om * om * u;
  }
};

// ----------------------------------------------------------------- whole-element routine
// Corner values (a = 0 .. 2^DIM - 1): u0/u1 = (phi, u) of the state, p0/p1 =
// (phi^n, u^n), v0/v1 = direction (JVP) or cotangent (VJP) parts.  For the FD
// product the caller passes the perturbed state as u0/u1.  out[0..1][a] are the
// two fields of the output vector; for the VJP out[2..3][a] those of gUprev.
// ge, gl: VJP parameter sums; for the residual ge is the cell integral of a^2.
template <int DIM, int MODE>
struct Element {
  static constexpr int NA = 1 << DIM;
  static constexpr int NO = MODE == MODE_VJP ? 4 : 2;

  template <int NG, int NV, int NS, int NP, class Phys>
  __device__ __forceinline__ static void quad(const Geo& G, const double (&ng)[NG][NA],
                                              const double (&nv)[NV][NA], double (&os)[NS > 0 ? NS : 1][NA],
                                              double (&op)[NP > 0 ? NP : 1][NA], Phys& ph) {
    if constexpr (DIM == 3) quad3<NG, NV, NS, NP>(G, ng, nv, os, op, ph);
    else quad2<NG, NV, NS, NP>(G, ng, nv, os, op, ph);
  }

  __device__ __forceinline__ static void lin(const Geo& G, const double (&xm)[NA], double cm,
                                             const double (&xk)[NA], double ck, double (&y)[NA]) {
    if constexpr (DIM == 3) mass_stiff3(G, xm, cm, xk, ck, y);
    else mass_stiff2(G, xm, cm, xk, ck, y);
  }

  // The tangent and adjoint modes (3-D) with corner values read on demand:
  // src.plane(gz) is called before Gauss plane gz's corner reads and
  // src.loaded(gz) after them; src.corner(a, u, p, v) gives the (phi, u)
  // pairs of the state, the previous state and the direction/cotangent at
  // corner a.  The linear part re-reads the direction after the Gauss rule, so
  // no corner value is held in registers across planes.  The element vector
  // is left in memory: output field o at corner a in src.out(o)[a *
  // src.stride()].  The analytic product and the transposed product
  // accumulate their Gauss-rule outputs there directly (no register
  // accumulators); the others accumulate in registers and store at the end.
  template <class Src>
  __device__ __forceinline__ static void run_src(const Geo& G, Src& src, double& ge, double& gl) {
    static_assert(DIM == 3 && MODE != MODE_RES && MODE != MODE_FD, "tangent and adjoint modes only");
    const int T = src.stride();
    if constexpr (MODE == MODE_JVP) {
      auto load = [&](int gz, double (&ng)[2][NA], double (&nv)[3][NA]) {
        src.plane(gz);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          double2 u, p, v;
          src.corner(a, u, p, v);
          ng[0][a] = u.x;
          ng[1][a] = v.x;
          nv[0][a] = u.y;
          nv[1][a] = u.x - p.x;
          nv[2][a] = v.y;
        }
        src.loaded(gz);
      };
      double* o0 = src.out(0);
      double* o1 = src.out(1);
#pragma unroll
      for (int a = 0; a < NA; ++a) o0[a * T] = 0.0;
      StridedAcc acc{o0, nullptr, T};
      PhysJvp<DIM> ph(G);
      quad3g<2, 3, 1, 0>(G, load, acc, ph);
      // d F2 = M (v_u - theta v_phi/2)/dt + theta D K v_u
      double y[NA], v1[NA], f2[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        double2 u, p, v;
        src.corner(a, u, p, v);
        v1[a] = v.y;
        y[a] = v.y - G.hth * v.x;
        f2[a] = 0.0;
        o0[a * T] = G.theta * o0[a * T];
      }
      lin(G, y, G.idt, v1, G.Dth, f2);
#pragma unroll
      for (int a = 0; a < NA; ++a) o1[a * T] = f2[a];
    } else {
      // adjoint modes: gradient fields {phi, w1}, value fields {u, phi - phi^n}
      auto load = [&](int gz, double (&ng)[2][NA], double (&nv)[2][NA]) {
        src.plane(gz);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          double2 u, p, v;
          src.corner(a, u, p, v);
          ng[0][a] = u.x;
          ng[1][a] = v.x;
          nv[0][a] = u.y;
          nv[1][a] = u.x - p.x;
        }
        src.loaded(gz);
      };
      double zero[NA], w2[NA];
      if constexpr (MODE == MODE_VJPU) {
        double* o0 = src.out(0);
        double* o1 = src.out(1);
#pragma unroll
        for (int a = 0; a < NA; ++a) o0[a * T] = o1[a * T] = 0.0;
        StridedAcc acc{o0, o1, T};
        PhysVjpU<DIM> ph(G);
        quad3g<2, 2, 1, 1>(G, load, acc, ph);
        // F2 part: gU_phi -= theta M w2/(2dt), gU_u += M w2/dt + theta D K w2
        double y[NA], f0[NA], f1[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          double2 u, p, v;
          src.corner(a, u, p, v);
          w2[a] = v.y;
          y[a] = G.idt * v.y;
          zero[a] = 0.0;
          f0[a] = G.theta * o0[a * T];
          f1[a] = G.theta * o1[a * T];
        }
        lin(G, y, 1.0, w2, G.Dth, f1);
        lin(G, y, -G.hth, zero, 0.0, f0);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          o0[a * T] = f0[a];
          o1[a * T] = f1[a];
        }
      } else if constexpr (MODE == MODE_VJPP) {
        double os[1][NA], op[1][NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) op[0][a] = 0.0;
        RegAcc<0, 1> acc{os, op};
        PhysVjpPrev<DIM> ph(G);
        quad3g<2, 2, 0, 1>(G, load, acc, ph);
        double mw[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          double2 u, p, v;
          src.corner(a, u, p, v);
          w2[a] = v.y;
          zero[a] = mw[a] = 0.0;
        }
        lin(G, w2, 1.0, zero, 0.0, mw);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          src.out(0)[a * T] = G.theta * op[0][a] + G.hth * G.idt * mw[a];
          src.out(1)[a * T] = -G.idt * mw[a];
        }
        ge = G.theta * ph.ge;
        gl = G.theta * ph.gl;
      } else {
        double os[1][NA], op[2][NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) os[0][a] = op[0][a] = op[1][a] = 0.0;
        RegAcc<1, 2> acc{os, op};
        PhysVjp<DIM> ph(G);
        quad3g<2, 2, 1, 2>(G, load, acc, ph);
        // F2 part (M, K symmetric): gU_phi -= theta M w2/(2dt), gU_u += M w2/dt +
        // theta D K w2, gUprev_phi += theta M w2/(2dt), gUprev_u -= M w2/dt
        double mw[NA], kw[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          double2 u, p, v;
          src.corner(a, u, p, v);
          w2[a] = v.y;
          zero[a] = mw[a] = kw[a] = 0.0;
        }
        lin(G, w2, 1.0, zero, 0.0, mw);
        lin(G, zero, 0.0, w2, G.Dth, kw);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          src.out(0)[a * T] = G.theta * os[0][a] - G.hth * G.idt * mw[a];
          src.out(1)[a * T] = G.theta * op[0][a] + G.idt * mw[a] + kw[a];
          src.out(2)[a * T] = G.theta * op[1][a] + G.hth * G.idt * mw[a];
          src.out(3)[a * T] = -G.idt * mw[a];
        }
        ge = G.theta * ph.ge;
        gl = G.theta * ph.gl;
      }
    }
  }

  __device__ __forceinline__ static void run(const Geo& G, const double (&u0)[NA],
                                             const double (&u1)[NA], const double (&p0)[NA],
                                             const double (&p1)[NA], const double (&v0)[NA],
                                             const double (&v1)[NA], double (&out)[NO][NA],
                                             double& ge, double& gl) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int a = 0; a < NA; ++a) out[o][a] = 0.0;
    double dphi[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) dphi[a] = u0[a] - p0[a];
    double dummy[1][NA];
    if constexpr (MODE == MODE_RES || MODE == MODE_FD) {
      // F2 = M (du - theta dphi/2)/dt + theta D K u
      double y[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) y[a] = (u1[a] - p1[a]) - G.hth * dphi[a];
      lin(G, y, G.idt, u1, G.Dth, out[1]);
      // F1 = theta [a^2 dphi/(theta dt) - R + J]: the Gauss rule sees the time
      // term over theta and the element vector is scaled once
      double ngv[1][NA], nvv[2][NA], os[1][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ngv[0][a] = u0[a];
        nvv[0][a] = u1[a];
        nvv[1][a] = dphi[a] * G.idtm;
        os[0][a] = 0.0;
      }
      PhysResidual<DIM> ph(G);
      quad<1, 2, 1, 0>(G, ngv, nvv, os, dummy, ph);
#pragma unroll
      for (int a = 0; a < NA; ++a) out[0][a] = G.theta * os[0][a];
      ge = ph.ca;  // cell integral of a^2 (the cell mean times the cell volume)
    } else if constexpr (MODE == MODE_JVP) {
      // d F2 = M (v_u - theta v_phi/2)/dt + theta D K v_u
      double y[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) y[a] = v1[a] - G.hth * v0[a];
      lin(G, y, G.idt, v1, G.Dth, out[1]);
      double ngv[2][NA], nvv[3][NA], os[1][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ngv[0][a] = u0[a];
        ngv[1][a] = v0[a];
        nvv[0][a] = u1[a];
        nvv[1][a] = dphi[a];
        nvv[2][a] = v1[a];
        os[0][a] = 0.0;
      }
      PhysJvp<DIM> ph(G);
      quad<2, 3, 1, 0>(G, ngv, nvv, os, dummy, ph);
#pragma unroll
      for (int a = 0; a < NA; ++a) out[0][a] = G.theta * os[0][a];
    } else if constexpr (MODE == MODE_VJPU) {
      double ngv[2][NA], nvv[2][NA], os[1][NA], op[1][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ngv[0][a] = u0[a];
        ngv[1][a] = v0[a];
        nvv[0][a] = u1[a];
        nvv[1][a] = dphi[a];
        os[0][a] = 0.0;
        op[0][a] = 0.0;
      }
      PhysVjpU<DIM> ph(G);
      quad<2, 2, 1, 1>(G, ngv, nvv, os, op, ph);
      // F2 part: gU_phi -= theta M w2/(2dt), gU_u += M w2/dt + theta D K w2
      double y[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        y[a] = G.idt * v1[a];
        out[0][a] = G.theta * os[0][a];
        out[1][a] = G.theta * op[0][a];
      }
      lin(G, y, 1.0, v1, G.Dth, out[1]);
      double zero[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) zero[a] = 0.0;
      lin(G, y, -G.hth, zero, 0.0, out[0]);
    } else if constexpr (MODE == MODE_VJPP) {
      // previous-state part of the adjoint: gUprev_phi = theta (time term) +
      // theta M w2/(2dt), gUprev_u = -M w2/dt; the parameter sums
      double zero[NA], mw[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) zero[a] = mw[a] = 0.0;
      lin(G, v1, 1.0, zero, 0.0, mw);
      double ngv[2][NA], nvv[2][NA], os[1][NA], op[1][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ngv[0][a] = u0[a];
        ngv[1][a] = v0[a];
        nvv[0][a] = u1[a];
        nvv[1][a] = dphi[a];
        op[0][a] = 0.0;
      }
      PhysVjpPrev<DIM> ph(G);
      quad<2, 2, 0, 1>(G, ngv, nvv, os, op, ph);
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        out[0][a] = G.theta * op[0][a] + G.hth * G.idt * mw[a];
        out[1][a] = -G.idt * mw[a];
      }
      ge = G.theta * ph.ge;
      gl = G.theta * ph.gl;
    } else {
      // F2 part of the adjoint (M, K symmetric): gU_phi -= theta M w2/(2dt),
      // gU_u += M w2/dt + theta D K w2, gUprev_phi += theta M w2/(2dt),
      // gUprev_u -= M w2/dt
      double zero[NA], mw[NA], kw[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) zero[a] = mw[a] = kw[a] = 0.0;
      lin(G, v1, 1.0, zero, 0.0, mw);
      lin(G, zero, 0.0, v1, G.Dth, kw);
      double ngv[2][NA], nvv[2][NA], os[1][NA], op[2][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ngv[0][a] = u0[a];
        ngv[1][a] = v0[a];
        nvv[0][a] = u1[a];
        nvv[1][a] = dphi[a];
        os[0][a] = op[0][a] = op[1][a] = 0.0;
      }
      PhysVjp<DIM> ph(G);
      quad<2, 2, 1, 2>(G, ngv, nvv, os, op, ph);
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        out[0][a] = G.theta * os[0][a] - G.hth * G.idt * mw[a];
        out[1][a] = G.theta * op[0][a] + G.idt * mw[a] + kw[a];
        out[2][a] = G.theta * op[1][a] + G.hth * G.idt * mw[a];
        out[3][a] = -G.idt * mw[a];
      }
      ge = G.theta * ph.ge;
      gl = G.theta * ph.gl;
    }
  }
};

}  // namespace pf
