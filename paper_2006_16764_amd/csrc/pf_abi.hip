// C ABI of libpfjfnk: handle management, the residual-family entry points,
// and the host drivers of the Newton-Krylov method (Sec. 2.2 of the paper):
// right-preconditioned flexible GMRES with classical Gram-Schmidt applied twice
// (FP64 Arnoldi, one host synchronisation per iteration), inexact Newton with
// the forcing term of Eqs. force1-forcing, the backtracking of Eq. glob and
// the termination test of Eq. tolerance; backward-Euler stepping and one step
// of its discrete adjoint.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "pf_internal.h"

namespace pf {

int elem_blocks(const pf_problem* pb);
constexpr int kNumTmp = 6;
static_assert(sizeof(((pf_problem*)nullptr)->tmp_vec) == kNumTmp * sizeof(double*), "tmp_vec size");

namespace {
thread_local std::string g_last_error;

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Start of a [sync] call's clock: the stream is drained first, so that work the
// caller queued before the call is not counted in its t_total_ms.
int clock_start(hipStream_t s, double* t0) {
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("hipStreamSynchronize failed before the call's work");
    return PF_ERR_HIP;
  }
  *t0 = now_ms();
  return PF_OK;
}

__global__ void k_misfit(Geo G, const double2* __restrict__ U, const double* __restrict__ target,
                         double2* __restrict__ g, double* __restrict__ partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < G.n_nodes;
       i += (long long)gridDim.x * 256) {
    const long long nn0 = G.nn[0], nn1 = G.nn[1];
    const int ix = (int)(i % nn0);
    const long long r = i / nn0;
    const int iy = G.dim == 2 ? (int)r : (int)(r % nn1);
    const int iz = G.dim == 2 ? 0 : (int)(r / nn1);
    // lumped mass: integral of psi_i = prod_k h_k (halved on boundary planes)
    double m = G.h[0] * ((ix == 0 || ix == G.n[0]) ? 0.5 : 1.0);
    m *= G.h[1] * ((iy == 0 || iy == G.n[1]) ? 0.5 : 1.0);
    if (G.dim == 3) m *= G.h[2] * ((iz == 0 || iz == G.n[2]) ? 0.5 : 1.0);
    const double d = U[i].x - target[i];
    if (g) g[i] = make_double2(m * d, 0.0);
    acc = fma(0.5 * m * d, d, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// Explicit part of a theta step, second stage: E holds the spatial operator
// at U^n; scale it by (1 - theta) and take the lagged half of the latent rate,
// (1 - theta)/(2 dt) (M (phi^n - phi^(n-1)))_i, off the u rows.  M is the
// consistent Q1 mass matrix, applied as the tensor product of the assembled
// 1-D rows h/6 [1 4 1] (h/6 [2 1] and h/6 [1 2] at the two ends).
__global__ void k_theta_hist(Geo G, const double2* __restrict__ Un,
                             const double2* __restrict__ Unm1, double2* __restrict__ E) {
  const double c = 1.0 - G.theta;
  double scale = (G.h[0] / 6.0) * (G.h[1] / 6.0);
  if (G.dim == 3) scale *= G.h[2] / 6.0;
  const double cu = c * 0.5 * G.idt * scale;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < G.n_nodes;
       i += (long long)gridDim.x * blockDim.x) {
    const long long nn0 = G.nn[0], nn1 = G.nn[1];
    const int ix = (int)(i % nn0);
    const long long r = i / nn0;
    const int iy = G.dim == 2 ? (int)r : (int)(r % nn1);
    const int iz = G.dim == 2 ? 0 : (int)(r / nn1);
    const int zlo = G.dim == 3 ? -1 : 0, zhi = G.dim == 3 ? 1 : 0;
    double acc = 0.0;
    for (int dz = zlo; dz <= zhi; ++dz) {
      const int jz = iz + dz;
      if (jz < 0 || jz >= G.nn[2]) continue;
      const double wz = G.dim == 2 ? 1.0 : (dz != 0 ? 1.0 : ((iz == 0 || iz == G.n[2]) ? 2.0 : 4.0));
      for (int dy = -1; dy <= 1; ++dy) {
        const int jy = iy + dy;
        if (jy < 0 || jy >= G.nn[1]) continue;
        const double wy = dy != 0 ? 1.0 : ((iy == 0 || iy == G.n[1]) ? 2.0 : 4.0);
        for (int dx = -1; dx <= 1; ++dx) {
          const int jx = ix + dx;
          if (jx < 0 || jx >= G.nn[0]) continue;
          const double wx = dx != 0 ? 1.0 : ((ix == 0 || ix == G.n[0]) ? 2.0 : 4.0);
          const long long j = jx + nn0 * (jy + nn1 * (long long)jz);
          acc = fma(wx * wy * wz, Un[j].x - Unm1[j].x, acc);
        }
      }
    }
    const double2 e = E[i];
    E[i] = make_double2(c * e.x, fma(-cu, acc, c * e.y));
  }
}

}  // namespace

int check_vec(const void* p, const char* name) {
  if (!p) {
    set_error(std::string("null device pointer: ") + name);
    return PF_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(p) % 16 != 0) {
    set_error(std::string("device array not 16-byte aligned: ") + name);
    return PF_ERR_INVALID_ARG;
  }
  return PF_OK;
}

int check_params(const pf_params* p) {
  if (!p) {
    set_error("params is NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (p->dim != 2 && p->dim != 3) {
    set_error("dim must be 2 or 3");
    return PF_ERR_INVALID_ARG;
  }
  long long nodes = 1;
  for (int k = 0; k < p->dim; ++k) {
    if (p->n[k] < 1 || p->n[k] > (1 << 20) || !(p->half_width[k] > 0.0)) {
      set_error("each n[k] must be in [1, 2^20] and half_width[k] > 0");
      return PF_ERR_INVALID_ARG;
    }
    nodes *= (p->n[k] + 1);
  }
  if (nodes > (1LL << 31)) {
    set_error("mesh too large (more than 2^31 nodes)");
    return PF_ERR_INVALID_ARG;
  }
  if (!(p->dt > 0.0) || !(p->D > 0.0) || !(p->delta2 > 0.0) || !std::isfinite(p->eps4) ||
      !std::isfinite(p->lambda)) {
    set_error("dt, D, delta2 must be > 0 and eps4, lambda finite");
    return PF_ERR_INVALID_ARG;
  }
  if (!(p->theta > 0.0 && p->theta <= 1.0)) {
    set_error("theta must be in (0, 1]");
    return PF_ERR_INVALID_ARG;
  }
  const int ord = p->order == 0 ? 1 : p->order;
  if (ord != 1 && ord != 2) {
    set_error("order must be 1 or 2");
    return PF_ERR_INVALID_ARG;
  }
  if (ord == 2 && p->dim != 2) {
    set_error("order-2 elements are 2-D only");
    return PF_ERR_INVALID_ARG;
  }
  return PF_OK;
}

namespace {

int check_opts(const pf_problem* pb, const pf_solver_opts* o) {
  if (!o) {
    set_error("opts is NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (o->gmres_m < 1 || o->gmres_m > pb->gmres_m_max || o->gmres_maxit < 1 || o->max_newton < 0 ||
      o->max_backtracks < 0 || (o->jv_mode != PF_JV_FD && o->jv_mode != PF_JV_ANALYTIC) ||
      o->pc < PF_PC_NONE || o->pc > PF_PC_GMG ||
      (o->pc_precision != PF_FP64 && o->pc_precision != PF_FP32) || !(o->tau_r >= 0.0) ||
      !(o->tau_a >= 0.0)) {
    set_error("invalid solver options (gmres_m must be in [1, gmres_m_max])");
    return PF_ERR_INVALID_ARG;
  }
  return PF_OK;
}


// |x|: the reduction also writes its result into mapped host memory, so the
// host reads it after the stream syncs without a copy.
int norm2(pf_problem* pb, const double* x, double* out, hipStream_t s) {
  PF_TRY(blas_multidot(pb, x, pb->n_dof, 1, x, pb->n_dof, pb->red_out + kSlotNorm, s,
                       pb->host_pinned_dev + kSlotNorm));
  PF_HIP_CHECK(hipStreamSynchronize(s));
  *out = std::sqrt(pb->host_pinned[kSlotNorm]);
  return PF_OK;
}

// Linear operator of a Krylov solve.
struct Op {
  pf_problem* pb;
  const double* U;
  const double* Uprev;
  const double* F0;  // F(U) for the FD product
  int kind;          // 0 = J (FD), 1 = J (analytic), 2 = J^T
  const double* unorm2 = nullptr;  // |U|^2 on the device (FD), computed by prepare()
  // have_unorm2: the slot already holds |U|^2 (formed with the trial state)
  int prepare(hipStream_t s, bool have_unorm2 = false) {
    if (kind != 0) return PF_OK;
    double* d = pb->red_out + kSlotUnorm;
    if (!have_unorm2) PF_TRY(blas_multidot(pb, U, pb->n_dof, 1, U, pb->n_dof, d, s));
    unorm2 = d;
    return PF_OK;
  }
  int apply(const double* z, double* w, hipStream_t s) const {
    if (kind == 0) {
      PF_TRY(blas_fd_eps_cached(pb, unorm2, z, pb->n_dof, pb->eps_dev, s));
      return launch_residual_family(pb, MODE_FD, U, Uprev, z, F0, pb->eps_dev, w, nullptr, nullptr, s);
    }
    if (kind == 1)
      return launch_residual_family(pb, MODE_JVP, U, Uprev, z, nullptr, nullptr, w, nullptr, nullptr, s);
    return launch_residual_family(pb, MODE_VJPU, U, Uprev, z, nullptr, nullptr, w, nullptr,
                                  pb->vjp_partials, s);
  }
};

// Right-preconditioned FGMRES(m) from x = 0 for A x = b, |b - A x| <= rtol |b|.
//
// Arnoldi with classical Gram-Schmidt and a delayed second projection: step j
// applies the preconditioner and the operator to V_j as left by step j-1,
// projected once and normalised by its Pythagorean norm estimate.  One sweep
// forms the products of V_j and of the new vector w with the basis; V_j is then
// finished (second projection, exact norm) and w projected once against the
// finished V_0..V_j in a second sweep.  The finishing step of V_{j+1} at step
// j+1 completes column j of the Hessenberg matrix:
//   A z_j = sum_{k<=j} h_k V_k + eta u,  u = sum_{k<=j} s_k V_k + rho V_{j+1}
// so H[k][j] = h_k + eta s_k and H[j+1][j] = eta rho.  The convergence test
// uses the column with s = 0, rho = 1; when it passes (or the cycle ends) the
// products of u are formed at once and the column completed before the exact
// residual is taken.  Two sweeps over the basis per iteration instead of three.
// The right-hand side is bsign b (bsign = 1 or -1); bnorm is |b| when the
// caller has it (the same norm2 value), else negative.  x is written by the
// first solution update (x = Z y, no zero fill read back) or zeroed on a return
// before it.
int fgmres_cycles(pf_problem* pb, const Op& op, const double* b, double bsign, double bnorm,
                  double* x, bool* xset, double rtol, const pf_solver_opts& o, int* its_out,
                  hipStream_t s) {
  const long long n = pb->n_dof;
  const int m = o.gmres_m;
  double* V = pb->V;
  double* Z = pb->Z;
  double* r = pb->tmp_vec[3];
  double* ydev = pb->red_out + kSlotY;
  double* dots_dev = pb->red_out + kSlotDots;
  double* hp = pb->host_pinned;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  std::vector<double> hcol(m + 1), sv(m + 1), col(m + 1);
  double beta = bnorm;
  if (!(bnorm >= 0.0)) PF_TRY(norm2(pb, b, &beta, s));
  *its_out = 0;
  if (!std::isfinite(beta)) {
    set_error("non-finite right-hand side in FGMRES");
    return PF_ERR_NONFINITE;
  }
  if (beta == 0.0) return PF_OK;
  const double target = rtol * beta;
  const double* rhs = b;
  double rsign = bsign;  // the sign of rhs in the right-hand side (1 after a restart)
  int total = 0;
  bool converged = false;
  double resid = beta;
  // Givens rotations 0..j-1 applied to column j of H, then rotation j formed
  // and applied to g; returns |g[j+1]|
  auto rotate = [&](int j) {
    for (int i = 0; i < j; ++i) {
      const double a = H[i * m + j], c = H[(i + 1) * m + j];
      H[i * m + j] = cs[i] * a + sn[i] * c;
      H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
    }
    const double a = H[j * m + j], c = H[(j + 1) * m + j];
    const double rr = std::hypot(a, c);
    cs[j] = rr > 0.0 ? a / rr : 1.0;
    sn[j] = rr > 0.0 ? c / rr : 0.0;
    H[j * m + j] = rr;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    return std::fabs(g[j + 1]);
  };
  // products of V_{j+1} with V_0..V_{j+1}: its second-projection
  // coefficients sv[0..j] and its norm after that projection
  auto finish_products = [&](int j, double* rho_out) -> int {
    PF_TRY(blas_multidot(pb, V, n, j + 2, V + (long long)(j + 1) * n, n, dots_dev, s,
                         pb->host_pinned_dev + kSlotDots));
    PF_HIP_CHECK(hipStreamSynchronize(s));
    double ssq = 0.0;
    for (int k = 0; k <= j; ++k) {
      sv[k] = hp[kSlotDots + k];
      ssq += sv[k] * sv[k];
    }
    const double r2 = hp[kSlotDots + j + 1] - ssq;
    *rho_out = r2 > 0.0 ? std::sqrt(r2) : 0.0;
    return PF_OK;
  };
  while (true) {
    // V_0 = r / |r|, final
    PF_TRY(blas_axpby(rsign / resid, rhs, 0.0, rhs, V, n, s));
    std::fill(g.begin(), g.end(), 0.0);
    std::fill(H.begin(), H.end(), 0.0);
    g[0] = resid;
    int jend = 0;       // completed columns
    bool pending = false;  // column jend computed, V_{jend+1} not yet finished
    double eta = 0.0;      // norm estimate that scaled the pending V_{jend+1}
    for (int j = 0; j < m; ++j) {
      double* vj = V + (long long)j * n;
      double* zj = Z + (long long)j * n;
      double* w = V + (long long)(j + 1) * n;
      PF_TRY(pc_apply(pb, vj, zj, s));
      PF_TRY(op.apply(zj, w, s));
      PF_TRY(blas_dcgs_dots(pb, V, n, j, n, dots_dev, s, pb->host_pinned_dev + kSlotDots));
      PF_HIP_CHECK(hipStreamSynchronize(s));
      const double* dt = hp + kSlotDots;    // V_k . V_j (k < j), |V_j|^2
      const double* dw = hp + kSlotDots + j + 1;  // V_k . w (k < j), V_j . w, |w|^2
      // finish V_j: second projection coefficients dt[0..j-1], norm rho
      double rho = 1.0;
      if (j > 0) {
        double ssq = 0.0;
        for (int k = 0; k < j; ++k) ssq += dt[k] * dt[k];
        const double r2 = dt[j] - ssq;
        rho = r2 > 0.0 ? std::sqrt(r2) : 0.0;
      }
      if (pending) {
        for (int k = 0; k < j; ++k) H[k * m + j - 1] = hcol[k] + eta * dt[k];
        H[j * m + j - 1] = eta * rho;
        resid = rotate(j - 1);
        jend = j;
        pending = false;
        if (!std::isfinite(resid)) {
          set_error("non-finite Arnoldi coefficient in FGMRES");
          return PF_ERR_NONFINITE;
        }
        if (resid <= target || rho == 0.0) {
          converged = resid <= target;
          break;
        }
      }
      // products of w with the finished V_0..V_j
      double dot_wv = dw[j];
      if (j > 0) {
        double c = 0.0;
        for (int k = 0; k < j; ++k) c += dt[k] * dw[k];
        dot_wv = (dw[j] - c) / rho;
      }
      double hsq = 0.0;
      for (int k = 0; k < j; ++k) {
        hcol[k] = dw[k];
        hsq += dw[k] * dw[k];
      }
      hcol[j] = dot_wv;
      hsq += dot_wv * dot_wv;
      const double wsq = dw[j + 1];
      if (!std::isfinite(wsq) || !std::isfinite(hsq)) {
        set_error("non-finite Arnoldi coefficient in FGMRES");
        return PF_ERR_NONFINITE;
      }
      // normalisation of the once-projected w: the Pythagorean estimate while
      // it keeps at least six digits, else the norm itself
      const double u2 = wsq - hsq;
      const bool explicit_norm = !(u2 > 1e-12 * wsq);
      eta = explicit_norm ? 1.0 : std::sqrt(u2);
      PF_TRY(blas_dcgs_update(V, n, j, dots_dev, hcol[j], 1.0 / rho, 1.0 / eta, n, s));
      if (explicit_norm) {
        PF_TRY(norm2(pb, w, &eta, s));
        if (eta > 0.0) PF_TRY(blas_axpby(1.0 / eta, w, 0.0, w, w, n, s));
      }
      ++total;
      pending = true;
      // convergence test on the column with the second projection of
      // V_{j+1} taken as zero
      for (int k = 0; k <= j; ++k) col[k] = hcol[k];
      col[j + 1] = eta;
      for (int i = 0; i < j; ++i) {
        const double a = col[i], c = col[i + 1];
        col[i] = cs[i] * a + sn[i] * c;
        col[i + 1] = -sn[i] * a + cs[i] * c;
      }
      const double rr = std::hypot(col[j], col[j + 1]);
      const double est = rr > 0.0 ? std::fabs(g[j] * col[j + 1] / rr) : std::fabs(g[j]);
      const bool last = j + 1 == m || total >= o.gmres_maxit || eta == 0.0;
      if (est <= target || last) {
        double rho1 = 0.0;
        if (eta > 0.0) PF_TRY(finish_products(j, &rho1));
        else std::fill(sv.begin(), sv.begin() + j + 1, 0.0);
        for (int k = 0; k <= j; ++k) H[k * m + j] = hcol[k] + eta * sv[k];
        H[(j + 1) * m + j] = eta * rho1;
        resid = rotate(j);
        jend = j + 1;
        pending = false;
        if (!std::isfinite(resid)) {
          set_error("non-finite Arnoldi coefficient in FGMRES");
          return PF_ERR_NONFINITE;
        }
        converged = resid <= target;
        if (converged || last || rho1 == 0.0) break;
      }
    }
    // y = H^-1 g (upper triangular), x += Z y
    for (int i = jend - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < jend; ++k) t -= H[i * m + k] * y[k];
      y[i] = H[i * m + i] != 0.0 ? t / H[i * m + i] : 0.0;
    }
    std::memcpy(pb->host_pinned + kSlotHostY, y.data(), jend * sizeof(double));
    PF_HIP_CHECK(hipMemcpyAsync(ydev, pb->host_pinned + kSlotHostY, jend * sizeof(double),
                                hipMemcpyHostToDevice, s));
    PF_TRY(blas_combine(pb, Z, n, jend, ydev, x, n, s, !*xset));
    *xset = true;
    PF_HIP_CHECK(hipStreamSynchronize(s));
    if (converged || total >= o.gmres_maxit) break;
    // restart: r = b - A x
    PF_TRY(op.apply(x, r, s));
    PF_TRY(blas_axpby(bsign, b, -1.0, r, r, n, s));
    PF_TRY(norm2(pb, r, &resid, s));
    if (resid <= target) {
      converged = true;
      break;
    }
    rhs = r;
    rsign = 1.0;
  }
  *its_out = total;
  if (!converged) {
    set_error("FGMRES did not reach its tolerance");
    return PF_ERR_LINEAR;
  }
  return PF_OK;
}

int fgmres(pf_problem* pb, const Op& op, const double* b, double bsign, double bnorm, double* x,
           double rtol, const pf_solver_opts& o, int* its_out, hipStream_t s) {
  bool xset = false;
  const int rc = fgmres_cycles(pb, op, b, bsign, bnorm, x, &xset, rtol, o, its_out, s);
  if (!xset) PF_HIP_CHECK(hipMemsetAsync(x, 0, pb->n_dof * sizeof(double), s));
  return rc;
}

void stats_reset(pf_solver_stats* st) {
  if (st) std::memset(st, 0, sizeof(*st));
}

int ensure_load_vec(pf_problem* pb) {
  if (pb->load_vec) return PF_OK;
  if (hipMalloc(&pb->load_vec, pb->n_dof * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    pb->load_vec = nullptr;
    set_error("out of device memory for the theta-step workspace");
    return PF_ERR_OOM;
  }
  return PF_OK;
}

// Explicit part of a theta step (see k_theta_hist): the theta = 1 residual at
// (U^n; U^n) -- whose time terms vanish -- is the spatial operator at U^n.
int theta_explicit_impl(pf_problem* pb, const double* Un, const double* Unm1, double* E,
                        hipStream_t s) {
  const long long n = pb->n_dof;
  if (pb->params.theta == 1.0) {
    PF_HIP_CHECK(hipMemsetAsync(E, 0, n * sizeof(double), s));
    return PF_OK;
  }
  const Geo saved = pb->geo;
  Geo g1 = saved;
  g1.theta = 1.0;
  g1.idtm = g1.idt;
  g1.Dth = g1.D;
  g1.hth = 0.5;
  pb->geo = g1;  // kernel arguments are captured at launch
  const int rc = launch_residual_family(pb, MODE_RES, Un, Un, nullptr, nullptr, nullptr, E,
                                        nullptr, nullptr, s);
  pb->geo = saved;
  PF_TRY(rc);
  const long long nb = std::min<long long>((pb->geo.n_nodes + 255) / 256, 65536);
  hipLaunchKernelGGL(k_theta_hist, dim3((unsigned)nb), dim3(256), 0, s, pb->geo,
                     reinterpret_cast<const double2*>(Un), reinterpret_cast<const double2*>(Unm1),
                     reinterpret_cast<double2*>(E));
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

// Newton-Krylov for F(U; Uprev) + load = 0 (load may be NULL).  The FD
// products use F(U; Uprev) itself as their base value: the load cancels.
int newton_impl(pf_problem* pb, const double* Uprev, const double* load, double* U,
                const pf_solver_opts& o, pf_solver_stats* st, hipStream_t s) {
  const long long n = pb->n_dof;
  double* F = pb->tmp_vec[0];
  double* dU = pb->tmp_vec[1];
  // the accepted state alternates between U and tmp_vec[2], the trial state
  // taking the other one: no copy per Newton step, one at the end if needed
  double* Uc = U;
  double* Ut = pb->tmp_vec[2];
  // tmp_vec[3] is FGMRES's restart vector
  double* Ft = pb->tmp_vec[4];
  double* B = pb->tmp_vec[5];
  double* coef = pc_coef_buffer(pb);
  // |X + load|, staged through B (free outside the linear solve)
  auto norm_loaded = [&](const double* X, double* out) -> int {
    if (!load) return norm2(pb, X, out, s);
    PF_TRY(blas_axpby(1.0, X, 1.0, load, B, n, s));
    return norm2(pb, B, out, s);
  };
  auto sync_u = [&]() -> int {
    if (Uc != U) PF_HIP_CHECK(hipMemcpyAsync(U, Uc, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return PF_OK;
  };
  PF_TRY(launch_residual_family(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, F, nullptr,
                                nullptr, s, coef));
  double f;
  PF_TRY(norm_loaded(F, &f));
  if (!std::isfinite(f)) {
    set_error("non-finite initial residual norm");
    if (st) st->status = PF_ERR_NONFINITE;
    return PF_ERR_NONFINITE;
  }
  const double f0 = f;
  if (st) {
    st->f0 = f0;
    st->fnorm[0] = f0;
  }
  double eta = o.eta0;
  int l = 0;
  while (!(f < o.tau_r * f0 + o.tau_a)) {
    if (l >= o.max_newton) {
      set_error("Newton did not converge within max_newton iterations");
      if (st) {
        st->status = PF_ERR_NOT_CONVERGED;
        st->f_final = f;
      }
      PF_TRY(sync_u());
      return PF_ERR_NOT_CONVERGED;
    }
    // the cell coefficients of the preconditioner came with the residual at U
    PF_TRY(pc_setup_prepared(pb, o.pc, o.pc_precision, s));
    // right-hand side -(F + load), whose norm is f: -F itself without a load
    if (load) PF_TRY(blas_axpby(-1.0, F, -1.0, load, B, n, s));
    Op op{pb, Uc, Uprev, F, o.jv_mode == PF_JV_FD ? 0 : 1};
    PF_TRY(op.prepare(s, l > 0));
    int its = 0;
    int rc = load ? fgmres(pb, op, B, 1.0, f, dU, eta, o, &its, s)
                  : fgmres(pb, op, F, -1.0, f, dU, eta, o, &its, s);
    if (st) {
      st->gmres_its_total += its;
      if (l < PF_MAX_LOG) st->gmres_its[l] = its;
    }
    if (rc != PF_OK && rc != PF_ERR_LINEAR) {
      if (st) st->status = rc;
      PF_TRY(sync_u());
      return rc;
    }
    // backtracking: Lambda = 1, 1/2, ... until |F(U + Lambda dU)| <= |F(U)|
    double lam = 1.0, ft = 0.0;
    bool ok = false;
    for (int bt = 0; bt <= o.max_backtracks; ++bt) {
      // the trial state and its |.|^2, which the next step's FD products take
      PF_TRY(blas_axpby_norm(pb, 1.0, Uc, lam, dU, Ut, n, pb->red_out + kSlotUnorm, s));
      PF_TRY(launch_residual_family(pb, MODE_RES, Ut, Uprev, nullptr, nullptr, nullptr, Ft, nullptr,
                                    nullptr, s, coef));
      PF_TRY(norm_loaded(Ft, &ft));
      if (std::isfinite(ft) && ft <= f) {
        ok = true;
        break;
      }
      lam *= 0.5;
      if (st) st->backtracks++;
    }
    if (!ok) {
      set_error("line search failed to reduce |F|");
      if (st) {
        st->status = std::isfinite(ft) ? PF_ERR_LINESEARCH : PF_ERR_NONFINITE;
        st->f_final = f;
      }
      PF_TRY(sync_u());
      return std::isfinite(ft) ? PF_ERR_LINESEARCH : PF_ERR_NONFINITE;
    }
    std::swap(Uc, Ut);  // the accepted trial state
    std::swap(F, Ft);   // and its residual (both are work vectors)
    // forcing term for the next linear solve
    const double ratio = ft / f;
    double en = o.gamma * std::pow(ratio, o.omega);
    const double safeg = o.gamma * std::pow(eta, o.omega);
    en = std::max(en, safeg);
    en = std::max(en, o.eta_min);
    eta = std::min(o.eta_max, en);
    f = ft;
    ++l;
    if (st && l <= PF_MAX_LOG) st->fnorm[l] = f;
  }
  PF_TRY(sync_u());
  if (st) {
    st->newton_its = l;
    st->f_final = f;
    st->status = PF_OK;
  }
  return PF_OK;
}

// One alloy step: the explicit part at t_prev, the history rate, then
// Newton-Krylov on F + E = 0 with the implicit part at t_prev + dt.
int alloy_step_impl(pf_problem* pb, const double* Uprev2, const double* Uprev, double t_prev,
                    double* U, const pf_solver_opts& o, pf_solver_stats* st, hipStream_t s) {
  PF_TRY(ensure_load_vec(pb));
  PF_TRY(alloy_explicit(pb, Uprev, t_prev, pb->load_vec, s));
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  pb->t_new = t_prev + pb->params.dt;
  return newton_impl(pb, Uprev, pb->params.theta == 1.0 ? nullptr : pb->load_vec, U, o, st, s);
}

// One free-growth step: explicit part, history rate, then Newton-Krylov.
int fg_step_impl(pf_problem* pb, const double* Uprev2, const double* Uprev, double* U,
                 const pf_solver_opts& o, pf_solver_stats* st, hipStream_t s) {
  PF_TRY(ensure_load_vec(pb));
  PF_TRY(fg_explicit(pb, Uprev, pb->load_vec, s));
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  return newton_impl(pb, Uprev, pb->params.theta == 1.0 ? nullptr : pb->load_vec, U, o, st, s);
}

// One thermal step (backward Euler, or theta < 1 with the explicit part).
int thermal_step_impl(pf_problem* pb, const double* Uprev2, const double* Uprev, double* U,
                      const pf_solver_opts& o, pf_solver_stats* st, hipStream_t s) {
  if (pb->params.theta == 1.0) return newton_impl(pb, Uprev, nullptr, U, o, st, s);
  PF_TRY(ensure_load_vec(pb));
  PF_TRY(theta_explicit_impl(pb, Uprev, Uprev2, pb->load_vec, s));
  return newton_impl(pb, Uprev, pb->load_vec, U, o, st, s);
}

// steps time steps over the checkpoint array states: step k goes from
// states[k] (and states[k-1]; U^(-1) = U^0) to states[k+1], starting Newton
// from a copy of states[k].  step(prev2, prev, k, next, stats) takes one step.
template <class Step>
int evolve_loop(pf_problem* pb, double* states, int steps, pf_solver_stats* stats, hipStream_t s,
                Step step) {
  const long long n = pb->n_dof;
  pf_solver_stats acc;
  stats_reset(&acc);
  double t0;
  PF_TRY(clock_start(s, &t0));
  for (int k = 0; k < steps; ++k) {
    double* prev = states + (long long)k * n;
    double* next = prev + n;
    const double* prev2 = k > 0 ? prev - n : prev;
    PF_HIP_CHECK(hipMemcpyAsync(next, prev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    pf_solver_stats st;
    stats_reset(&st);
    const int rc = step(prev2, prev, k, next, &st);
    acc.newton_its += st.newton_its;
    acc.gmres_its_total += st.gmres_its_total;
    acc.backtracks += st.backtracks;
    if (k < PF_MAX_LOG) acc.gmres_its[k] = st.gmres_its_total;
    acc.f0 = st.f0;
    acc.f_final = st.f_final;
    if (rc != PF_OK) {
      acc.status = rc;
      if (stats) *stats = acc;
      return rc;
    }
  }
  acc.t_total_ms = now_ms() - t0;
  if (stats) *stats = acc;
  return PF_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

// HIP keeps one sticky "last error" per thread that any runtime call (ours or
// another library's) may set.  Entry points clear it first so that the checks
// after their own launches report only their own failures.
void clear_stale_error() { (void)hipGetLastError(); }

Geo make_geo(const pf_params& p) {
  Geo G{};
  G.dim = p.dim;
  G.n_nodes = 1;
  G.n_elems = 1;
  G.jac = 1.0;
  // order 2: the grid of element nodes, viewed as 2 n cells of width h/2
  const int sub = p.order == 2 ? 2 : 1;
  for (int k = 0; k < 3; ++k) {
    if (k < p.dim) {
      G.n[k] = sub * p.n[k];
      G.nn[k] = sub * p.n[k] + 1;
      G.h[k] = 2.0 * p.half_width[k] / (sub * p.n[k]);
      G.ih[k] = 1.0 / G.h[k];
      G.jac *= 0.5 * G.h[k];
    } else {
      G.n[k] = 1;
      G.nn[k] = 1;
      G.h[k] = 1.0;
      G.ih[k] = 1.0;
    }
    G.n_nodes *= G.nn[k];
    G.n_elems *= (k < p.dim) ? G.n[k] : 1;
  }
  G.dt = p.dt;
  G.idt = 1.0 / p.dt;
  G.eps4 = p.eps4;
  G.lam = p.lambda;
  G.D = p.D;
  G.delta2 = p.delta2;
  G.a0 = 1.0 - 3.0 * p.eps4;
  G.e4x4 = 4.0 * p.eps4;
  G.e16 = 16.0 * p.eps4;
  G.theta = p.theta;
  G.idtm = 1.0 / (p.theta * p.dt);
  G.Dth = p.theta * p.D;
  G.hth = 0.5 * p.theta;
  return G;
}

// The thermal entry points and the pf_alloy_* entry points each need a
// handle of their own model.
int require_model(const pf_problem* pb, int model) {
  static const char* names[3] = {"thermal (pf_residual, pf_newton_step, ...)",
                                 "alloy (pf_set_alloy, pf_alloy_*)",
                                 "free-growth (pf_set_freegrowth, pf_fg_*)"};
  if (pb->model == model) {
    if (model != 2 && pb->params.order == 2) {
      set_error("order-2 elements are available in the free-growth model only");
      return PF_ERR_INVALID_ARG;
    }
    return PF_OK;
  }
  set_error(std::string("this call needs a handle in the ") + names[model] + " model; the handle is in the " +
            names[pb->model] + " model");
  return PF_ERR_INVALID_ARG;
}

}  // namespace pf

using namespace pf;

extern "C" {

void pf_default_opts(pf_solver_opts* o) {
  if (!o) return;
  o->tau_r = 1e-10;
  o->tau_a = 0.0;
  o->max_newton = 30;
  o->max_backtracks = 8;
  o->gmres_m = 30;
  o->gmres_maxit = 300;
  o->eta0 = 0.1;
  o->eta_min = 1e-6;
  o->eta_max = 0.01;
  o->gamma = 0.9;
  o->omega = 1.5;
  o->jv_mode = PF_JV_FD;
  o->pc = PF_PC_GMG;
  o->pc_precision = PF_FP64;
}

const char* pf_last_error(void) { return g_last_error.c_str(); }

int pf_create(const pf_params* params, int gmres_m_max, pf_problem** out) {
  g_last_error.clear();
  if (!out) {
    set_error("out is NULL");
    return PF_ERR_INVALID_ARG;
  }
  *out = nullptr;
  PF_TRY(check_params(params));
  if (gmres_m_max < 1 || gmres_m_max > kMaxGmresM) {
    set_error("gmres_m_max must be in [1, 60]");
    return PF_ERR_INVALID_ARG;
  }
  pf_problem* pb = new pf_problem();
  std::memset(pb, 0, sizeof(*pb));
  pb->params = *params;
  if (pb->params.order == 0) pb->params.order = 1;
  pb->geo = make_geo(pb->params);
  pb->n_dof = 2 * pb->geo.n_nodes;
  pb->gmres_m_max = gmres_m_max;
  PF_HIP_CHECK(hipGetDevice(&pb->device));
  auto fail = [&](int rc) {
    pf_destroy(pb);
    return rc;
  };
  const long long n = pb->n_dof;
  long long rb = (n / 2 + 255) / 256;
  pb->n_red_blocks = (int)std::min<long long>(std::max<long long>(rb, 1), 1024);
  pb->n_elem_blocks = elem_blocks(pb);
  const int NA = 1 << pb->geo.dim;
  pb->elem_buf_len = pb->geo.dim == 2 ? (long long)4 * NA * pb->geo.n_elems : 1;
  pb->side_len = pb->geo.dim == 3 ? fused3_side_len(pb->geo) : 1;
  if (hipMalloc(&pb->red_partials, (size_t)kRedRows * pb->n_red_blocks * sizeof(double)) !=
          hipSuccess ||
      hipMalloc(&pb->red_out, kRedSlots * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&pb->host_pinned, kRedSlots * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&pb->host_pinned_dev), pb->host_pinned, 0) !=
          hipSuccess ||
      hipMalloc(&pb->elem_buf, (size_t)pb->elem_buf_len * sizeof(double)) != hipSuccess ||
      hipMalloc(&pb->side_buf, (size_t)pb->side_len * sizeof(double)) != hipSuccess ||
      hipMalloc(&pb->vjp_partials, (size_t)2 * pb->n_elem_blocks * sizeof(double)) != hipSuccess ||
      hipMalloc(&pb->eps_dev, 8 * sizeof(double)) != hipSuccess) {
    set_error("device allocation failed (workspace)");
    return fail(PF_ERR_OOM);
  }
  for (int i = 0; i < kNumTmp; ++i) {
    if (hipMalloc(&pb->tmp_vec[i], (size_t)n * sizeof(double)) != hipSuccess) {
      set_error("device allocation failed (work vectors)");
      return fail(PF_ERR_OOM);
    }
  }
  if (hipMalloc(&pb->V, (size_t)(gmres_m_max + 1) * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&pb->Z, (size_t)gmres_m_max * n * sizeof(double)) != hipSuccess) {
    set_error("device allocation failed (Krylov basis)");
    return fail(PF_ERR_OOM);
  }
  int rc = pc_alloc(pb);
  if (rc != PF_OK) {
    set_error("device allocation failed (preconditioner)");
    return fail(rc);
  }
  *out = pb;
  return PF_OK;
}

int pf_destroy(pf_problem* pb) {
  if (!pb) return PF_OK;
  int rc = PF_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == PF_OK) {
      set_error(std::string("pf_destroy: ") + what + ": " + hipGetErrorString(e));
      rc = PF_ERR_HIP;
    }
  };
  chk(hipDeviceSynchronize(), "hipDeviceSynchronize");
  chk(pc_free(pb), "preconditioner buffers");
  double* bufs[] = {pb->red_partials, pb->red_out, pb->elem_buf, pb->vjp_partials, pb->eps_dev,
                    pb->V, pb->Z, pb->side_buf, pb->load_vec, pb->hist};
  const char* names[] = {"red_partials", "red_out", "elem_buf", "vjp_partials", "eps_dev", "V", "Z",
                         "side_buf", "load_vec", "hist"};
  for (int i = 0; i < 10; ++i)
    if (bufs[i]) chk(hipFree(bufs[i]), names[i]);
  for (int i = 0; i < kNumTmp; ++i)
    if (pb->tmp_vec[i]) chk(hipFree(pb->tmp_vec[i]), "tmp_vec");
  if (pb->host_pinned) chk(hipHostFree(pb->host_pinned), "host_pinned");
  delete pb;
  (void)hipGetLastError();  // leave no sticky error behind for other libraries
  return rc;
}

int pf_set_params(pf_problem* pb, const pf_params* p) {
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_params(p));
  if (p->dim != pb->params.dim) {
    set_error("mesh of pf_set_params differs from the handle");
    return PF_ERR_INVALID_ARG;
  }
  if ((p->order == 2) != (pb->params.order == 2)) {
    set_error("element order of pf_set_params differs from the handle");
    return PF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < p->dim; ++k) {
    if (p->n[k] != pb->params.n[k] || p->half_width[k] != pb->params.half_width[k]) {
      set_error("mesh of pf_set_params differs from the handle");
      return PF_ERR_INVALID_ARG;
    }
  }
  pb->params = *p;
  if (pb->params.order == 0) pb->params.order = 1;
  pb->geo = make_geo(pb->params);
  return PF_OK;
}

long long pf_num_nodes(const pf_problem* pb) { return pb ? pb->geo.n_nodes : -1; }

int pf_residual(pf_problem* pb, const double* U, const double* Uprev, const double* rhs, double* F,
                void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(F, "F"));
  if (rhs) PF_TRY(check_vec(rhs, "rhs"));
  hipStream_t s = S(stream);
  PF_TRY(launch_residual_family(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, F, nullptr,
                                nullptr, s));
  // F - b: fma(1, F, -b) rounds once, so the result is the exact difference rounded
  if (rhs) PF_TRY(blas_axpby(1.0, F, -1.0, rhs, F, pb->n_dof, s));
  return PF_OK;
}

int pf_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* v, const double* F0,
           int mode, double* Jv, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(v, "v"));
  PF_TRY(check_vec(Jv, "Jv"));
  hipStream_t s = S(stream);
  if (mode == PF_JV_ANALYTIC)
    return launch_residual_family(pb, MODE_JVP, U, Uprev, v, nullptr, nullptr, Jv, nullptr, nullptr, s);
  if (mode != PF_JV_FD) {
    set_error("mode must be PF_JV_FD or PF_JV_ANALYTIC");
    return PF_ERR_INVALID_ARG;
  }
  if (!F0) {
    F0 = pb->tmp_vec[0];
    PF_TRY(launch_residual_family(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr,
                                  pb->tmp_vec[0], nullptr, nullptr, s));
  } else {
    PF_TRY(check_vec(F0, "F0"));
  }
  PF_TRY(blas_fd_eps(pb, U, v, pb->n_dof, pb->eps_dev, s));
  return launch_residual_family(pb, MODE_FD, U, Uprev, v, F0, pb->eps_dev, Jv, nullptr, nullptr, s);
}

int pf_vjp(pf_problem* pb, const double* U, const double* Uprev, const double* w, double* gU,
           double* gUprev, double* gparams, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(w, "w"));
  if (gU) PF_TRY(check_vec(gU, "gU"));
  if (gUprev) PF_TRY(check_vec(gUprev, "gUprev"));
  hipStream_t s = S(stream);
  // lean kernels where outputs are left out: gU alone is the transposed
  // operator; without gU only the previous state and the parameters are formed
  if (gU && !gUprev && !gparams)
    return launch_residual_family(pb, MODE_VJPU, U, Uprev, w, nullptr, nullptr, gU, nullptr,
                                  nullptr, s);
  PF_TRY(launch_residual_family(pb, gU ? MODE_VJP : MODE_VJPP, U, Uprev, w, nullptr, nullptr, gU,
                                gUprev, pb->vjp_partials, s));
  if (gparams) PF_TRY(blas_reduce_partials(pb->vjp_partials, pb->n_elem_blocks, 2, gparams, 1.0, s));
  return PF_OK;
}

int pf_precond_setup(pf_problem* pb, const double* U, int kind, int precision, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(U, "U"));
  if (kind < PF_PC_NONE || kind > PF_PC_GMG || (precision != PF_FP64 && precision != PF_FP32)) {
    set_error("invalid preconditioner kind or precision");
    return PF_ERR_INVALID_ARG;
  }
  if (pb->model != 0) {
    // alloy / free growth: the phi-block coefficient (cell mean of cu a^2,
    // resp. a^2) comes out of the residual kernel; the residual is discarded
    hipStream_t s = S(stream);
    PF_TRY(launch_residual_family(pb, MODE_RES, U, U, nullptr, nullptr, nullptr, pb->tmp_vec[0],
                                  nullptr, nullptr, s, pc_coef_buffer(pb)));
    return pc_setup_prepared(pb, kind, precision, s);
  }
  return pc_setup(pb, U, kind, precision, S(stream));
}

int pf_precond_apply(pf_problem* pb, const double* r, double* z, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(r, "r"));
  PF_TRY(check_vec(z, "z"));
  return pc_apply(pb, r, z, S(stream));
}

int pf_linear_solve(pf_problem* pb, const double* U, const double* Uprev, const double* b, double* x,
                    int transpose, double rtol, const pf_solver_opts* opts, pf_solver_stats* stats,
                    void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(b, "b"));
  PF_TRY(check_vec(x, "x"));
  hipStream_t s = S(stream);
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(s, &t0));
  double* F = pb->tmp_vec[0];
  int kind = transpose ? 2 : (opts->jv_mode == PF_JV_FD ? 0 : 1);
  if (kind == 0)
    PF_TRY(launch_residual_family(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, F, nullptr, nullptr, s));
  Op op{pb, U, Uprev, F, kind};
  PF_TRY(op.prepare(s));
  int its = 0;
  int rc = fgmres(pb, op, b, 1.0, -1.0, x, rtol, *opts, &its, s);
  if (stats) {
    stats->gmres_its_total = its;
    stats->gmres_its[0] = its;
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_newton_step(pf_problem* pb, const double* Uprev, double* U, const pf_solver_opts* opts,
                   pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(U, "U"));
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(S(stream), &t0));
  int rc = newton_impl(pb, Uprev, nullptr, U, *opts, stats, S(stream));
  if (stats) {
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_newton_step_theta(pf_problem* pb, const double* Uprev2, const double* Uprev, double* U,
                         const pf_solver_opts* opts, pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(U, "U"));
  if (pb->params.theta != 1.0) PF_TRY(check_vec(Uprev2, "Uprev2"));
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(S(stream), &t0));
  const int rc = thermal_step_impl(pb, Uprev2, Uprev, U, *opts, stats, S(stream));
  if (stats) {
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_theta_explicit(pf_problem* pb, const double* Uprev, const double* Uprev2, double* E,
                      void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(E, "E"));
  return theta_explicit_impl(pb, Uprev, Uprev2, E, S(stream));
}

int pf_evolve(pf_problem* pb, double* states, int steps, const pf_solver_opts* opts,
              pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(states, "states"));
  if (steps < 0) {
    set_error("steps must be >= 0");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  return evolve_loop(pb, states, steps, stats, s,
                     [&](const double* prev2, const double* prev, int, double* next,
                         pf_solver_stats* st) {
                       return thermal_step_impl(pb, prev2, prev, next, *opts, st, s);
                     });
}

int pf_adjoint_step(pf_problem* pb, const double* U, const double* Uprev, const double* mu,
                    double* lam, double* mu_prev, double* gparams, const pf_solver_opts* opts,
                    pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  if (pb->params.theta != 1.0) {
    set_error("pf_adjoint_step covers backward Euler (theta = 1) only");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(mu, "mu"));
  PF_TRY(check_vec(lam, "lam"));
  if (mu_prev) PF_TRY(check_vec(mu_prev, "mu_prev"));
  if (!gparams) {
    set_error("gparams is NULL");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(s, &t0));
  PF_TRY(pc_setup(pb, U, opts->pc, opts->pc_precision, s));
  Op op{pb, U, Uprev, nullptr, 2};
  int its = 0;
  int rc = fgmres(pb, op, mu, 1.0, -1.0, lam, opts->tau_r, *opts, &its, s);
  if (stats) {
    stats->gmres_its_total = its;
    stats->gmres_its[0] = its;
    stats->status = rc;
  }
  if (rc != PF_OK) return rc;
  double* gP = pb->tmp_vec[4];
  double* gp_local = pb->red_out + kSlotParams;
  PF_TRY(launch_residual_family(pb, MODE_VJPP, U, Uprev, lam, nullptr, nullptr, nullptr, gP,
                                pb->vjp_partials, s));
  PF_TRY(blas_reduce_partials(pb->vjp_partials, pb->n_elem_blocks, 2, gp_local, 1.0, s));
  PF_TRY(blas_sub_scalars(gparams, gp_local, 2, s));
  if (mu_prev) PF_TRY(blas_axpby(-1.0, gP, 0.0, gP, mu_prev, pb->n_dof, s));
  PF_HIP_CHECK(hipStreamSynchronize(s));
  if (stats) stats->t_total_ms = now_ms() - t0;
  return PF_OK;
}

int pf_adjoint_solve(pf_problem* pb, const double* U, const double* Uprev, const double* rhs,
                     double* lam, const pf_solver_opts* opts, pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 0));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(rhs, "rhs"));
  PF_TRY(check_vec(lam, "lam"));
  hipStream_t s = S(stream);
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(s, &t0));
  PF_TRY(pc_setup(pb, U, opts->pc, opts->pc_precision, s));
  Op op{pb, U, Uprev, nullptr, 2};
  int its = 0;
  const int rc = fgmres(pb, op, rhs, 1.0, -1.0, lam, opts->tau_r, *opts, &its, s);
  if (stats) {
    stats->gmres_its_total = its;
    stats->gmres_its[0] = its;
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_set_alloy(pf_problem* pb, const pf_alloy_params* a) {
  clear_stale_error();
  if (!pb || !a) {
    set_error("handle or alloy parameters are NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (pb->params.order == 2) {
    set_error("the alloy model uses order-1 elements");
    return PF_ERR_INVALID_ARG;
  }
  if (!(a->k > 0.0 && a->k <= 1.0) || !(a->l_T > 0.0) || !std::isfinite(a->x_iso) ||
      !std::isfinite(a->v_pull)) {
    set_error("alloy parameters need 0 < k <= 1, l_T > 0 and finite x_iso, v_pull");
    return PF_ERR_INVALID_ARG;
  }
  const int NA = 1 << pb->geo.dim;
  const long long need = (long long)2 * NA * pb->geo.n_elems;
  if (pb->elem_buf_len < need) {
    if (pb->elem_buf) PF_HIP_CHECK(hipFree(pb->elem_buf));
    pb->elem_buf = nullptr;
    pb->elem_buf_len = 0;
    if (hipMalloc(&pb->elem_buf, (size_t)need * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      pb->elem_buf = nullptr;
      set_error("out of device memory for the alloy element buffer");
      return PF_ERR_OOM;
    }
    pb->elem_buf_len = need;
  }
  if (!pb->hist) {
    if (hipMalloc(&pb->hist, (size_t)pb->geo.n_nodes * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      pb->hist = nullptr;
      set_error("out of device memory for the alloy history field");
      return PF_ERR_OOM;
    }
  }
  pb->alloy = *a;
  pb->model = 1;
  return PF_OK;
}

int pf_alloy_residual(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                      double t, double* F, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 1));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(F, "F"));
  hipStream_t s = S(stream);
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  pb->t_new = t;
  return launch_alloy(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, F, nullptr, s);
}

int pf_alloy_explicit(pf_problem* pb, const double* Uprev, double t_prev, double* E, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 1));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(E, "E"));
  return alloy_explicit(pb, Uprev, t_prev, E, S(stream));
}

int pf_alloy_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                 double t, const double* v, const double* F0, int mode, double* Jv, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 1));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(v, "v"));
  PF_TRY(check_vec(Jv, "Jv"));
  if (mode != PF_JV_FD && mode != PF_JV_ANALYTIC) {
    set_error("mode must be PF_JV_FD or PF_JV_ANALYTIC");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  pb->t_new = t;
  if (mode == PF_JV_ANALYTIC)
    return launch_alloy(pb, MODE_JVP, U, Uprev, v, nullptr, nullptr, Jv, nullptr, s);
  const double* base = F0;
  if (!base) {
    PF_TRY(launch_alloy(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, pb->tmp_vec[0], nullptr,
                        s));
    base = pb->tmp_vec[0];
  } else {
    PF_TRY(check_vec(F0, "F0"));
  }
  PF_TRY(blas_fd_eps(pb, U, v, pb->n_dof, pb->eps_dev, s));
  return launch_alloy(pb, MODE_FD, U, Uprev, v, base, pb->eps_dev, Jv, nullptr, s);
}

int pf_alloy_step(pf_problem* pb, const double* Uprev2, const double* Uprev, double t_prev,
                  double* U, const pf_solver_opts* opts, pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 1));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(U, "U"));
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(S(stream), &t0));
  int rc = alloy_step_impl(pb, Uprev2, Uprev, t_prev, U, *opts, stats, S(stream));
  if (stats) {
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_alloy_evolve(pf_problem* pb, double* states, int steps, double t0,
                    const pf_solver_opts* opts, pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 1));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(states, "states"));
  if (steps < 0) {
    set_error("steps must be >= 0");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  return evolve_loop(pb, states, steps, stats, s,
                     [&](const double* prev2, const double* prev, int k, double* next,
                         pf_solver_stats* st) {
                       return alloy_step_impl(pb, prev2, prev, t0 + k * pb->params.dt, next,
                                              *opts, st, s);
                     });
}

int pf_set_freegrowth(pf_problem* pb, const pf_freegrowth_params* f) {
  clear_stale_error();
  if (!pb || !f) {
    set_error("handle or free-growth parameters are NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (!(f->Gamma > 0.0) || !(f->W > 0.0) || !(f->alpha > 0.0) || !std::isfinite(f->beta) ||
      !std::isfinite(f->Gamma) || !std::isfinite(f->Lcp) || !std::isfinite(f->Tm)) {
    set_error("free-growth parameters need Gamma, W, alpha > 0 and finite beta, Lcp, Tm");
    return PF_ERR_INVALID_ARG;
  }
  pb->fg = *f;
  const long long need = fg_elem_buf_len(pb);
  if (pb->elem_buf_len < need) {
    if (pb->elem_buf) PF_HIP_CHECK(hipFree(pb->elem_buf));
    pb->elem_buf = nullptr;
    pb->elem_buf_len = 0;
    if (hipMalloc(&pb->elem_buf, (size_t)need * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      pb->elem_buf = nullptr;
      set_error("out of device memory for the free-growth element buffer");
      return PF_ERR_OOM;
    }
    pb->elem_buf_len = need;
  }
  if (!pb->hist) {
    if (hipMalloc(&pb->hist, (size_t)pb->geo.n_nodes * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      pb->hist = nullptr;
      set_error("out of device memory for the history field");
      return PF_ERR_OOM;
    }
  }
  pb->model = 2;
  return PF_OK;
}

int pf_fg_residual(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                   double* F, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 2));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(F, "F"));
  hipStream_t s = S(stream);
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  return launch_fg(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, F, nullptr, s);
}

int pf_fg_explicit(pf_problem* pb, const double* Uprev, double* E, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 2));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(E, "E"));
  return fg_explicit(pb, Uprev, E, S(stream));
}

int pf_fg_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
              const double* v, const double* F0, int mode, double* Jv, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 2));
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(v, "v"));
  PF_TRY(check_vec(Jv, "Jv"));
  if (mode != PF_JV_FD && mode != PF_JV_ANALYTIC) {
    set_error("mode must be PF_JV_FD or PF_JV_ANALYTIC");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  PF_TRY(history_rate(pb, Uprev, Uprev2, s));
  if (mode == PF_JV_ANALYTIC)
    return launch_fg(pb, MODE_JVP, U, Uprev, v, nullptr, nullptr, Jv, nullptr, s);
  const double* base = F0;
  if (!base) {
    PF_TRY(launch_fg(pb, MODE_RES, U, Uprev, nullptr, nullptr, nullptr, pb->tmp_vec[0], nullptr, s));
    base = pb->tmp_vec[0];
  } else {
    PF_TRY(check_vec(F0, "F0"));
  }
  PF_TRY(blas_fd_eps(pb, U, v, pb->n_dof, pb->eps_dev, s));
  return launch_fg(pb, MODE_FD, U, Uprev, v, base, pb->eps_dev, Jv, nullptr, s);
}

int pf_fg_step(pf_problem* pb, const double* Uprev2, const double* Uprev, double* U,
               const pf_solver_opts* opts, pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 2));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(Uprev2, "Uprev2"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(U, "U"));
  stats_reset(stats);
  double t0;
  PF_TRY(clock_start(S(stream), &t0));
  int rc = fg_step_impl(pb, Uprev2, Uprev, U, *opts, stats, S(stream));
  if (stats) {
    stats->status = rc;
    stats->t_total_ms = now_ms() - t0;
  }
  return rc;
}

int pf_fg_evolve(pf_problem* pb, double* states, int steps, const pf_solver_opts* opts,
                 pf_solver_stats* stats, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(require_model(pb, 2));
  PF_TRY(check_opts(pb, opts));
  PF_TRY(check_vec(states, "states"));
  if (steps < 0) {
    set_error("steps must be >= 0");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = S(stream);
  return evolve_loop(pb, states, steps, stats, s,
                     [&](const double* prev2, const double* prev, int, double* next,
                         pf_solver_stats* st) {
                       return fg_step_impl(pb, prev2, prev, next, *opts, st, s);
                     });
}

int pf_misfit(pf_problem* pb, const double* U, const double* phi_target, double* L_dev,
              double* dLdU, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(U, "U"));
  if (!phi_target || !L_dev) {
    set_error("phi_target and L_dev must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (dLdU) PF_TRY(check_vec(dLdU, "dLdU"));
  hipStream_t s = S(stream);
  const int nb = pb->n_red_blocks;
  hipLaunchKernelGGL(k_misfit, dim3(nb), dim3(256), 0, s, pb->geo,
                     reinterpret_cast<const double2*>(U), phi_target,
                     reinterpret_cast<double2*>(dLdU), pb->red_partials);
  PF_HIP_CHECK(hipGetLastError());
  return blas_reduce_partials(pb->red_partials, nb, 1, L_dev, 1.0, s);
}

int pf_dot(pf_problem* pb, const double* x, const double* y, double* out_dev, void* stream) {
  clear_stale_error();
  if (!pb) {
    set_error("handle is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(x, "x"));
  PF_TRY(check_vec(y, "y"));
  if (!out_dev) {
    set_error("out_dev is NULL");
    return PF_ERR_INVALID_ARG;
  }
  return blas_dot(pb, x, y, pb->n_dof, out_dev, S(stream));
}

}  // extern "C"
