// Internal definitions shared by the HIP translation units of libpfjfnk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pfjfnk.h"

namespace pf {

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_stale_error();

#define PF_HIP_CHECK(call)                                                         \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::pf::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return PF_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

#define PF_TRY(call)              \
  do {                            \
    int rc_ = (call);             \
    if (rc_ != PF_OK) return rc_; \
  } while (0)

// ----------------------------------------------------------------- geometry
// Mesh and model constants passed by value to every kernel.
struct Geo {
  int dim;
  int n[3];    // elements per axis (n[2] = 1 in 2-D)
  int nn[3];   // nodes per axis (nn[2] = 1 in 2-D)
  long long n_nodes;
  long long n_elems;
  double h[3];
  double ih[3];  // 1/h
  double jac;    // prod(h/2): Jacobian of the reference map
  double dt, idt, eps4, lam, D, delta2;
  double a0, e4x4, e16;  // 1 - 3 eps4, 4 eps4, 16 eps4
  // time weight: the phi-row terms are theta * [a^2 dphi idtm + spatial],
  // idtm = 1/(theta dt); Dth = theta D, hth = theta/2 (latent rate)
  double theta, idtm, Dth, hth;
};

Geo make_geo(const pf_params& p);

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Tiled kernels map the hardware workgroup index i to the logical tile so
// that each XCD runs a contiguous run of tiles: neighbours then share their
// halo rows in one L2 instead of fetching them from HBM separately.  The
// first 8 floor(T/8) indices are permuted, the remainder keeps its order.
#ifndef PF_XCD_REMAP
#define PF_XCD_REMAP 1
#endif
constexpr unsigned kNumXcd = 8;
__device__ __forceinline__ unsigned xcd_tile(unsigned i, unsigned T) {
  if (!PF_XCD_REMAP) return i;
  const unsigned q = T / kNumXcd;
  if (i >= kNumXcd * q) return i;
  return (i % kNumXcd) * q + i / kNumXcd;
}

// Alloy-model constants of one element-kernel launch (host-computed).
struct AlloyConst {
  double omk;       // 1 - k
  double hopk;      // (1 + k)/2
  double g4a, g4b;  // G4 = g4a x + g4b at the launch's time level
  double x0, h0;    // node x coordinate = x0 + i h0 (axis 0)
  double theta;     // time weight of this launch (1 for the explicit part)
  int use_hist;     // 0: the history rate is zero
};

// Free-growth constants of one element-kernel launch (host-computed).
struct FgConst {
  double bg;      // beta Gamma
  double c_dw;    // beta Gamma / W^2 (double-well term)
  double c_drv;   // 5 beta / W (driving-force term)
  double Tm, alpha, Lcp;
  double theta;   // time weight of this launch (1 for the explicit part)
  int use_hist;   // 0: the history rate is zero
  int n_macro[2]; // order 2: elements per axis; h_macro = 2 G.h
};

// Element-loop modes of the residual kernel family.
// MODE_VJPU: (dF/dU)^T w only (the operator of the transposed Krylov solve).
// MODE_VJPP: the adjoint's previous-state output (dF/dUprev)^T w and the two
// parameter sums only (no (dF/dU)^T w).
enum Mode { MODE_RES = 0, MODE_FD = 1, MODE_JVP = 2, MODE_VJP = 3, MODE_VJPU = 4, MODE_VJPP = 5 };

// 3-D single-pass kernels (pf_fused3.hip).  For the FD product, eps_dev[0]
// is the step eps and eps_dev[1] its reciprocal (0 when eps is 0), both
// written by blas_fd_eps / blas_fd_eps_cached.
long long fused3_side_len(const Geo& G);
int fused3_tiles(const Geo& G);
int launch_fused3(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
                  const double* F0, const double* eps_dev, double* out0, double* out1,
                  double* vjp_part, double* coef, hipStream_t s);

// The thermal residual alone with caller-provided scratch: 3-D through the
// fused kernel with side buffer `side` (fused3_residual_side_len(G) doubles),
// 2-D through the two-pass kernels with element buffer `elem`
// (residual2_elem_len(G) doubles).  Same kernels as pf_residual.
long long fused3_residual_side_len(const Geo& G);
int launch_fused3_residual(const Geo& G, double* side, const double* U, const double* Uprev,
                           double* F, hipStream_t s);
long long residual2_elem_len(const Geo& G);
int launch_residual2(const Geo& G, double* elem, const double* U, const double* Uprev, double* F,
                     hipStream_t s);
// Host-side argument checks shared by the entry points (pf_abi.hip).
int check_params(const pf_params* p);
int check_vec(const void* p, const char* name);

// Launch helpers (defined in pf_residual.hip).
// coef (optional, residual mode only): receives the cell mean of a(grad phi)^2,
// the coefficient of the preconditioner's phi block.
int launch_residual_family(pf_problem* pb, int mode, const double* U, const double* Uprev,
                           const double* v, const double* F0, const double* eps_dev,
                           double* out0, double* out1, double* gparams_partial,
                           hipStream_t s, double* coef = nullptr);
// Node sums of the element buffer (pf_residual.hip): out0 = sums, or
// (sums - F0)/eps when fd != 0.
int launch_gather2(pf_problem* pb, double* out0, const double* F0, const double* eps_dev, int fd,
                   hipStream_t s);

// Alloy model (pf_alloy.hip).  launch_alloy: modes RES, FD, JVP at pb->t_new
// with the history rate pb->hist; explicit: the spatial operator at (U, t)
// scaled by 1 - theta.
AlloyConst alloy_const(const pf_problem* pb, double t, double theta, int use_hist);
int launch_alloy(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
                 const double* F0, const double* eps_dev, double* out0, double* coef,
                 hipStream_t s);
int alloy_explicit(pf_problem* pb, const double* Un, double t_n, double* E, hipStream_t s);
int history_rate(pf_problem* pb, const double* Un, const double* Unm1, hipStream_t s);

// Free-growth model (pf_freegrowth.hip), orders 1 and 2: launch_fg modes RES,
// FD, JVP with the history rate pb->hist; fg_explicit: spatial terms at U^n
// scaled by 1 - theta.  Order-2 handles index nodes on the (2n+1)^dim grid
// (pb->geo describes it as an order-1 grid of 2n cells per axis).
int launch_fg(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
              const double* F0, const double* eps_dev, double* out0, double* coef, hipStream_t s);
int fg_explicit(pf_problem* pb, const double* Un, double* E, hipStream_t s);
long long fg_elem_buf_len(const pf_problem* pb);

// ----------------------------------------------------------------- BLAS-1 (pf_blas.hip)
// Deterministic reductions over n doubles: fixed grid, fixed order.
int blas_dot(pf_problem* pb, const double* x, const double* y, long long n, double* out_dev,
             hipStream_t s);
// out_host (device alias of mapped host memory, may be NULL) receives a copy
// of the results for the host, valid once the stream has synchronised.
int blas_multidot(pf_problem* pb, const double* V, long long ld, int k, const double* w,
                  long long n, double* out_dev, hipStream_t s, double* out_host = nullptr);
// Rows of the reduction workspace (red_partials holds kRedRows * n_red_blocks).
constexpr int kRedRows = 128;

// Slots of the handle's 1024-double result arrays: red_out on the device and
// host_pinned (mapped host memory, written by reductions the host waits for).
constexpr int kMaxGmresM = 60;  // largest gmres_m_max pf_create accepts
constexpr int kRedSlots = 1024;
constexpr int kSlotFdU = 200;   // red_out: |U|^2 of the FD step size (one-off form)
constexpr int kSlotFdV = 201;   // red_out: |v|^2 of the FD step size
constexpr int kSlotUnorm = 203; // red_out: |U|^2 kept for the FD operator of a Krylov solve
constexpr int kSlotNorm = 250;  // red_out and host_pinned: |x|^2 of a norm the host reads
constexpr int kSlotHostY = 160; // host_pinned: staging of the FGMRES combination y
constexpr int kSlotY = 300;     // red_out: the FGMRES combination y (<= kMaxGmresM)
constexpr int kSlotParams = 400;  // red_out: the two parameter sums of a VJP
constexpr int kSlotDots = 512;  // red_out and host_pinned: Gram-Schmidt products (<= 2m + 3)
static_assert(kSlotHostY + kMaxGmresM <= kSlotNorm, "host y staging overlaps the norm slot");
static_assert(kSlotY + kMaxGmresM <= kSlotParams, "y overlaps the parameter sums");
static_assert(kSlotDots + 2 * kMaxGmresM + 3 <= kRedSlots, "Gram-Schmidt products overflow");
static_assert(2 * kMaxGmresM + 3 <= kRedRows, "Gram-Schmidt products exceed the reduction rows");
// One Gram-Schmidt step with a delayed second projection (t = V_j, w = V_{j+1}):
// out[0..2j+2] = V_{<j}^T t, t.t, V_{<j}^T w, t.w, w.w in one sweep; then the
// in-place updates t <- (t - V_{<j} s) inv_rho, w <- (w - V_{<j} h - hj t) inv_eta with
// s = out[0..j-1] and h = out[j+1..2j] of that product sweep (left on the device).
int blas_dcgs_dots(pf_problem* pb, const double* V, long long ld, int j, long long n,
                   double* out_dev, hipStream_t s, double* out_host = nullptr);
int blas_dcgs_update(double* V, long long ld, int j, const double* dots_dev, double hj,
                     double inv_rho, double inv_eta, long long n, hipStream_t s);
// x += sum_{j<k} coef_dev[j] V_j; assign: x = that sum (x not read; zeros when k = 0)
int blas_combine(pf_problem* pb, const double* V, long long ld, int k, const double* coef_dev,
                 double* x, long long n, hipStream_t s, bool assign = false);
int blas_scale_copy(const double* x, const double* alpha_dev, int invert, double* y,
                    long long n, hipStream_t s);
// z = a x + b y, and |z|^2 into out_dev (device), the value blas_multidot of z with itself gives
int blas_axpby_norm(pf_problem* pb, double a, const double* x, double b, const double* y, double* z,
                    long long n, double* out_dev, hipStream_t s);
int blas_axpby(double a, const double* x, double b, const double* y, double* z, long long n,
               hipStream_t s);
int blas_fd_eps(pf_problem* pb, const double* U, const double* v, long long n, double* eps_dev,
                hipStream_t s);
// eps from a precomputed |U|^2 (device scalar) and |v|^2 computed here
int blas_fd_eps_cached(pf_problem* pb, const double* unorm2_dev, const double* v, long long n,
                       double* eps_dev, hipStream_t s);
int blas_reduce_partials(const double* partials, int nparts, int k, double* out_dev,
                         double scale, hipStream_t s);
int blas_sub_scalars(double* acc_dev, const double* x_dev, int k, hipStream_t s);

// ----------------------------------------------------------------- preconditioner (pf_gmg.hip)
struct GmgLevel;
int pc_alloc(pf_problem* pb);
hipError_t pc_free(pf_problem* pb);
int pc_setup(pf_problem* pb, const double* U, int kind, int precision, hipStream_t s);
// Setup from cell coefficients already written (by a residual evaluation at the
// same state) into pc_coef_buffer(pb).
int pc_setup_prepared(pf_problem* pb, int kind, int precision, hipStream_t s);
double* pc_coef_buffer(pf_problem* pb);
int pc_apply(pf_problem* pb, const double* r, double* z, hipStream_t s);

// ----------------------------------------------------------------- misc kernels
int misfit_launch(pf_problem* pb, const double* U, const double* target, double* L_dev,
                  double* dLdU, hipStream_t s);

}  // namespace pf

// The opaque handle.
struct pf_problem {
  pf_params params;
  pf::Geo geo;
  int device;
  long long n_dof;  // 2 * n_nodes
  int gmres_m_max;

  // reduction scratch: partial sums [k][n_red_blocks] and results
  int n_red_blocks;
  double* red_partials;  // kRedRows * n_red_blocks
  double* red_out;       // kRedSlots doubles of device results
  double* host_pinned;   // kRedSlots doubles of pinned, mapped host staging
  double* host_pinned_dev;  // its device alias (reductions write results there)

  // residual-family scratch
  double* elem_buf;      // element contributions (element pass)
  long long elem_buf_len;
  double* vjp_partials;  // 2 * n_elem_blocks
  double* side_buf;      // 3-D: partial node sums on tile boundaries
  long long side_len;
  int n_elem_blocks;
  double* eps_dev;       // FD epsilon (device scalar)
  double* tmp_vec[6];    // work vectors of n_dof doubles (kNumTmp)
  double* load_vec;      // theta < 1: the explicit part E of the step (lazy)

  // alloy model (pf_set_alloy): parameters, the history rate
  // (1 - theta)(phi^n - phi^(n-1))/dt per node, and the time of the implicit part
  int model;             // 0 thermal, 1 alloy, 2 free growth
  pf_alloy_params alloy;
  pf_freegrowth_params fg;
  double* hist;          // n_nodes doubles
  double t_new;

  // FGMRES basis
  double* V;  // (m+1) * n_dof
  double* Z;  // m * n_dof

  // preconditioner state
  int pc_kind;
  int pc_precision;
  void* pc;  // pf::PcState*
};
