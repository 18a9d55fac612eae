// pf_residual_noalloc: the thermal residual without a handle and without any
// device allocation, for callers that cannot allocate (graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The kernels' scratch -- the tile-face partial sums of the 3-D fused kernel,
// or the element vectors of the 2-D two-pass kernels -- lives in one fixed
// array `scratch` inside the library.  Every device that runs the library
// holds its own copy of it from module load until the process ends.  In host
// code the array's name is only a host-side stand-in, so its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and that address, never the name, is what the kernels receive.
#include <mutex>

#include "pf_internal.h"

namespace pf {

namespace {

// 64 MiB: 2727 tiles of 16^3 elements (192^3 fits) or 2^20 elements in 2-D.
constexpr long long kScratchBytes = 64LL << 20;
constexpr long long kScratchDoubles = kScratchBytes / (long long)sizeof(double);

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// Device address of the current device's copy of `scratch`.
int scratch_address(double** out) {
  int dev = -1;
  PF_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("pf_residual_noalloc: device index out of range");
    return PF_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("pf_residual_noalloc: hipGetSymbolAddress(scratch): ") +
                hipGetErrorString(e));
      return PF_ERR_HIP;
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return PF_OK;
}

}  // namespace

}  // namespace pf

extern "C" int pf_residual_noalloc(const pf_params* params, const double* U, const double* Uprev,
                                   double* F, void* stream) {
  using namespace pf;
  clear_stale_error();
  PF_TRY(check_params(params));
  if (params->order == 2) {
    set_error("pf_residual_noalloc: order-1 elements only");
    return PF_ERR_INVALID_ARG;
  }
  PF_TRY(check_vec(U, "U"));
  PF_TRY(check_vec(Uprev, "Uprev"));
  PF_TRY(check_vec(F, "F"));
  pf_params p = *params;
  p.order = 1;
  const Geo G = make_geo(p);
  const long long need = G.dim == 3 ? fused3_residual_side_len(G) : residual2_elem_len(G);
  if (need > kScratchDoubles) {
    set_error("pf_residual_noalloc: mesh needs " + std::to_string(need * 8) +
              " bytes of scratch, more than the fixed " + std::to_string(kScratchBytes) +
              " (3-D: at most 2727 tiles of 16^3 elements; 2-D: at most 2^20 elements)");
    return PF_ERR_INVALID_ARG;
  }
  double* scr = nullptr;
  PF_TRY(scratch_address(&scr));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (G.dim == 3) return launch_fused3_residual(G, scr, U, Uprev, F, s);
  return launch_residual2(G, scr, U, Uprev, F, s);
}
