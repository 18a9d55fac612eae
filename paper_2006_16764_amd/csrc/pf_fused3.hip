// Single-pass 3-D residual family (F, fused FD Jv, analytic Jv, VJP).
//
// A workgroup of 256 lanes owns a tile of 16 x 16 element columns and marches
// through KZ element layers in z.  Per layer it stages the next node plane
// (17 x 17 nodes of U, U^n and the direction/cotangent V; for the FD product
// the perturbed state U + eps V) in LDS, every lane evaluates one element
// (pf_element.h) and the node sums are formed in LDS in a fixed order:
//   plane k = (top contributions of layer k-1, carried in registers)
//           + (bottom contributions of layer k).
// Nodes strictly inside the tile box are complete and written once.  Nodes on
// the tile's side faces or on its first/last plane also receive contributions
// from neighbouring tiles; their partial sums go to a side buffer that holds,
// per tile and densely, only those ring nodes (the first and last planes
// whole, the perimeter of every plane between them), and k_fixup3 -- one
// workgroup per tile, over the ring nodes that tile owns -- adds the partials
// of the <= 8 tiles that share such a node, in a fixed tile order.  No atomics:
// results are bitwise reproducible.
#include "pf_element.h"

namespace pf {

namespace {

// element layers per z-chunk (a build-time tuning knob: 8 and 32 measured
// 1-2 % slower for the residual and FD product at 256^3)
#ifndef PF_FUSED_KZ
#define PF_FUSED_KZ 16
#endif
constexpr int TX = 16, TY = 16, KZ = PF_FUSED_KZ;
constexpr int PX = TX + 1, PY = TY + 1;
constexpr int PN = PX * PY;  // nodes per staged plane
constexpr int kThreads = TX * TY;
// side buffer: per tile the first plane (PN nodes), the last plane (PN) and
// the perimeter ring of each of the KZ - 1 planes between them (RING nodes)
constexpr int RING = 2 * (TX + TY);
constexpr int SN = 2 * PN + (KZ - 1) * RING;

// Position of node (lx, ly) on the perimeter of the lxmax x lymax node box of
// a tile plane: bottom edge left to right, right edge upwards, top edge right
// to left, left edge downwards (2 (lxmax + lymax) positions).
__device__ __forceinline__ int ring_pos(int lx, int ly, int lxmax, int lymax) {
  if (ly == 0 && lx < lxmax) return lx;
  if (lx == lxmax && ly < lymax) return lxmax + ly;
  if (ly == lymax && lx > 0) return lxmax + lymax + (lxmax - lx);
  return 2 * lxmax + lymax + (lymax - ly);
}

// Inverse of ring_pos; false for positions beyond the perimeter.
__device__ __forceinline__ bool ring_node(int r, int lxmax, int lymax, int& lx, int& ly) {
  if (r < lxmax) {
    lx = r;
    ly = 0;
    return true;
  }
  r -= lxmax;
  if (r < lymax) {
    lx = lxmax;
    ly = r;
    return true;
  }
  r -= lymax;
  if (r < lxmax) {
    lx = lxmax - r;
    ly = lymax;
    return true;
  }
  r -= lxmax;
  if (r < lymax) {
    lx = 0;
    ly = lymax - r;
    return true;
  }
  return false;
}

// Side-buffer node slot (0 .. SN - 1) of ring node (lx, ly, lz) of a tile with
// node extents lxmax, lymax, kzmax.
__device__ __forceinline__ int side_slot(int lx, int ly, int lz, int lxmax, int lymax, int kzmax) {
  if (lz == 0) return lx + PX * ly;
  if (lz == kzmax) return PN + lx + PX * ly;
  return 2 * PN + (lz - 1) * RING + ring_pos(lx, ly, lxmax, lymax);
}

struct Tiles {
  int ntx, nty, ntz;
};

// Residual and FD product: node planes go from HBM straight into LDS
// (global_load_lds_dwordx4, one double2 per lane, no registers) two planes
// ahead through a ring of three plane slots.  PF_FUSED_DMA=0 at build time
// keeps the register-staged loads instead.
#ifndef PF_FUSED_DMA
#define PF_FUSED_DMA 1
#endif
// the same copies for the tangent and adjoint kernels (else register prefetch)
#ifndef PF_FUSED_DMA_ALL
#define PF_FUSED_DMA_ALL 1
#endif
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// One double2 per active lane from src into the LDS slot of the lane's node:
// the instruction writes lane i of the wave at base + 16 i, so the destination
// is the wave's first node (n rounded down to a multiple of 64).
__device__ __forceinline__ void dma16(const double2* src, double2* lds_row, int n) {
  __builtin_amdgcn_global_load_lds((glb_void_t*)src, (lds_void_t*)(lds_row + (n & ~63)), 16, 0, 0);
}

// s_waitcnt vmcnt(0): this wave's outstanding memory operations, the plane
// copies into LDS included, have completed.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

#ifndef PF_TAN_SRC
#define PF_TAN_SRC 1
#endif
// the residual stages all 8 corners of its element vectors at once (0: halves)
#ifndef PF_RES_CB8
#define PF_RES_CB8 1
#endif
// waves per SIMD of the analytic product and the lean adjoint products when
// they read corners from the staged planes (a build-time knob: 1 or 2)
#ifndef PF_TAN_WAVES
#define PF_TAN_WAVES 2
#endif
template <int MODE>
constexpr int kWavesPerSimd = (MODE == MODE_RES || MODE == MODE_FD) ? 2
                              : (MODE == MODE_VJP || !PF_TAN_SRC || !PF_FUSED_DMA || !PF_FUSED_DMA_ALL) ? 1
                                                                                      : PF_TAN_WAVES;

// Corner source of Element::run_src built from three callables.
template <class C, class P, class L>
struct LdsCorners {
  C c;
  P p;
  L l;
  double* out0;  // this lane's slot of output field 0, corner 0
  int ostride;   // between output fields
  int cstride;   // between corners
  __device__ __forceinline__ void corner(int a, double2& u, double2& pp, double2& v) { c(a, u, pp, v); }
  __device__ __forceinline__ void plane(int gz) { p(gz); }
  __device__ __forceinline__ void loaded(int gz) { l(gz); }
  __device__ __forceinline__ double* out(int o) { return out0 + o * ostride; }
  __device__ __forceinline__ int stride() const { return cstride; }
};

template <int MODE>
struct ModeInfo {
  static constexpr bool kHasV = MODE != MODE_RES;
  static constexpr int NO = MODE == MODE_VJP ? 4 : 2;  // doubles per node output
};

__device__ __forceinline__ long long gnode(const Geo& G, int x, int y, int z) {
  return x + (long long)G.nn[0] * (y + (long long)G.nn[1] * z);
}

// Waves per SIMD (the launch bound): two for the residual, the FD product and
// -- reading their corner values from the staged planes at every Gauss plane
// -- the analytic product and the two lean adjoint products; one for the
// adjoint with all outputs, which needs the whole register file.  kCoef (residual
// only): also write the cell means of a^2 for the preconditioner -- a
// separate instantiation, so that the plain residual carries no branch or
// store for it and profiles name the two kernels apart.
template <int MODE, bool kCoef = false>
__global__ void __launch_bounds__(kThreads, kWavesPerSimd<MODE>)
    k_fused3(Geo G, Tiles T, const double2* __restrict__ U, const double2* __restrict__ Up,
             const double2* __restrict__ V, const double* __restrict__ eps_dev,
             const double2* __restrict__ F0, double2* __restrict__ out0, double2* __restrict__ out1,
             double* __restrict__ side, double* __restrict__ vjp_part, double* __restrict__ coef) {
  using MI = ModeInfo<MODE>;
  constexpr int NO = MI::NO;
  // plane copies straight into LDS (residual, FD product): three slots
  constexpr bool kDma = PF_FUSED_DMA && (PF_FUSED_DMA_ALL || MODE == MODE_RES || MODE == MODE_FD);
  constexpr int NS = kDma ? 3 : 2;
  // FD through the copies: raw U and V staged, U + eps V formed at the corner reads
  constexpr bool kRawV = kDma && MODE == MODE_FD;
  // tangent and adjoint modes with copies: corner values read from the staged
  // planes at every Gauss plane instead of held in registers (PF_TAN_SRC=0 at
  // build time keeps them in registers)
  constexpr bool kSrc = PF_TAN_SRC && kDma && !(MODE == MODE_RES || MODE == MODE_FD);
  __shared__ double2 su[NS][PN];
  __shared__ double2 sp[NS][PN];
  __shared__ double2 sv[(MI::kHasV && MODE != MODE_FD) || kRawV ? NS : 1]
                       [(MI::kHasV && MODE != MODE_FD) || kRawV ? PN : 1];
  // FD product: F0 of the staged planes, so that the node writes need no load
  __shared__ double2 sf[MODE == MODE_FD ? NS : 1][MODE == MODE_FD ? PN : 1];
  // element vectors for the node sums: corner halves staged one at a time
  // (4 corners), or -- the modes that read corners from the planes -- all 8
  // corners, accumulated there by the element routine itself
  // (the residual stages all 8 too: two barriers per layer fewer; the FD
  // product keeps the halves, its staged F0 planes leave no LDS for them)
  constexpr bool kCb8 = kSrc || (MODE == MODE_RES && PF_RES_CB8);
  constexpr int kCbA = kCb8 ? 8 : 4;
  __shared__ double cb[NO][kCbA][kThreads];

  const int tid = threadIdx.x;
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % T.ntx;
  const int ty = (tile / T.ntx) % T.nty;
  const int tz = tile / (T.ntx * T.nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * KZ;
  const int lxmax = min(TX, G.n[0] - x0);  // last local node index in x
  const int lymax = min(TY, G.n[1] - y0);
  const int kzmax = min(KZ, G.n[2] - z0);  // element layers in this chunk
  const int ei = tid % TX, ej = tid / TX;  // this lane's element column
  const bool has_elem = ei < lxmax && ej < lymax;
  // FD product: eps_dev holds eps and 1/eps (0 when eps is 0)
  const double eps = (MODE == MODE_FD) ? eps_dev[0] : 0.0;
  const double ieps = (MODE == MODE_FD) ? eps_dev[1] : 0.0;

  // node ownership for the gathers: lane owns node tid and, for tid < PN - 256, node 256 + tid
  constexpr int kSecond = PN - kThreads;  // 33
  const int nA = tid, nB = tid + kThreads;
  const bool ownB = tid < kSecond;
  // top-corner sums carried to the next plane, per owned node, in LDS (only
  // the owning lane reads and writes its entries): no registers held across
  // the element evaluation
  __shared__ double carry[NO][PN];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    carry[o][nA] = 0.0;
    if (ownB) carry[o][nB] = 0.0;
  }

  auto load_plane = [&](int slot, int z) {
    for (int n = tid; n < PN; n += kThreads) {
      const int lx = n % PX, ly = n / PX;
      if (lx <= lxmax && ly <= lymax) {
        const long long g = gnode(G, x0 + lx, y0 + ly, z);
        double2 u = U[g];
        if (MODE == MODE_FD) {
          const double2 v = V[g];
          u.x = fma(eps, v.x, u.x);
          u.y = fma(eps, v.y, u.y);
          sf[slot][n] = F0[g];
        } else if (MI::kHasV) {
          sv[slot][n] = V[g];
        }
        su[slot][n] = u;
        sp[slot][n] = Up[g];
      }
    }
  };

  // Plane z into ring slot `slot` by direct copies into LDS (kDma modes); the
  // copies complete by the wave's next wait_vm().
  auto dma_plane = [&](int slot, int z) {
    for (int n = tid; n < PN; n += kThreads) {
      const int lx = n % PX, ly = n / PX;
      if (lx <= lxmax && ly <= lymax) {
        const long long g = gnode(G, x0 + lx, y0 + ly, z);
        dma16(U + g, &su[slot][0], n);
        dma16(Up + g, &sp[slot][0], n);
        if (kRawV) {
          dma16(V + g, &sv[slot][0], n);
          dma16(F0 + g, &sf[slot][0], n);
        } else if (MI::kHasV && MODE != MODE_FD) {
          dma16(V + g, &sv[slot][0], n);
        }
      }
    }
  };

  // Plane prefetch (modes at one wave per SIMD, whose single workgroup per
  // compute unit would otherwise wait out every plane load): the next-but-one
  // node plane is read right after the element evaluation and stored to its
  // LDS slot after the next barrier, so its memory latency is spent in the
  // node-sum phase.  The residual and FD product run two workgroups per
  // compute unit, which cover each other's loads, and have no registers to
  // spare for it.
  constexpr bool kPrefetch = !kDma && !(MODE == MODE_RES || MODE == MODE_FD);
  static_assert(!(kPrefetch && MODE == MODE_FD), "the prefetch path does not stage F0");
  // Node tid of the plane goes through registers; the few nodes beyond the
  // first kThreads are read when stored.
  double2 fu, fp, fv;
  bool fok;
  auto fetch_plane = [&](int z) {
    const int lx = tid % PX, ly = tid / PX;
    fok = lx <= lxmax && ly <= lymax;
    if (fok) {
      const long long g = gnode(G, x0 + lx, y0 + ly, z);
      fu = U[g];
      fp = Up[g];
      if (MI::kHasV) fv = V[g];
    }
  };
  auto store_plane = [&](int slot, int z) {
    if (fok) {
      double2 u = fu;
      if (MODE == MODE_FD) {
        u.x = fma(eps, fv.x, u.x);
        u.y = fma(eps, fv.y, u.y);
      } else if (MI::kHasV) {
        sv[slot][tid] = fv;
      }
      su[slot][tid] = u;
      sp[slot][tid] = fp;
    }
    for (int n = tid + kThreads; n < PN; n += kThreads) {
      const int lx = n % PX, ly = n / PX;
      if (lx <= lxmax && ly <= lymax) {
        const long long g = gnode(G, x0 + lx, y0 + ly, z);
        double2 u = U[g];
        if (MODE == MODE_FD) {
          const double2 v = V[g];
          u.x = fma(eps, v.x, u.x);
          u.y = fma(eps, v.y, u.y);
        } else if (MI::kHasV) {
          sv[slot][n] = V[g];
        }
        su[slot][n] = u;
        sp[slot][n] = Up[g];
      }
    }
  };

  const long long tile_base = (long long)tile * SN;
  // Write the sum of node n (local) of plane lz: final value or side-buffer
  // partial.  Plane lz is staged in slot lz % 3 (plane copies) or lz & 1.
  auto emit = [&](int n, int lz, const double* acc) {
    const int lx = n % PX, ly = n / PX;
    if (lx > lxmax || ly > lymax) return;
    const bool ring = lx == 0 || lx == lxmax || ly == 0 || ly == lymax || lz == 0 || lz == kzmax;
    if (ring) {
      double* s = side + (tile_base + side_slot(lx, ly, lz, lxmax, lymax, kzmax)) * NO;
      if (MODE == MODE_FD) {
        // the tile that owns the node in the fixup (below its upper extent
        // along every axis, or on the mesh's upper face) subtracts F0 from its
        // partial, so that the fixup needs no F0: Jv = (sum of partials)/eps
        const bool owned = (lx < lxmax || tx == T.ntx - 1) && (ly < lymax || ty == T.nty - 1) &&
                           (lz < kzmax || tz == T.ntz - 1);
        const double2 f0 = owned ? sf[kDma ? lz % 3 : lz & 1][n] : make_double2(0.0, 0.0);
        s[0] = acc[0] - f0.x;
        s[1] = acc[1] - f0.y;
        return;
      }
#pragma unroll
      for (int o = 0; o < NO; ++o) s[o] = acc[o];
      return;
    }
    const long long g = gnode(G, x0 + lx, y0 + ly, z0 + lz);
    if (MODE == MODE_FD) {
      const double2 f0 = sf[kDma ? lz % 3 : lz & 1][n];
      out0[g] = make_double2((acc[0] - f0.x) * ieps, (acc[1] - f0.y) * ieps);
    } else {
      if (out0) out0[g] = make_double2(acc[0], acc[1]);
      if (NO == 4 && out1) out1[g] = make_double2(acc[2 % NO], acc[3 % NO]);
    }
  };

  // Sum of corner half h (0 = bottom corners a = 0..3, 1 = top a = 4..7) of the
  // <= 4 in-plane elements around local node n.
  auto gather = [&](int n, double* acc, int half) {
    const int lx = n % PX, ly = n / PX;
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int e_j = ly - 1 + by;
      if (e_j < 0 || e_j >= lymax) continue;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int e_i = lx - 1 + bx;
        if (e_i < 0 || e_i >= lxmax) continue;
        const int lane = e_i + TX * e_j;
        const int a = (1 - bx) + 2 * (1 - by);
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] += cb[o][(kCb8 ? 4 * half : 0) + a][lane];
      }
    }
  };

  double ge = 0.0, gl = 0.0;
  if (kDma) {
    dma_plane(0, z0);
    dma_plane(1, z0 + 1);
    wait_vm();
    __syncthreads();
  } else {
    load_plane(0, z0);
    if (kPrefetch) {
      load_plane(1, z0 + 1);
      __syncthreads();
    }
  }
  for (int kz = 0; kz < kzmax; ++kz) {
    // ring slots: plane kz in kz % 3 (copies) or kz & 1
    const int bot = kDma ? kz % 3 : kz & 1;
    const int top = kDma ? (kz + 1) % 3 : bot ^ 1;
    const bool more = kPrefetch && kz + 2 <= kzmax;  // plane z0 + kz + 2 exists in this chunk
    if (!kDma && !kPrefetch) {
      load_plane(top, z0 + kz + 1);
      __syncthreads();
    }
    double out[NO][8];
    double u0[8], u1[8], p0[8], p1[8], v0[8], v1[8];
    if (!kSrc && has_elem) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int slot = (a & 4) ? top : bot;
        const int n = (ei + (a & 1)) + PX * (ej + ((a >> 1) & 1));
        double2 u = su[slot][n];
        if (kRawV) {
          const double2 v = sv[slot][n];
          u.x = fma(eps, v.x, u.x);
          u.y = fma(eps, v.y, u.y);
        }
        const double2 up = sp[slot][n];
        u0[a] = u.x;
        u1[a] = u.y;
        p0[a] = up.x;
        p1[a] = up.y;
        if (MODE == MODE_JVP || MODE == MODE_VJP || MODE == MODE_VJPU || MODE == MODE_VJPP) {
          const double2 v = sv[slot][n];
          v0[a] = v.x;
          v1[a] = v.y;
        } else {
          v0[a] = v1[a] = 0.0;
        }
      }
    }
    // the next-but-one plane is copied once the corner values are in registers
    // (the compiler orders LDS reads of the ring after copies into it): slot
    // (kz + 2) % 3 last held plane kz - 1, which no lane reads any more
    if (kDma && kz + 2 <= kzmax && !(kSrc && has_elem)) dma_plane((kz + 2) % 3, z0 + kz + 2);
    if (has_elem) {
      double eg = 0.0, lg = 0.0;
      if constexpr (kSrc) {
        // corner values straight from the staged planes at every Gauss plane;
        // the next-but-one plane is copied after the first plane's reads (its
        // copy then overlaps the first plane's work: the reads of the next
        // planes wait for it)
        auto corner = [&](int a, double2& u, double2& p, double2& v) {
          const int slot = (a & 4) ? top : bot;
          const int n = (ei + (a & 1)) + PX * (ej + ((a >> 1) & 1));
          u = su[slot][n];
          p = sp[slot][n];
          v = sv[slot][n];
        };
        auto plane = [&](int) { __asm__ volatile("" ::: "memory"); };
        auto loaded = [&](int gz) {
          if (gz == 0 && kz + 2 <= kzmax) dma_plane((kz + 2) % 3, z0 + kz + 2);
        };
        LdsCorners<decltype(corner), decltype(plane), decltype(loaded)> src{corner, plane, loaded,
                                                                            &cb[0][0][tid], kCbA * kThreads,
                                                                            kThreads};
        Element<3, MODE>::run_src(G, src, eg, lg);
      } else {
        Element<3, MODE>::run(G, u0, u1, p0, p1, v0, v1, out, eg, lg);
      }
      if (MODE == MODE_RES) {
        // cell mean of a^2 for the preconditioner (weights sum to 8 jac)
        if (kCoef) coef[(x0 + ei) + (long long)G.n[0] * ((y0 + ej) + (long long)G.n[1] * (z0 + kz))] =
            eg / (8.0 * G.jac);
      } else {
        ge += eg;
        gl += lg;
      }
    } else {
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int a = 0; a < 8; ++a) out[o][a] = 0.0;
    }
    // bottom corners -> plane kz (kSrc: all corners are in cb already;
    // kCb8: all corners staged at once)
    if constexpr (!kSrc) {
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int a = 0; a < kCbA; ++a) cb[o][a][tid] = out[o][a];
    }
    if (more) fetch_plane(z0 + kz + 2);
    __syncthreads();
    {
      double acc[NO];
      gather(nA, acc, 0);
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] += carry[o][nA];
      emit(nA, kz, acc);
      if (ownB) {
        gather(nB, acc, 0);
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] += carry[o][nB];
        emit(nB, kz, acc);
      }
    }
    // slot bot (plane kz) is no longer read: every lane has passed the
    // element evaluation; it takes plane kz + 2
    if (more) store_plane(bot, z0 + kz + 2);
    // top corners -> carried to plane kz + 1
    if constexpr (!kCb8) {
      __syncthreads();
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int a = 0; a < 4; ++a) cb[o][a][tid] = out[o][a + 4];
      __syncthreads();
    }
    {
      double acc[NO];
      gather(nA, acc, 1);
#pragma unroll
      for (int o = 0; o < NO; ++o) carry[o][nA] = acc[o];
      if (ownB) {
        gather(nB, acc, 1);
#pragma unroll
        for (int o = 0; o < NO; ++o) carry[o][nB] = acc[o];
      }
    }
    // the plane copied at the top of this iteration is read in the next one
    if (kDma) wait_vm();
    __syncthreads();
  }
  {
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = carry[o][nA];
    emit(nA, kzmax, acc);
    if (ownB) {
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] = carry[o][nB];
      emit(nB, kzmax, acc);
    }
  }

  if (MODE == MODE_VJP || MODE == MODE_VJPP) {
    // fixed-order block reduction of the parameter sums (cb reused as scratch)
    double* red = &cb[0][0][0];
    red[tid] = ge;
    red[kThreads + tid] = gl;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[tid] += red[tid + w];
        red[kThreads + tid] += red[kThreads + tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      vjp_part[tile] = red[0];
      vjp_part[gridDim.x + tile] = red[kThreads];
    }
  }
}

// Tiles containing coordinate c along an axis with tile width w, tile count nt
// and last node index nmax; returns the count and fills t[0..1], l[0..1].
__device__ __forceinline__ int axis_tiles(int c, int w, int nt, int nmax, int* t, int* l) {
  int k = 0;
  const int hi = c / w;
  if (c % w == 0 && hi - 1 >= 0) {
    t[k] = hi - 1;
    l[k] = w;
    ++k;
  }
  if (hi < nt) {
    t[k] = hi;
    l[k] = c - hi * w;
    ++k;
  }
  (void)nmax;
  return k;
}

// One workgroup per tile: the ring nodes the tile owns -- those whose local
// coordinates are below the tile's upper extent along every axis, or on the
// mesh's upper face along that axis -- each receive the sum of the partials of
// all tiles sharing the node, taken in increasing tile order.  The tile's own
// side-buffer slots enumerate its ring nodes (a superset of the owned ones).
template <int MODE>
__global__ void __launch_bounds__(256)
    k_fixup3(Geo G, Tiles T, const double* __restrict__ side,
             const double* __restrict__ eps_dev, double2* __restrict__ out0,
             double2* __restrict__ out1) {
  constexpr int NO = ModeInfo<MODE>::NO;
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % T.ntx;
  const int ty = (tile / T.ntx) % T.nty;
  const int tz = tile / (T.ntx * T.nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * KZ;
  const int lxmax = min(TX, G.n[0] - x0);
  const int lymax = min(TY, G.n[1] - y0);
  const int kzmax = min(KZ, G.n[2] - z0);
  const bool lastx = tx == T.ntx - 1, lasty = ty == T.nty - 1, lastz = tz == T.ntz - 1;
  const double ie = MODE == MODE_FD ? eps_dev[1] : 0.0;  // 1/eps
  for (int i = (int)threadIdx.x; i < SN; i += 256) {
    int lx, ly, lz;
    if (i < PN) {
      lz = 0;
      lx = i % PX;
      ly = i / PX;
    } else if (i < 2 * PN) {
      if (!lastz) continue;  // the next tile's first plane
      lz = kzmax;
      lx = (i - PN) % PX;
      ly = (i - PN) / PX;
    } else {
      const int j = i - 2 * PN;
      lz = 1 + j / RING;
      if (lz >= kzmax || !ring_node(j % RING, lxmax, lymax, lx, ly)) continue;
    }
    if (lx > lxmax || ly > lymax) continue;
    if ((lx == lxmax && !lastx) || (ly == lymax && !lasty)) continue;  // a neighbour's node
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    int txs[2], lxs[2], tys[2], lys[2], tzs[2], lzs[2];
    const int nx = axis_tiles(x, TX, T.ntx, G.n[0], txs, lxs);
    const int ny = axis_tiles(y, TY, T.nty, G.n[1], tys, lys);
    const int nz = axis_tiles(z, KZ, T.ntz, G.n[2], tzs, lzs);
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    for (int c = 0; c < nz; ++c)
      for (int b = 0; b < ny; ++b)
        for (int a = 0; a < nx; ++a) {
          const long long t = txs[a] + (long long)T.ntx * (tys[b] + (long long)T.nty * tzs[c]);
          const int slot = side_slot(lxs[a], lys[b], lzs[c], min(TX, G.n[0] - TX * txs[a]),
                                     min(TY, G.n[1] - TY * tys[b]), min(KZ, G.n[2] - KZ * tzs[c]));
          const double* sp = side + (t * SN + slot) * NO;
#pragma unroll
          for (int o = 0; o < NO; ++o) acc[o] += sp[o];
        }
    const long long g = gnode(G, x, y, z);
    if (MODE == MODE_FD) {
      // the owning tile's partial already holds -F0 (k_fused3)
      out0[g] = make_double2(acc[0] * ie, acc[1] * ie);
    } else {
      if (out0) out0[g] = make_double2(acc[0], acc[1]);
      if (NO == 4 && out1) out1[g] = make_double2(acc[2 % NO], acc[3 % NO]);
    }
  }
}

Tiles tiles_for(const Geo& G) {
  Tiles T;
  T.ntx = (G.n[0] + TX - 1) / TX;
  T.nty = (G.n[1] + TY - 1) / TY;
  T.ntz = (G.n[2] + KZ - 1) / KZ;
  return T;
}

// side: the tile-face partial sums, fused3_side_len(G) doubles (the first
// tiles x SN x NO of them are used).
template <int MODE>
int launch_mode(const Geo& G, double* side, const double* U, const double* Uprev, const double* v,
                const double* F0, const double* eps_dev, double* out0, double* out1,
                double* vjp_part, double* coef, hipStream_t s) {
  const Tiles T = tiles_for(G);
  const unsigned nt = (unsigned)(T.ntx * T.nty * T.ntz);
  auto d2 = [](const double* p) { return reinterpret_cast<const double2*>(p); };
  bool with_coef = false;
  if constexpr (MODE == MODE_RES) with_coef = coef != nullptr;
  if constexpr (MODE == MODE_RES) {
    if (with_coef)
      hipLaunchKernelGGL((k_fused3<MODE_RES, true>), dim3(nt), dim3(kThreads), 0, s, G, T, d2(U),
                         d2(Uprev), d2(v), eps_dev, d2(F0), reinterpret_cast<double2*>(out0),
                         reinterpret_cast<double2*>(out1), side, vjp_part, coef);
  }
  if (!with_coef)
    hipLaunchKernelGGL((k_fused3<MODE, false>), dim3(nt), dim3(kThreads), 0, s, G, T, d2(U),
                       d2(Uprev), d2(v), eps_dev, d2(F0), reinterpret_cast<double2*>(out0),
                       reinterpret_cast<double2*>(out1), side, vjp_part, nullptr);
  PF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_fixup3<MODE>), dim3(nt), dim3(256), 0, s, G, T, side,
                     eps_dev, reinterpret_cast<double2*>(out0), reinterpret_cast<double2*>(out1));
  PF_HIP_CHECK(hipGetLastError());
  return PF_OK;
}

}  // namespace

long long fused3_side_len(const Geo& G) {
  const Tiles T = tiles_for(G);
  return (long long)T.ntx * T.nty * T.ntz * SN * 4;
}

int fused3_tiles(const Geo& G) {
  const Tiles T = tiles_for(G);
  return T.ntx * T.nty * T.ntz;
}

long long fused3_residual_side_len(const Geo& G) {
  const Tiles T = tiles_for(G);
  return (long long)T.ntx * T.nty * T.ntz * SN * ModeInfo<MODE_RES>::NO;
}

int launch_fused3_residual(const Geo& G, double* side, const double* U, const double* Uprev,
                           double* F, hipStream_t s) {
  return launch_mode<MODE_RES>(G, side, U, Uprev, nullptr, nullptr, nullptr, F, nullptr, nullptr,
                               nullptr, s);
}

int launch_fused3(pf_problem* pb, int mode, const double* U, const double* Uprev, const double* v,
                  const double* F0, const double* eps_dev, double* out0, double* out1,
                  double* vjp_part, double* coef, hipStream_t s) {
  const Geo& G = pb->geo;
  double* side = pb->side_buf;
  switch (mode) {
    case MODE_RES:
      return launch_mode<MODE_RES>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, coef, s);
    case MODE_FD:
      return launch_mode<MODE_FD>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, nullptr, s);
    case MODE_JVP:
      return launch_mode<MODE_JVP>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, nullptr, s);
    case MODE_VJPU:
      return launch_mode<MODE_VJPU>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, nullptr, s);
    case MODE_VJPP:
      return launch_mode<MODE_VJPP>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, nullptr, s);
    default:
      return launch_mode<MODE_VJP>(G, side, U, Uprev, v, F0, eps_dev, out0, out1, vjp_part, nullptr, s);
  }
}

}  // namespace pf
