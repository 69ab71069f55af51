// Compact-stencil Helmholtz operator kernels: apply, residual and the
// omega-Jacobi smoothing step (Sec. 4: V-cycle with omega-Jacobi smoothers).
// One thread per unknown node; the fastest grid axis (y) maps to threadIdx.x
// so that the loads of x along y are coalesced.  One kernel per operator
// kind.
#include "internal.h"

namespace hsp {

namespace {

template <class Ta, class Tx>
__device__ __forceinline__ cx<Ta> ld(const cx<Tx>* v, size_t i) {
  return cvt<Ta>(v[i]);
}

// Loads are unconditional, from clamped (valid) addresses, and neighbours
// outside the grid are masked by a zero coefficient afterwards: a load inside
// a branch would make the compiler wait for it before the join.

// v where ok, else 0, component by component (a select of the whole struct
// would be lowered through private memory).
__device__ __forceinline__ cd keep(bool ok, cd v) { return mk<double>(ok ? v.re : 0.0, ok ? v.im : 0.0); }

// The output stage shared by both kinds: ax = (A x)_id.
template <class Ta, class Tb, class Ty>
__device__ __forceinline__ void stencil_out(int mode, cx<Ta> ax, cx<Ta> xc, bool has_x, const cx<Tb>* b, size_t id,
                                            cd c11, double w, cx<Ty>* y) {
  if (mode == 0) {
    y[id] = cvt<Ty>(ax);
    return;
  }
  const cx<Ta> r = ld<Ta>(b, id) - ax;
  if (mode == 1) {
    y[id] = cvt<Ty>(r);
    return;
  }
  // Jacobi: x + w D^{-1} r
  const cx<Ta> dinv = cvt<Ta>(cinv(c11));
  cx<Ta> out = mk<Ta>(has_x ? xc.re : Ta(0), has_x ? xc.im : Ta(0));
  cfma(out, cvt<Ta>(mk<double>(w, 0.0)) * dinv, r);
  y[id] = cvt<Ty>(out);
}

// 5-point kind (eq. define_pml_fd): coefficients from the per-axis arrays and
// k^2 (the arithmetic of stencil_coefs, kind 5), neighbours in the order
// west, south, centre, north, east.
template <class Ta, class Tx, class Tb, class Ty>
__global__ void __launch_bounds__(256) k_stencil5(LevelDev L, int mode, const cx<Tx>* __restrict__ x,
                                                  const cx<Tb>* __restrict__ b, cx<Ty>* __restrict__ y,
                                                  double w, BIdx bx, BIdx bb, BIdx by) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;  // y node 1..n2
  const int i = blockIdx.y + 1;                             // x node 1..n1
  const int n1 = L.n1, n2 = L.n2;
  if (k > n2) return;
  const int z = blockIdx.z;
  const bool has_x = x != nullptr;
  if (has_x) x += bx.off(z);
  if (b != nullptr) b += bb.off(z);
  y += by.off(z);
  const size_t id = (size_t)(i - 1) * n2 + (k - 1);
  cx<Ta> xw = mk<Ta>(0, 0), xs = xw, xc = xw, xn = xw, xe = xw;
  if (has_x) {
    const size_t iw = i > 1 ? id - n2 : id, ie = i < n1 ? id + n2 : id;
    const size_t is = k > 1 ? id - 1 : id, in = k < n2 ? id + 1 : id;
    xw = ld<Ta>(x, iw);
    xs = ld<Ta>(x, is);
    xc = ld<Ta>(x, id);
    xn = ld<Ta>(x, in);
    xe = ld<Ta>(x, ie);
  }
  const int row = L.xmap ? L.xmap[i - 1] : (i - 1);
  const cd k2 = k2_at(L, (size_t)row * n2 + (k - 1));
  const cd ian = L.xB[i], ikn = L.yB[k];
  cd cw = -(L.xA[i - 1] * ikn), ce = -(L.xA[i] * ikn);
  cd cs = -(L.yA[k - 1] * ian), cn = -(L.yA[k] * ian);
  const cd c11 = -(cw + ce + cs + cn) - (L.h2 * k2) * (ian * ikn);
  cw = keep(i > 1, cw);
  ce = keep(i < n1, ce);
  cs = keep(k > 1, cs);
  cn = keep(k < n2, cn);
  cx<Ta> ax = mk<Ta>(0, 0);
  if (has_x) {
    cfma(ax, cvt<Ta>(cw), xw);
    cfma(ax, cvt<Ta>(cs), xs);
    cfma(ax, cvt<Ta>(c11), xc);
    cfma(ax, cvt<Ta>(cn), xn);
    cfma(ax, cvt<Ta>(ce), xe);
  }
  stencil_out<Ta, Tb, Ty>(mode, ax, xc, has_x, b, id, c11, w, y);
}

// 9-point finite-element kind (App. A): stencil_coefs, all nine neighbours
// loaded from clamped addresses.
template <class Ta, class Tx, class Tb, class Ty>
__global__ void __launch_bounds__(256) k_stencil9(LevelDev L, int mode, const cx<Tx>* __restrict__ x,
                                                  const cx<Tb>* __restrict__ b, cx<Ty>* __restrict__ y,
                                                  double w, BIdx bx, BIdx bb, BIdx by) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;  // y node 1..n2
  const int i = blockIdx.y + 1;                             // x node 1..n1
  const int n1 = L.n1, n2 = L.n2;
  if (k > n2) return;
  const int z = blockIdx.z;
  const bool has_x = x != nullptr;
  if (has_x) x += bx.off(z);
  if (b != nullptr) b += bb.off(z);
  y += by.off(z);
  const size_t id = (size_t)(i - 1) * n2 + (k - 1);
  cx<Ta> xv[3][3];
#pragma unroll
  for (int di = -1; di <= 1; ++di)
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      int ii = i + di, kk = k + dk;
      ii = ii < 1 ? 1 : (ii > n1 ? n1 : ii);
      kk = kk < 1 ? 1 : (kk > n2 ? n2 : kk);
      xv[di + 1][dk + 1] = mk<Ta>(0, 0);
      if (has_x) xv[di + 1][dk + 1] = ld<Ta>(x, (size_t)(ii - 1) * n2 + (kk - 1));
    }
  cd c[3][3];
  stencil_coefs(L, i, k, c);
  cx<Ta> ax = mk<Ta>(0, 0);
#pragma unroll
  for (int di = -1; di <= 1; ++di) {
    const bool okx = i + di >= 1 && i + di <= n1;
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      const bool ok = okx && k + dk >= 1 && k + dk <= n2;
      const cd cc = keep(ok, c[di + 1][dk + 1]);
      cfma(ax, cvt<Ta>(cc), xv[di + 1][dk + 1]);
    }
  }
  stencil_out<Ta, Tb, Ty>(mode, ax, xv[1][1], has_x, b, id, c[1][1], w, y);
}

// Both kinds for nb right-hand sides at once: blockIdx.z selects a group of
// kStencilZ right-hand sides, the coefficients of a node are formed once per
// group and applied to each right-hand side of the group in turn, so the
// batched kernel mostly streams the vectors (the per-node coefficient
// arithmetic and the k^2 / cell data are not repeated per right-hand side).
// Same arithmetic, in the same order, as the one-right-hand-side kernels
// above.
constexpr int kStencilZ = 16;
// Workgroups are dealt to the eight XCDs in turn by their linear index, and
// each XCD has an L2 of its own.  Rows i - 1, i, i + 1 of one group of right-
// hand sides are several workgroups apart, so in launch order they sit on
// different XCDs and every row of x comes from HBM three times.  The
// workgroups are renumbered so that XCD q takes one contiguous range of
// (node block, group) tiles: a permutation of the grid, whatever the dispatch
// order.
__device__ __forceinline__ void xcd_tile(int& tx, int& ty, int& tz) {
  constexpr unsigned kXcd = 8;
  const unsigned gx = gridDim.x, gy = gridDim.y, T = gx * gy * gridDim.z;
  const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned per = T / kXcd, rem = T % kXcd, q = lin % kXcd, slot = lin / kXcd;
  const unsigned t = (q < rem ? q * (per + 1) : rem * (per + 1) + (q - rem) * per) + slot;
  tx = (int)(t % gx);
  ty = (int)((t / gx) % gy);
  tz = (int)(t / (gx * gy));
}
template <int KIND, class Ta, class Tx, class Tb, class Ty>
__global__ void __launch_bounds__(256) k_stencil_multi(LevelDev L, int mode, const cx<Tx>* __restrict__ x,
                                                       const cx<Tb>* __restrict__ b, cx<Ty>* __restrict__ y,
                                                       double w, BIdx bx, BIdx bb, BIdx by, int nb) {
  // the nodes are numbered row by row and taken 256 at a time, so that no
  // lanes idle at the end of each row
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  const int n1 = L.n1, n2 = L.n2;
  const size_t id = (size_t)tx * blockDim.x + threadIdx.x;
  if (id >= (size_t)n1 * n2) return;
  const int i = (int)(id / (unsigned)n2) + 1;        // x node 1..n1
  const int k = (int)(id - (size_t)(i - 1) * n2) + 1;  // y node 1..n2
  const bool has_x = x != nullptr;
  // coefficients (masked toward the boundary) and clamped neighbour indices
  cd c[3][3];
  if constexpr (KIND == 5) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) c[a][q] = mk<double>(0, 0);
    const int row = L.xmap ? L.xmap[i - 1] : (i - 1);
    const cd k2 = k2_at(L, (size_t)row * n2 + (k - 1));
    const cd ian = L.xB[i], ikn = L.yB[k];
    const cd cw = -(L.xA[i - 1] * ikn), ce = -(L.xA[i] * ikn);
    const cd cs = -(L.yA[k - 1] * ian), cn = -(L.yA[k] * ian);
    c[1][1] = -(cw + ce + cs + cn) - (L.h2 * k2) * (ian * ikn);
    c[0][1] = keep(i > 1, cw);
    c[2][1] = keep(i < n1, ce);
    c[1][0] = keep(k > 1, cs);
    c[1][2] = keep(k < n2, cn);
  } else {
    stencil_coefs(L, i, k, c);
  }
  cx<Ta> cc[3][3];
  size_t nid[3][3];
#pragma unroll
  for (int di = -1; di <= 1; ++di)
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      int ii = i + di, kk = k + dk;
      const bool ok = ii >= 1 && ii <= n1 && kk >= 1 && kk <= n2;
      ii = ii < 1 ? 1 : (ii > n1 ? n1 : ii);
      kk = kk < 1 ? 1 : (kk > n2 ? n2 : kk);
      nid[di + 1][dk + 1] = (size_t)(ii - 1) * n2 + (kk - 1);
      cc[di + 1][dk + 1] = cvt<Ta>(KIND == 5 ? c[di + 1][dk + 1] : keep(ok, c[di + 1][dk + 1]));
    }
  const int z0 = tz * kStencilZ, z1 = min(nb, z0 + kStencilZ);
#pragma unroll 2
  for (int z = z0; z < z1; ++z) {
    const cx<Tx>* xz = has_x ? x + bx.off(z) : x;
    const cx<Tb>* bz = b != nullptr ? b + bb.off(z) : b;
    cx<Ty>* yz = y + by.off(z);
    cx<Ta> ax = mk<Ta>(0, 0), xc = mk<Ta>(0, 0);
    if constexpr (KIND == 5) {
      if (has_x) {
        const cx<Ta> xw = ld<Ta>(xz, nid[0][1]), xs = ld<Ta>(xz, nid[1][0]);
        xc = ld<Ta>(xz, id);
        const cx<Ta> xn = ld<Ta>(xz, nid[1][2]), xe = ld<Ta>(xz, nid[2][1]);
        cfma(ax, cc[0][1], xw);
        cfma(ax, cc[1][0], xs);
        cfma(ax, cc[1][1], xc);
        cfma(ax, cc[1][2], xn);
        cfma(ax, cc[2][1], xe);
      }
    } else {
      cx<Ta> xv[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 3; ++q) xv[a][q] = has_x ? ld<Ta>(xz, nid[a][q]) : mk<Ta>(0, 0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 3; ++q) cfma(ax, cc[a][q], xv[a][q]);
      xc = xv[1][1];
    }
    stencil_out<Ta, Tb, Ty>(mode, ax, xc, has_x, bz, id, c[1][1], w, yz);
  }
}

}  // namespace

template <class Ta, class Tx, class Tb, class Ty>
void launch_stencil(const LevelDev& L, int mode, const cx<Tx>* x, const cx<Tb>* b, cx<Ty>* y,
                    double w, hipStream_t s, int nb, BIdx bx, BIdx bb, BIdx by) {
  if (nb < 1) return;
  dim3 blk(256);
  if (nb > 1) {
    const size_t nodes = (size_t)L.n1 * L.n2;
    const dim3 g2((unsigned)((nodes + 255) / 256), 1, (nb + kStencilZ - 1) / kStencilZ);
    if (L.kind == 5)
      hipLaunchKernelGGL((k_stencil_multi<5, Ta, Tx, Tb, Ty>), g2, blk, 0, s, L, mode, x, b, y, w, bx, bb, by, nb);
    else
      hipLaunchKernelGGL((k_stencil_multi<9, Ta, Tx, Tb, Ty>), g2, blk, 0, s, L, mode, x, b, y, w, bx, bb, by, nb);
    return;
  }
  dim3 grd((L.n2 + 255) / 256, L.n1, nb);
  if (L.kind == 5)
    hipLaunchKernelGGL((k_stencil5<Ta, Tx, Tb, Ty>), grd, blk, 0, s, L, mode, x, b, y, w, bx, bb, by);
  else
    hipLaunchKernelGGL((k_stencil9<Ta, Tx, Tb, Ty>), grd, blk, 0, s, L, mode, x, b, y, w, bx, bb, by);
}

#define INST(Ta, Tx, Tb, Ty) \
  template void launch_stencil<Ta, Tx, Tb, Ty>(const LevelDev&, int, const cx<Tx>*, const cx<Tb>*, cx<Ty>*, double, \
                                               hipStream_t, int, BIdx, BIdx, BIdx);
INST(double, double, double, double)
INST(double, float, double, double)
INST(double, float, double, float)
INST(float, float, float, float)
INST(float, float, double, float)
INST(double, double, double, float)
INST(double, float, float, float)
INST(float, float, double, double)
INST(double, float, float, double)
INST(float, float, float, double)
INST(double, double, float, double)
INST(double, double, float, float)
#undef INST

}  // namespace hsp
