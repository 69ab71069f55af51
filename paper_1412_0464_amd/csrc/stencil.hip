// Compact-stencil Helmholtz operator kernels: apply, residual and the
// omega-Jacobi smoothing step (Sec. 4: V-cycle with omega-Jacobi smoothers).
// One thread per unknown node; the fastest grid axis (y) maps to threadIdx.x
// so that the loads of x along y are coalesced.
#include "internal.h"

namespace hsp {

namespace {

template <class Ta, class Tx>
__device__ __forceinline__ cx<Ta> ld(const cx<Tx>* v, size_t i) {
  return cvt<Ta>(v[i]);
}

template <class Ta, class Tx, class Tb, class Ty>
__global__ void __launch_bounds__(256) k_stencil(LevelDev L, int mode, const cx<Tx>* __restrict__ x,
                                                 const cx<Tb>* __restrict__ b, cx<Ty>* __restrict__ y,
                                                 double w, BIdx bx, BIdx bb, BIdx by) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;  // y node 1..n2
  const int i = blockIdx.y + 1;                             // x node 1..n1
  const int n1 = L.n1, n2 = L.n2;
  if (k > n2) return;
  // vector z of a batch (blockIdx.z)
  const int z = blockIdx.z;
  if (x != nullptr) x += bx.off(z);
  if (b != nullptr) b += bb.off(z);
  y += by.off(z);
  cd c[3][3];
  stencil_coefs(L, i, k, c);
  const size_t id = (size_t)(i - 1) * n2 + (k - 1);
  cx<Ta> ax = mk<Ta>(0, 0);
  if (x != nullptr) {
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 1 || ii > n1) continue;
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
        const int kk = k + dk;
        if (kk < 1 || kk > n2) continue;
        const cd cc = c[di + 1][dk + 1];
        if (cc.re == 0.0 && cc.im == 0.0) continue;
        cfma(ax, cvt<Ta>(cc), ld<Ta>(x, (size_t)(ii - 1) * n2 + (kk - 1)));
      }
    }
  }
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
  const cx<Ta> dinv = cvt<Ta>(cinv(c[1][1]));
  cx<Ta> out = (x != nullptr) ? ld<Ta>(x, id) : mk<Ta>(0, 0);
  cfma(out, cvt<Ta>(mk<double>(w, 0.0)) * dinv, r);
  y[id] = cvt<Ty>(out);
}

}  // namespace

template <class Ta, class Tx, class Tb, class Ty>
void launch_stencil(const LevelDev& L, int mode, const cx<Tx>* x, const cx<Tb>* b, cx<Ty>* y,
                    double w, hipStream_t s, int nb, BIdx bx, BIdx bb, BIdx by) {
  if (nb < 1) return;
  dim3 blk(256);
  dim3 grd((L.n2 + 255) / 256, L.n1, nb);
  hipLaunchKernelGGL((k_stencil<Ta, Tx, Tb, Ty>), grd, blk, 0, s, L, mode, x, b, y, w, bx, bb, by);
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
#undef INST

}  // namespace hsp
