// Grid transfers of the two-grid method with PML-aware coarsening (Sec. 4):
// tent prolongation P as a tensor product of 1-D maps and restriction
// R = P^T.  The 1-D maps are tabulated on the host (at most 3 fine nodes per
// coarse node for R, at most 2 coarse nodes per fine node for P); the
// kernels gather, so no atomics are needed.  Arithmetic in double.
#include "internal.h"

namespace hsp {

namespace {

template <class Tin, class Tout>
__global__ void __launch_bounds__(256) k_restrict(TransferDev T, const cx<Tin>* __restrict__ rf,
                                                  cx<Tout>* __restrict__ rc, BIdx bi, BIdx bo) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;  // coarse y unknown (0-based)
  const int I = blockIdx.y;                             // coarse x unknown
  if (K >= T.nc2) return;
  rf += bi.off(blockIdx.z);
  rc += bo.off(blockIdx.z);
  cd acc = mk<double>(0, 0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int fi = T.rx[3 * I + a];
    if (fi < 0) continue;
    const double wa = T.rwx[3 * I + a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int fk = T.ry[3 * K + b];
      if (fk < 0) continue;
      acc += (wa * T.rwy[3 * K + b]) * cvt<double>(rf[(size_t)fi * T.nf2 + fk]);
    }
  }
  rc[(size_t)I * T.nc2 + K] = cvt<Tout>(acc);
}

template <class Tc, class Tf>
__global__ void __launch_bounds__(256) k_prolong_add(TransferDev T, const cx<Tc>* __restrict__ ec,
                                                     cx<Tf>* __restrict__ xf, BIdx bi, BIdx bo) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // fine y unknown
  const int i = blockIdx.y;
  if (k >= T.nf2) return;
  ec += bi.off(blockIdx.z);
  xf += bo.off(blockIdx.z);
  cd acc = mk<double>(0, 0);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int ci = T.px[2 * i + a];
    if (ci < 0) continue;
    const double wa = T.pwx[2 * i + a];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int ck = T.py[2 * k + b];
      if (ck < 0) continue;
      acc += (wa * T.pwy[2 * k + b]) * cvt<double>(ec[(size_t)ci * T.nc2 + ck]);
    }
  }
  const size_t id = (size_t)i * T.nf2 + k;
  xf[id] = cvt<Tf>(cvt<double>(xf[id]) + acc);
}

}  // namespace

template <class Tin, class Tout>
void launch_restrict(const TransferDev& T, const cx<Tin>* rf, cx<Tout>* rc, hipStream_t s, int nb, BIdx bi,
                     BIdx bo) {
  if (nb < 1) return;
  dim3 grd((T.nc2 + 255) / 256, T.nc1, nb);
  hipLaunchKernelGGL((k_restrict<Tin, Tout>), grd, dim3(256), 0, s, T, rf, rc, bi, bo);
}
template <class Tc, class Tf>
void launch_prolong_add(const TransferDev& T, const cx<Tc>* ec, cx<Tf>* xf, hipStream_t s, int nb, BIdx bi,
                        BIdx bo) {
  if (nb < 1) return;
  dim3 grd((T.nf2 + 255) / 256, T.nf1, nb);
  hipLaunchKernelGGL((k_prolong_add<Tc, Tf>), grd, dim3(256), 0, s, T, ec, xf, bi, bo);
}

template void launch_restrict<double, double>(const TransferDev&, const cd*, cd*, hipStream_t, int, BIdx, BIdx);
template void launch_restrict<double, float>(const TransferDev&, const cd*, cf*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<double, double>(const TransferDev&, const cd*, cd*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<float, float>(const TransferDev&, const cf*, cf*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<float, double>(const TransferDev&, const cf*, cd*, hipStream_t, int, BIdx, BIdx);

}  // namespace hsp
