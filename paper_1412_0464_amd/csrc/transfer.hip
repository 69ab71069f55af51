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
  // all taps loaded unconditionally: a missing tap (index -1) has weight 0
  // and reads row / column 0 instead
  int fi[3], fk[3];
  double wi[3], wk[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    fi[a] = max(T.rx[3 * I + a], 0);
    wi[a] = T.rwx[3 * I + a];
    fk[a] = max(T.ry[3 * K + a], 0);
    wk[a] = T.rwy[3 * K + a];
  }
  cx<Tin> v[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) v[a][b] = rf[(size_t)fi[a] * T.nf2 + fk[b]];
  cd acc = mk<double>(0, 0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc += (wi[a] * wk[b]) * cvt<double>(v[a][b]);
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
  // all taps loaded unconditionally: a missing tap (index -1) has weight 0
  // and reads row / column 0 instead
  int ci[2], ck[2];
  double wi[2], wk[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    ci[a] = max(T.px[2 * i + a], 0);
    wi[a] = T.pwx[2 * i + a];
    ck[a] = max(T.py[2 * k + a], 0);
    wk[a] = T.pwy[2 * k + a];
  }
  const size_t id = (size_t)i * T.nf2 + k;
  cx<Tc> v[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) v[a][b] = ec[(size_t)ci[a] * T.nc2 + ck[b]];
  const cx<Tf> x0 = xf[id];
  cd acc = mk<double>(0, 0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc += (wi[a] * wk[b]) * cvt<double>(v[a][b]);
  xf[id] = cvt<Tf>(cvt<double>(x0) + acc);
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
template void launch_restrict<float, float>(const TransferDev&, const cf*, cf*, hipStream_t, int, BIdx, BIdx);
template void launch_restrict<float, double>(const TransferDev&, const cf*, cd*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<double, double>(const TransferDev&, const cd*, cd*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<float, float>(const TransferDev&, const cf*, cf*, hipStream_t, int, BIdx, BIdx);
template void launch_prolong_add<float, double>(const TransferDev&, const cf*, cd*, hipStream_t, int, BIdx, BIdx);

}  // namespace hsp
