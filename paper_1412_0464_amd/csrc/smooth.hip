// Fused smoothing phases of the two-grid cycle (Sec. 4) on a 5-point fine
// level: the nu omega-Jacobi steps of a phase run inside one kernel on an
// LDS tile with a halo of nu nodes (each step shrinks the valid region by
// one node), so the vectors cross HBM once per phase instead of once per
// step.
//
//   pre:  x_1 = w D^{-1} r, x_{s+1} = x_s + w D^{-1} (r - A x_s), s < nu;
//         outputs x_nu and the fine residual r - A x_nu (complex128);
//   post: x_0 = x + P e_c (prolongation of the coarse correction), then nu
//         steps; output x_nu (complex64 or complex128).
//
// Complex64 smoother (the mixed-precision path): the coefficients are formed
// in complex64 from complex64 row / column factors and k^2 (w D^{-1} once per
// node and kept in LDS with r and the two iterates; the off-diagonals per
// step).  A step is written (1 - w) x + (w D^{-1}) (r - (A - D) x), so the
// diagonal itself is not kept.  The residual that starts the coarse-grid
// correction and the prolongation sums are in double, as in the separate
// kernels (stencil.hip, transfer.hip).
#include "internal.h"

namespace hsp {

namespace {

constexpr int kTX = 16;  // tile rows (x)
constexpr int kTY = 64;  // tile columns (y, the contiguous axis)
// Threads per workgroup: the LDS tile allows three workgroups per CU, so the
// pre-smoothing (few registers) runs 512 threads to keep more loads in
// flight; the post-smoothing (prolongation taps in registers) runs 256.
constexpr int kPreThreads = 512;
constexpr int kPostThreads = 256;

// Extended tile (tile + halo of NU nodes) of the complex64 smoother.
template <int NU>
struct SmoothTile {
  static constexpr int H = NU;
  static constexpr int EX = kTX + 2 * H, EY = kTY + 2 * H, NE = EX * EY;
};

// Row / column factors of the off-diagonal coefficients, complex64:
// west = -xA[i-1] yB[k], east = -xA[i] yB[k], south = -yA[k-1] xB[i],
// north = -yA[k] xB[i]; zero toward a Dirichlet boundary.
struct Axes5 {
  cf rAm[kTX + 8], rAp[kTX + 8], rB[kTX + 8];
  cf cAm[kTY + 8], cAp[kTY + 8], cB[kTY + 8];
};

__device__ __forceinline__ void load_axes(const LevelDev& L, int i0, int k0, int EX, int EY, Axes5& ax) {
  for (int t = threadIdx.x; t < EX; t += blockDim.x) {
    const int i = i0 + t;
    const bool ok = i >= 1 && i <= L.n1;
    const int ic = ok ? i : 1;
    ax.rAm[t] = cvt<float>(L.xA[ic - 1]);
    ax.rAp[t] = cvt<float>(L.xA[ic]);
    ax.rB[t] = cvt<float>(L.xB[ic]);
  }
  for (int t = threadIdx.x; t < EY; t += blockDim.x) {
    const int k = k0 + t;
    const bool ok = k >= 1 && k <= L.n2;
    const int kc = ok ? k : 1;
    ax.cAm[t] = cvt<float>(L.yA[kc - 1]);
    ax.cAp[t] = cvt<float>(L.yA[kc]);
    ax.cB[t] = cvt<float>(L.yB[kc]);
  }
}

__device__ __forceinline__ cf keepf(bool ok, cf v) { return mk<float>(ok ? v.re : 0.f, ok ? v.im : 0.f); }

// Off-diagonal part of A cur at tile node (ti, tk) (complex64).
template <int EY>
__device__ __forceinline__ cf offdiag5(const Axes5& ax, const cf* cur, int e, int ti, int tk, bool iw, bool ie,
                                       bool ks, bool kn) {
  const cf ian = ax.rB[ti], ikn = ax.cB[tk];
  const cf cw = keepf(iw, -(ax.rAm[ti] * ikn)), ce = keepf(ie, -(ax.rAp[ti] * ikn));
  const cf cs = keepf(ks, -(ax.cAm[tk] * ian)), cn = keepf(kn, -(ax.cAp[tk] * ian));
  cf a = mk<float>(0, 0);
  cfma(a, cw, cur[e - EY]);
  cfma(a, cs, cur[e - 1]);
  cfma(a, cn, cur[e + 1]);
  cfma(a, ce, cur[e + EY]);
  return a;
}

// One Jacobi step on the region of halo hs: nxt = cur + (w D^{-1}) (r - A cur)
// = (1 - w) cur + (w D^{-1}) (r - (A - D) cur), so that only w D^{-1} is kept
// per node.
template <int NU>
__device__ __forceinline__ void jacobi_region(const LevelDev& L, int i0, int k0, int hs, float omw, const cf* cur,
                                              cf* nxt, const cf* rr, const cf* dws, const Axes5& ax) {
  using S = SmoothTile<NU>;
  const int RX = S::EX - 2 * hs, RY = S::EY - 2 * hs;
  for (int idx = threadIdx.x; idx < RX * RY; idx += blockDim.x) {
    const int ti = hs + idx / RY, tk = hs + idx % RY;
    const int i = i0 + ti, k = k0 + tk;
    const int e = ti * S::EY + tk;
    const bool in = i >= 1 && i <= L.n1 && k >= 1 && k <= L.n2;
    const cf a = offdiag5<S::EY>(ax, cur, e, ti, tk, i > 1, i < L.n1, k > 1, k < L.n2);
    cf out = omw * cur[e];
    cfma(out, dws[e], rr[e] - a);
    nxt[e] = keepf(in, out);
  }
}

// Node data of the extended tile: r (complex64), the diagonal and w D^{-1}
// (formed in complex64 from the row / column factors and k^2).  All global
// loads of a thread are issued before any is used (one memory round trip for
// the whole tile); the axes must already be in LDS.
template <int NU, class TR, int NT>
struct NodeLoads {
  static constexpr int NI = (SmoothTile<NU>::NE + NT - 1) / NT;
  cx<TR> r[NI];
  double k2[NI];
};

template <int NU, class TR, int NT>
__device__ __forceinline__ void fetch_nodes(const LevelDev& L, int i0, int k0, const cx<TR>* r,
                                            NodeLoads<NU, TR, NT>& ld) {
  using S = SmoothTile<NU>;
#pragma unroll
  for (int q = 0; q < NodeLoads<NU, TR, NT>::NI; ++q) {
    const int idx = min((int)threadIdx.x + NT * q, S::NE - 1);
    const int i = i0 + idx / S::EY, k = k0 + idx % S::EY;
    const bool in = i >= 1 && i <= L.n1 && k >= 1 && k <= L.n2;
    const size_t g = in ? (size_t)(i - 1) * L.n2 + (k - 1) : 0;
    ld.r[q] = r[g];
    ld.k2[q] = L.k2[g];
  }
}

template <int NU, class TR, int NT>
__device__ __forceinline__ void store_nodes(const LevelDev& L, int i0, int k0, double w,
                                            const NodeLoads<NU, TR, NT>& ld, const Axes5& ax, cf* rr, cf* dws) {
  using S = SmoothTile<NU>;
  const cf wt = cvt<float>(mk<double>(w, 0.0));
  const float h2 = (float)L.h2;
#pragma unroll
  for (int q = 0; q < NodeLoads<NU, TR, NT>::NI; ++q) {
    const int idx = (int)threadIdx.x + NT * q;
    if (idx >= S::NE) break;
    const int ti = idx / S::EY, tk = idx % S::EY;
    const int i = i0 + ti, k = k0 + tk;
    const bool in = i >= 1 && i <= L.n1 && k >= 1 && k <= L.n2;
    const cf ian = ax.rB[ti], ikn = ax.cB[tk];
    const cf cw = -(ax.rAm[ti] * ikn), ce = -(ax.rAp[ti] * ikn);
    const cf cs = -(ax.cAm[tk] * ian), cn = -(ax.cAp[tk] * ian);
    const cf c11 = -(cw + ce + cs + cn) - (h2 * (float)ld.k2[q]) * (ian * ikn);
    rr[idx] = keepf(in, cvt<float>(ld.r[q]));
    dws[idx] = wt * cinv(c11);
  }
}

template <int NU, class TR>
__global__ void __launch_bounds__(kPreThreads) k_smooth_pre(LevelDev L, double w, const cx<TR>* __restrict__ r, BIdx br,
                                                    cf* __restrict__ xo, BIdx bxo, cd* __restrict__ res, BIdx bres) {
  using S = SmoothTile<NU>;
  constexpr int EY = S::EY, NE = S::NE, H = S::H;
  __shared__ cf xa[NE], xb[NE], rr[NE], dws[NE];
  __shared__ Axes5 ax;
  const int n1 = L.n1, n2 = L.n2;
  const int i0 = blockIdx.y * kTX + 1 - H, k0 = blockIdx.x * kTY + 1 - H;
  const int z = blockIdx.z;
  const float omw = (float)(1.0 - w);
  r += br.off(z);
  xo += bxo.off(z);
  res += bres.off(z);
  constexpr int NT = kPreThreads;
  NodeLoads<NU, TR, NT> ld;
  fetch_nodes<NU, TR, NT>(L, i0, k0, r, ld);
  load_axes(L, i0, k0, S::EX, EY, ax);
  __syncthreads();
  store_nodes<NU, TR, NT>(L, i0, k0, w, ld, ax, rr, dws);
  __syncthreads();
  // x_1 = (w D^{-1}) r
  for (int idx = threadIdx.x; idx < NE; idx += blockDim.x) {
    cf out = mk<float>(0, 0);
    cfma(out, dws[idx], rr[idx]);
    xa[idx] = out;
  }
  __syncthreads();
  cf* cur = xa;
  cf* nxt = xb;
  for (int s = 2; s <= NU; ++s) {
    jacobi_region<NU>(L, i0, k0, s - 1, omw, cur, nxt, rr, dws, ax);
    __syncthreads();
    cf* t = cur;
    cur = nxt;
    nxt = t;
  }
  // x_nu and the residual r - A x_nu in double (stencil_coefs arithmetic:
  // the coarse-grid correction starts from a complex128 residual).  Each
  // thread takes the interior nodes among the ones it fetched, so r and k^2
  // come from its registers rather than a second read.
#pragma unroll
  for (int q = 0; q < NodeLoads<NU, TR, NT>::NI; ++q) {
    const int e = (int)threadIdx.x + NT * q;
    if (e >= NE) break;
    const int ti = e / EY, tk = e - (e / EY) * EY;
    if (ti < H || ti >= H + kTX || tk < H || tk >= H + kTY) continue;
    const int i = i0 + ti, k = k0 + tk;
    if (i > n1 || k > n2) continue;
    const size_t g = (size_t)(i - 1) * n2 + (k - 1);
    const cd ian = L.xB[i], ikn = L.yB[k];
    const cd cw = -(L.xA[i - 1] * ikn), ce = -(L.xA[i] * ikn);
    const cd cs = -(L.yA[k - 1] * ian), cn = -(L.yA[k] * ian);
    const cd c11 = -(cw + ce + cs + cn) - (L.h2 * ld.k2[q]) * (ian * ikn);
    cd a = mk<double>(0, 0);
    if (i > 1) cfma(a, cw, cvt<double>(cur[e - EY]));
    if (k > 1) cfma(a, cs, cvt<double>(cur[e - 1]));
    cfma(a, c11, cvt<double>(cur[e]));
    if (k < n2) cfma(a, cn, cvt<double>(cur[e + 1]));
    if (i < n1) cfma(a, ce, cvt<double>(cur[e + EY]));
    xo[g] = cur[e];
    res[g] = cvt<double>(ld.r[q]) - a;
  }
}

template <int NU, class TR, class TZ>
__global__ void __launch_bounds__(kPostThreads) k_smooth_post(LevelDev L, TransferDev Tr, double w, const cx<TR>* __restrict__ r,
                                                     BIdx br, const cf* __restrict__ xin, BIdx bxin,
                                                     const cf* __restrict__ ec, BIdx bec, cx<TZ>* __restrict__ zo,
                                                     BIdx bzo) {
  using S = SmoothTile<NU>;
  constexpr int EY = S::EY, NE = S::NE, H = S::H;
  __shared__ cf xa[NE], xb[NE], rr[NE], dws[NE];
  __shared__ Axes5 ax;
  const int n1 = L.n1, n2 = L.n2;
  const int i0 = blockIdx.y * kTX + 1 - H, k0 = blockIdx.x * kTY + 1 - H;
  const int z = blockIdx.z;
  const float omw = (float)(1.0 - w);
  r += br.off(z);
  xin += bxin.off(z);
  ec += bec.off(z);
  zo += bzo.off(z);
  constexpr int NT = kPostThreads;
  NodeLoads<NU, TR, NT> ld;
  fetch_nodes<NU, TR, NT>(L, i0, k0, r, ld);
  // x_0 = x + P e_c (prolongation sums in double, as k_prolong_add).  The
  // taps are separable (rows times columns): the row and column taps of the
  // tile are staged in LDS with the axes, then every node issues its four
  // coarse loads.  (The tent weights are 0, 1/2 and 1: exact in float.)
  constexpr int NI = NodeLoads<NU, TR, NT>::NI;
  __shared__ int tpi[2][S::EX], tpk[2][EY];
  __shared__ float twi[2][S::EX], twk[2][EY];
  for (int t = threadIdx.x; t < S::EX + EY; t += blockDim.x) {
    const bool row = t < S::EX;
    const int tt = row ? t : t - S::EX;
    const int g = row ? i0 + tt : k0 + tt;
    const int ng = row ? n1 : n2;
    const int gc = (g >= 1 && g <= ng) ? g - 1 : 0;  // 0-based fine index
    const int* pi = row ? Tr.px : Tr.py;
    const double* pw = row ? Tr.pwx : Tr.pwy;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int ci = max(pi[2 * gc + a], 0);
      const float wa = (float)pw[2 * gc + a];
      if (row) {
        tpi[a][tt] = ci;
        twi[a][tt] = wa;
      } else {
        tpk[a][tt] = ci;
        twk[a][tt] = wa;
      }
    }
  }
  load_axes(L, i0, k0, S::EX, EY, ax);
  __syncthreads();
  cf x0[NI], v[NI][2][2];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int idx = min((int)threadIdx.x + NT * q, NE - 1);
    const int ti = idx / EY, tk = idx - (idx / EY) * EY;
    const int i = i0 + ti, k = k0 + tk;
    const bool in = i >= 1 && i <= n1 && k >= 1 && k <= n2;
    x0[q] = xin[in ? (size_t)(i - 1) * n2 + (k - 1) : 0];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) v[q][a][b] = ec[(size_t)tpi[a][ti] * Tr.nc2 + tpk[b][tk]];
  }
  store_nodes<NU, TR, NT>(L, i0, k0, w, ld, ax, rr, dws);
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int idx = (int)threadIdx.x + NT * q;
    if (idx >= NE) break;
    const int ti = idx / EY, tk = idx - (idx / EY) * EY;
    const int i = i0 + ti, k = k0 + tk;
    const bool in = i >= 1 && i <= n1 && k >= 1 && k <= n2;
    cd acc = mk<double>(0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc += (double)(twi[a][ti] * twk[b][tk]) * cvt<double>(v[q][a][b]);
    xa[idx] = keepf(in, cvt<float>(cvt<double>(x0[q]) + acc));
  }
  __syncthreads();
  cf* cur = xa;
  cf* nxt = xb;
  for (int s = 1; s < NU; ++s) {
    jacobi_region<NU>(L, i0, k0, s, omw, cur, nxt, rr, dws, ax);
    __syncthreads();
    cf* t = cur;
    cur = nxt;
    nxt = t;
  }
  // the last step on the tile, written out in TZ
  for (int idx = threadIdx.x; idx < kTX * kTY; idx += blockDim.x) {
    const int ti = H + idx / kTY, tk = H + idx % kTY;
    const int i = i0 + ti, k = k0 + tk;
    if (i > n1 || k > n2) continue;
    const int e = ti * EY + tk;
    const cf a = offdiag5<EY>(ax, cur, e, ti, tk, i > 1, i < n1, k > 1, k < n2);
    cf out = omw * cur[e];
    cfma(out, dws[e], rr[e] - a);
    zo[(size_t)(i - 1) * n2 + (k - 1)] = cvt<TZ>(out);
  }
}

}  // namespace

// (the fused kernels hold a real k^2 per node: no sponge layers)
bool smooth_fused_ok(const LevelDev& L, int nu) {
  return L.kind == 5 && L.xmap == nullptr && L.k2i == nullptr && nu >= 1 && nu <= 3;
}

template <class TR>
void launch_smooth_pre(const LevelDev& L, int nu, double w, const cx<TR>* r, BIdx br, cf* xo, BIdx bxo, cd* res,
                       BIdx bres, int nb, hipStream_t s) {
  if (nb < 1) return;
  const dim3 grd((L.n2 + kTY - 1) / kTY, (L.n1 + kTX - 1) / kTX, nb);
  switch (nu) {
    case 1: hipLaunchKernelGGL((k_smooth_pre<1, TR>), grd, dim3(kPreThreads), 0, s, L, w, r, br, xo, bxo, res, bres); break;
    case 2: hipLaunchKernelGGL((k_smooth_pre<2, TR>), grd, dim3(kPreThreads), 0, s, L, w, r, br, xo, bxo, res, bres); break;
    default: hipLaunchKernelGGL((k_smooth_pre<3, TR>), grd, dim3(kPreThreads), 0, s, L, w, r, br, xo, bxo, res, bres); break;
  }
}

template <class TR, class TZ>
void launch_smooth_post(const LevelDev& L, const TransferDev& Tr, int nu, double w, const cx<TR>* r, BIdx br,
                        const cf* xin, BIdx bxin, const cf* ec, BIdx bec, cx<TZ>* zo, BIdx bzo, int nb, hipStream_t s) {
  if (nb < 1) return;
  const dim3 grd((L.n2 + kTY - 1) / kTY, (L.n1 + kTX - 1) / kTX, nb);
  switch (nu) {
    case 1:
      hipLaunchKernelGGL((k_smooth_post<1, TR, TZ>), grd, dim3(kPostThreads), 0, s, L, Tr, w, r, br, xin, bxin, ec, bec, zo,
                         bzo);
      break;
    case 2:
      hipLaunchKernelGGL((k_smooth_post<2, TR, TZ>), grd, dim3(kPostThreads), 0, s, L, Tr, w, r, br, xin, bxin, ec, bec, zo,
                         bzo);
      break;
    default:
      hipLaunchKernelGGL((k_smooth_post<3, TR, TZ>), grd, dim3(kPostThreads), 0, s, L, Tr, w, r, br, xin, bxin, ec, bec, zo,
                         bzo);
      break;
  }
}

#define INST(TR)                                                                                                \
  template void launch_smooth_pre<TR>(const LevelDev&, int, double, const cx<TR>*, BIdx, cf*, BIdx, cd*, BIdx,  \
                                      int, hipStream_t);
INST(double)
INST(float)
#undef INST
#define INST(TR, TZ)                                                                                               \
  template void launch_smooth_post<TR, TZ>(const LevelDev&, const TransferDev&, int, double, const cx<TR>*, BIdx, \
                                           const cf*, BIdx, const cf*, BIdx, cx<TZ>*, BIdx, int, hipStream_t);
INST(double, double)
INST(double, float)
INST(float, double)
INST(float, float)
#undef INST

}  // namespace hsp
