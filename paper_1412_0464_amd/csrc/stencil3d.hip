// Three-dimensional level kernels: the 7-point PML operator of the fine
// level and the 27-point finite-element operator of the coarse level
// (application, residual, omega-Jacobi step), the tensor-product transfers
// of the two-grid cycle, the right-hand-side scaling and the coarse medium
// (cell k^2 and Table (b) coefficients).
//
// The operators are matrix-free: every thread forms the coefficients of its
// node from the per-axis PML arrays and the medium (coefs27).  Threads run
// over the nodes in memory order (z fastest), so the x and y neighbours of a
// block's nodes are the same planes for every thread and stay in L2.
#include <algorithm>
#include <cmath>

#include "d3.h"

namespace hsp {
namespace d3 {

namespace {

inline int nblk(size_t n, int t = 256) { return (int)std::min<size_t>((n + t - 1) / t, (size_t)1 << 20); }

template <int KIND, class Ta, class Tx, class Tb, class Ty>
__global__ void __launch_bounds__(256) k_stencil3(Level3 L, int mode, const cx<Tx>* __restrict__ x,
                                                  const cx<Tb>* __restrict__ b, cx<Ty>* __restrict__ y, double w) {
  const size_t n = (size_t)L.m1 * L.m2 * L.m3;
  const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int k = (int)(id % L.m3) + 1;
  const size_t rest = id / L.m3;
  const int j = (int)(rest % L.m2) + 1;
  const int i = (int)(rest / L.m2) + 1;
  const size_t sy = L.m3, sx = (size_t)L.m2 * L.m3;
  cx<Ta> acc = mk<Ta>(0, 0);
  cx<Ta> diag;
  if (KIND == 7) {
    const int row = L.xmap ? L.xmap[i - 1] : (i - 1);
    const double k2 = L.k2[((size_t)row * L.m2 + (j - 1)) * L.m3 + (k - 1)];
    const cd ix = L.B[0][i], iy = L.B[1][j], iz = L.B[2][k];
    const double h = L.hs;
    const cd tx = h * (iy * iz), ty = h * (ix * iz), tz = h * (ix * iy);
    const cd xl = -(L.A[0][i - 1] * tx), xr = -(L.A[0][i] * tx);
    const cd yl = -(L.A[1][j - 1] * ty), yr = -(L.A[1][j] * ty);
    const cd zl = -(L.A[2][k - 1] * tz), zr = -(L.A[2][k] * tz);
    diag = cvt<Ta>(-(xl + xr + yl + yr + zl + zr) - (h * h * h * k2) * (ix * (iy * iz)));
    if (x) {
      if (i > 1) cfma(acc, cvt<Ta>(xl), cvt<Ta>(x[id - sx]));
      if (i < L.m1) cfma(acc, cvt<Ta>(xr), cvt<Ta>(x[id + sx]));
      if (j > 1) cfma(acc, cvt<Ta>(yl), cvt<Ta>(x[id - sy]));
      if (j < L.m2) cfma(acc, cvt<Ta>(yr), cvt<Ta>(x[id + sy]));
      if (k > 1) cfma(acc, cvt<Ta>(zl), cvt<Ta>(x[id - 1]));
      if (k < L.m3) cfma(acc, cvt<Ta>(zr), cvt<Ta>(x[id + 1]));
      cfma(acc, diag, cvt<Ta>(x[id]));
    }
  } else {
    cd c[27];
    coefs27(L, i, j, k, c);
    diag = cvt<Ta>(c[13]);
    if (x) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (i + dx < 1 || i + dx > L.m1) continue;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          if (j + dy < 1 || j + dy > L.m2) continue;
#pragma unroll
          for (int dz = -1; dz <= 1; ++dz) {
            if (k + dz < 1 || k + dz > L.m3) continue;
            const long o = (long)dx * (long)sx + (long)dy * (long)sy + dz;
            cfma(acc, cvt<Ta>(c[(dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)]), cvt<Ta>(x[(long)id + o]));
          }
        }
      }
    }
  }
  if (mode == 0) {
    y[id] = cvt<Ty>(acc);
    return;
  }
  const cx<Ta> r = cvt<Ta>(b[id]) - acc;
  if (mode == 1) {
    y[id] = cvt<Ty>(r);
    return;
  }
  const cx<Ta> xv = x ? cvt<Ta>(x[id]) : mk<Ta>(0, 0);
  const cx<Ta> d = cinv(diag) * r;
  y[id] = cvt<Ty>(mk<Ta>(xv.re + Ta(w) * d.re, xv.im + Ta(w) * d.im));
}

// r_c(I, J, K) = sum over the 3 x 3 x 3 taps of the restriction weights
template <class Tin, class Tout>
__global__ void __launch_bounds__(256) k_restrict3(Transfer3 T, const cx<Tin>* __restrict__ rf,
                                                   cx<Tout>* __restrict__ rc) {
  const size_t n = (size_t)T.nc[0] * T.nc[1] * T.nc[2];
  const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int K = (int)(id % T.nc[2]);
  const size_t rest = id / T.nc[2];
  const int J = (int)(rest % T.nc[1]);
  const int I = (int)(rest / T.nc[1]);
  cd acc = mk<double>(0, 0);
  for (int a = 0; a < 3; ++a) {
    const int fi = T.r[0][3 * I + a];
    if (fi < 0) continue;
    const double wa = T.rw[0][3 * I + a];
    for (int bq = 0; bq < 3; ++bq) {
      const int fj = T.r[1][3 * J + bq];
      if (fj < 0) continue;
      const double wab = wa * T.rw[1][3 * J + bq];
      const size_t base = ((size_t)fi * T.nf[1] + fj) * T.nf[2];
      for (int c = 0; c < 3; ++c) {
        const int fk = T.r[2][3 * K + c];
        if (fk < 0) continue;
        const cd v = cvt<double>(rf[base + fk]);
        const double ww = wab * T.rw[2][3 * K + c];
        acc.re += ww * v.re;
        acc.im += ww * v.im;
      }
    }
  }
  rc[id] = cvt<Tout>(acc);
}

// x_f(i, j, k) += sum over the (up to) 2 x 2 x 2 coarse taps
template <class Tc, class Tf>
__global__ void __launch_bounds__(256) k_prolong_add3(Transfer3 T, const cx<Tc>* __restrict__ ec,
                                                      cx<Tf>* __restrict__ xf) {
  const size_t n = (size_t)T.nf[0] * T.nf[1] * T.nf[2];
  const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int k = (int)(id % T.nf[2]);
  const size_t rest = id / T.nf[2];
  const int j = (int)(rest % T.nf[1]);
  const int i = (int)(rest / T.nf[1]);
  cd acc = mk<double>(0, 0);
  for (int a = 0; a < 2; ++a) {
    const int ci = T.p[0][2 * i + a];
    if (ci < 0) continue;
    const double wa = T.pw[0][2 * i + a];
    for (int bq = 0; bq < 2; ++bq) {
      const int cj = T.p[1][2 * j + bq];
      if (cj < 0) continue;
      const double wab = wa * T.pw[1][2 * j + bq];
      const size_t base = ((size_t)ci * T.nc[1] + cj) * T.nc[2];
      for (int c = 0; c < 2; ++c) {
        const int ck = T.p[2][2 * k + c];
        if (ck < 0) continue;
        const cd v = cvt<double>(ec[base + ck]);
        const double ww = wab * T.pw[2][2 * k + c];
        acc.re += ww * v.re;
        acc.im += ww * v.im;
      }
    }
  }
  const cd o = cvt<double>(xf[id]);
  xf[id] = cvt<Tf>(mk<double>(o.re + acc.re, o.im + acc.im));
}

__global__ void __launch_bounds__(256) k_rhs3(int m1, int m2, int m3, double h3, const cd* __restrict__ ib0,
                                              const cd* __restrict__ ib1, const cd* __restrict__ ib2,
                                              const cd* __restrict__ f, cd* __restrict__ b) {
  const size_t n = (size_t)m1 * m2 * m3;
  const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int k = (int)(id % m3);
  const size_t rest = id / m3;
  const int j = (int)(rest % m2);
  const int i = (int)(rest / m2);
  b[id] = h3 * (f[id] * (ib0[i + 1] * (ib1[j + 1] * ib2[k + 1])));
}

struct Avg3 {
  int m[3], nc[3];
  const int* x0[3];
  const double* w[3];
};

__global__ void __launch_bounds__(256) k_cell_average3(const double* __restrict__ k2n, Avg3 A,
                                                       double* __restrict__ k2c) {
  const size_t n = (size_t)A.nc[0] * A.nc[1] * A.nc[2];
  const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int r = (int)(id % A.nc[2]);
  const size_t rest = id / A.nc[2];
  const int q = (int)(rest % A.nc[1]);
  const int p = (int)(rest / A.nc[1]);
  double acc = 0;
  for (int a = 0; a < 3; ++a) {
    const double wa = A.w[0][3 * p + a];
    if (wa == 0.0) continue;
    int gi = A.x0[0][p] + a;  // node 0..m+1; Dirichlet nodes take the edge value
    gi = gi < 1 ? 1 : (gi > A.m[0] ? A.m[0] : gi);
    for (int bq = 0; bq < 3; ++bq) {
      const double wb = A.w[1][3 * q + bq];
      if (wb == 0.0) continue;
      int gj = A.x0[1][q] + bq;
      gj = gj < 1 ? 1 : (gj > A.m[1] ? A.m[1] : gj);
      for (int c = 0; c < 3; ++c) {
        const double wc = A.w[2][3 * r + c];
        if (wc == 0.0) continue;
        int gk = A.x0[2][r] + c;
        gk = gk < 1 ? 1 : (gk > A.m[2] ? A.m[2] : gk);
        acc += wa * wb * wc * k2n[((size_t)(gi - 1) * A.m[1] + (gj - 1)) * A.m[2] + (gk - 1)];
      }
    }
  }
  k2c[id] = acc;
}

// Optimized coefficients of the 27-point scheme (App. A, Table (b)): c_1..c_5
// at the support points 1/G_k = 0, 0.04, ..., 0.40.
__constant__ double kOptTable3D[11][5] = {
    {0.56428, 0.35970, 0.20490, 0.77998, 0.17505}, {0.56571, 0.36071, 0.20541, 0.78635, 0.17442},
    {0.56298, 0.36150, 0.20719, 0.78273, 0.16881}, {0.56540, 0.35620, 0.20287, 0.76438, 0.18678},
    {0.56370, 0.35299, 0.20299, 0.74684, 0.19603}, {0.55813, 0.35277, 0.20452, 0.72755, 0.20131},
    {0.54673, 0.35830, 0.20693, 0.70298, 0.20847}, {0.52423, 0.38368, 0.19633, 0.66863, 0.22424},
    {0.49946, 0.39740, 0.20725, 0.62734, 0.23845}, {0.47567, 0.40216, 0.22132, 0.58198, 0.25329},
    {0.45011, 0.36784, 0.29962, 0.53417, 0.23589}};

__global__ void k_cell_coefs3(const double* __restrict__ k2c, size_t n, double h_nom, double* __restrict__ coef) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    // 1/G = h k / (2 pi), clamped to the table range, linear interpolation
    double g = h_nom * sqrt(k2c[i]) * (0.5 / M_PI);
    g = fmin(fmax(g, 0.0), 0.40);
    const double s = g / 0.04;
    int j = (int)floor(s);
    if (j > 9) j = 9;
    const double t = s - j;
    for (int c = 0; c < 5; ++c) coef[5 * i + c] = (1.0 - t) * kOptTable3D[j][c] + t * kOptTable3D[j + 1][c];
  }
}

}  // namespace

template <class Ta, class Tx, class Tb, class Ty>
void launch_stencil3(const Level3& L, int mode, const cx<Tx>* x, const cx<Tb>* b, cx<Ty>* y, double w,
                     hipStream_t s) {
  const size_t n = (size_t)L.m1 * L.m2 * L.m3;
  if (n == 0) return;
  if (L.kind == 7)
    hipLaunchKernelGGL((k_stencil3<7, Ta, Tx, Tb, Ty>), dim3(nblk(n)), dim3(256), 0, s, L, mode, x, b, y, w);
  else
    hipLaunchKernelGGL((k_stencil3<27, Ta, Tx, Tb, Ty>), dim3(nblk(n)), dim3(256), 0, s, L, mode, x, b, y, w);
}

template <class Tin, class Tout>
void launch_restrict3(const Transfer3& T, const cx<Tin>* rf, cx<Tout>* rc, hipStream_t s) {
  const size_t n = (size_t)T.nc[0] * T.nc[1] * T.nc[2];
  hipLaunchKernelGGL((k_restrict3<Tin, Tout>), dim3(nblk(n)), dim3(256), 0, s, T, rf, rc);
}

template <class Tc, class Tf>
void launch_prolong_add3(const Transfer3& T, const cx<Tc>* ec, cx<Tf>* xf, hipStream_t s) {
  const size_t n = (size_t)T.nf[0] * T.nf[1] * T.nf[2];
  hipLaunchKernelGGL((k_prolong_add3<Tc, Tf>), dim3(nblk(n)), dim3(256), 0, s, T, ec, xf);
}

void launch_rhs3(int m1, int m2, int m3, double h3, const cd* ib0, const cd* ib1, const cd* ib2, const cd* f, cd* b,
                 hipStream_t s) {
  const size_t n = (size_t)m1 * m2 * m3;
  hipLaunchKernelGGL(k_rhs3, dim3(nblk(n)), dim3(256), 0, s, m1, m2, m3, h3, ib0, ib1, ib2, f, b);
}

void launch_cell_average3(const double* k2n, const int m[3], const int* x0[3], const double* w[3], const int nc[3],
                          double* k2c, hipStream_t s) {
  Avg3 A;
  for (int a = 0; a < 3; ++a) {
    A.m[a] = m[a];
    A.nc[a] = nc[a];
    A.x0[a] = x0[a];
    A.w[a] = w[a];
  }
  const size_t n = (size_t)nc[0] * nc[1] * nc[2];
  hipLaunchKernelGGL(k_cell_average3, dim3(nblk(n)), dim3(256), 0, s, k2n, A, k2c);
}

void launch_cell_coefs3(const double* k2c, size_t ncell, double h_nom, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_coefs3, dim3(nblk(ncell)), dim3(256), 0, s, k2c, ncell, h_nom, coef);
}

#define INST_ST(Ta, Tx, Tb, Ty) \
  template void launch_stencil3<Ta, Tx, Tb, Ty>(const Level3&, int, const cx<Tx>*, const cx<Tb>*, cx<Ty>*, double, \
                                                hipStream_t);
INST_ST(double, double, double, double)
INST_ST(float, float, float, float)
INST_ST(float, float, double, float)
INST_ST(double, float, double, double)
INST_ST(float, float, double, double)
#undef INST_ST
template void launch_restrict3<double, double>(const Transfer3&, const cd*, cd*, hipStream_t);
template void launch_restrict3<double, float>(const Transfer3&, const cd*, cf*, hipStream_t);
template void launch_prolong_add3<double, double>(const Transfer3&, const cd*, cd*, hipStream_t);
template void launch_prolong_add3<float, float>(const Transfer3&, const cf*, cf*, hipStream_t);

}  // namespace d3
}  // namespace hsp
