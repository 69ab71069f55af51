// Device-side building blocks shared by the HIP kernels of the library:
// complex arithmetic, the level view (a compact-stencil Helmholtz operator on
// a rectilinear mesh with PML) and its per-node stencil coefficients.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace hsp {

// ---------------------------------------------------------------------------
// Interleaved complex number.
// ---------------------------------------------------------------------------
template <class R>
struct __align__(2 * sizeof(R)) cx {
  R re, im;
};

template <class R>
__host__ __device__ __forceinline__ cx<R> mk(R re, R im) {
  cx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <class R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <class R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <class R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return mk<R>(-a.re, -a.im); }
template <class R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return mk<R>(s * a.re, s * a.im); }
template <class R>
__host__ __device__ __forceinline__ cx<R>& operator+=(cx<R>& a, cx<R> b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
template <class R>
__host__ __device__ __forceinline__ cx<R>& operator-=(cx<R>& a, cx<R> b) {
  a.re -= b.re;
  a.im -= b.im;
  return a;
}
// acc += a * b
template <class R>
__host__ __device__ __forceinline__ void cfma(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <class R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return mk<R>(a.re, -a.im); }
template <class R>
__host__ __device__ __forceinline__ R abs2(cx<R> a) { return a.re * a.re + a.im * a.im; }
template <class R>
__host__ __device__ __forceinline__ cx<R> cinv(cx<R> a) {
  R d = R(1) / (a.re * a.re + a.im * a.im);
  return mk<R>(a.re * d, -a.im * d);
}
template <class To, class From>
__host__ __device__ __forceinline__ cx<To> cvt(cx<From> a) { return mk<To>(To(a.re), To(a.im)); }

using cd = cx<double>;
using cf = cx<float>;

// ---------------------------------------------------------------------------
// Level view: a compact-stencil Helmholtz operator on an n1 x n2 grid of
// unknown nodes (x slowest).  Two kinds:
//
//  kind 5 - 5-point PML finite differences (eq. define_pml_fd), FE scaled:
//    xA[p]  = alpha_1 at half node p + 1/2      (p = 0..n1)
//    xB[i]  = 1 / alpha_1 at node i             (i = 0..n1+1)
//    yA, yB likewise along y; k2 at unknown nodes, row stride n2.
//
//  kind 9 - finite-element form of the compact 9-point operator (App. A):
//    xA[p]  = alpha_1 / h_1 of cell p (between nodes p and p+1), p = 0..n1
//    xB[p]  = h_1 / alpha_1 of cell p
//    yA, yB likewise; k2 and coef (c1, c2, c3) per cell, row stride n2+1.
//
// xmap (optional) maps the view's own x row (node i-1 for kind 5, cell p
// for kind 9) to the row of k2 / coef; it lets a slab reuse the global
// medium arrays with the k continuation of its added layers.
// k2i (optional, same layout as k2): imaginary part of k^2 - the sponge
// layers of Sec. 2.1 replace k by k (1 + i beta).
// ---------------------------------------------------------------------------
struct LevelDev {
  int kind;
  int n1, n2;
  double h2;  // h^2 (kind 5)
  const cd* xA;
  const cd* xB;
  const cd* yA;
  const cd* yB;
  const double* k2;
  const double* coef;
  const int* xmap;
  const double* k2i;
};

// k^2 at entry idx of the medium arrays (complex inside sponge layers).
__device__ __forceinline__ cd k2_at(const LevelDev& L, size_t idx) {
  return mk<double>(L.k2[idx], L.k2i ? L.k2i[idx] : 0.0);
}

// Stencil coefficients of row (i, k) (1-based unknown node):
// c[di+1][dk+1] multiplies u(i+di, k+dk).  Always computed in double.
__device__ __forceinline__ void stencil_coefs(const LevelDev& L, int i, int k, cd c[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) c[a][b] = mk<double>(0.0, 0.0);
  if (L.kind == 5) {
    const int row = L.xmap ? L.xmap[i - 1] : (i - 1);
    const cd k2 = k2_at(L, (size_t)row * L.n2 + (k - 1));
    const cd ian = L.xB[i], ikn = L.yB[k];
    const cd w = -(L.xA[i - 1] * ikn), e = -(L.xA[i] * ikn);
    const cd s = -(L.yA[k - 1] * ian), n = -(L.yA[k] * ian);
    c[0][1] = w;
    c[2][1] = e;
    c[1][0] = s;
    c[1][2] = n;
    c[1][1] = -(w + e + s + n) - (L.h2 * k2) * (ian * ikn);
    return;
  }
  // kind 9: sum of the element matrices of the four cells around the node.
#pragma unroll
  for (int px = 0; px < 2; ++px) {
#pragma unroll
    for (int qy = 0; qy < 2; ++qy) {
      const int p = i - 1 + px, q = k - 1 + qy;  // cell indices
      const int ax = i - p, ay = k - q;          // corner of the node in the cell
      const int row = L.xmap ? L.xmap[p] : p;
      const size_t ci = (size_t)row * (L.n2 + 1) + q;
      const cd k2 = k2_at(L, ci);
      const double c1 = L.coef[3 * ci], c2 = L.coef[3 * ci + 1], c3 = L.coef[3 * ci + 2];
      const double I0 = 0.25 * c1, I1 = 0.125 * c2, I2 = 0.25 * (1.0 - c1 - c2);
      const double J0 = 0.5 * c3, J1 = 0.5 * (1.0 - c3);
      const cd xa = L.xA[p], xb = L.xB[p], ya = L.yA[q], yb = L.yB[q];
      const cd sx = xa * yb, sy = ya * xb, m = k2 * (xb * yb);
      cd e[2][2];
      e[0][0] = J0 * (sx + sy) - I0 * m;
      e[1][0] = J1 * sy - J0 * sx - I1 * m;
      e[0][1] = J1 * sx - J0 * sy - I1 * m;
      e[1][1] = -(J1 * (sx + sy)) - I2 * m;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          const int di = p + bx - i, dk = q + by - k;
          c[di + 1][dk + 1] += e[bx != ax][by != ay];
        }
    }
  }
}

}  // namespace hsp
