// Vector kernels: conversions, the fused Gram-Schmidt pieces of FGMRES
// (multi-dot, multi-axpy, normalisation), right-hand-side scaling and the
// per-node / per-cell medium preprocessing of the setup.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace hsp {

namespace {

template <class To, class Ti>
__global__ void k_convert(const cx<Ti>* __restrict__ in, cx<To>* __restrict__ out, size_t n, int cj, BIdx bi,
                          BIdx bo) {
  in += bi.off(blockIdx.y);
  out += bo.off(blockIdx.y);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    cx<To> v = cvt<To>(in[i]);
    if (cj) v.im = -v.im;
    out[i] = v;
  }
}

template <class T>
__global__ void k_zero(cx<T>* v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = mk<T>(0, 0);
}

__global__ void k_fill(cd* v, size_t n, cd value) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = value;
}

__device__ __forceinline__ cd block_sum(cd v, cd* sh) {
  // 256 threads
  const int t = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_down(v.re, off, 64);
    v.im += __shfl_down(v.im, off, 64);
  }
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  cd r = mk<double>(0, 0);
  if (t == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  return r;
}

__global__ void __launch_bounds__(256) k_multiaxpy(const cd* __restrict__ V, size_t ldv, int m,
                                                   const cd* __restrict__ h, cd* __restrict__ w, size_t n,
                                                   int sub) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    cd acc = mk<double>(0, 0);
    for (int j = 0; j < m; ++j) cfma(acc, h[j], V[(size_t)j * ldv + i]);
    w[i] = sub ? (w[i] - acc) : (w[i] + acc);
  }
}

__global__ void k_normalize(const cd* __restrict__ w, const cd* __restrict__ nrm2, cd* __restrict__ v, size_t n) {
  const double s = 1.0 / sqrt(nrm2[0].re);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = s * w[i];
}

__global__ void k_scale_rhs(int n1, int n2, double h2, const cd* __restrict__ ixn, const cd* __restrict__ iyn,
                            const cd* __restrict__ f, cd* __restrict__ b) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n2) return;
  const size_t id = (size_t)i * n2 + k;
  b[id] = h2 * ((ixn[i + 1] * iyn[k + 1]) * f[id]);
}

__global__ void __launch_bounds__(1024) k_stats(const double* __restrict__ c, size_t n, double* __restrict__ out) {
  __shared__ double s_sum[16], s_min[16], s_max[16], s_bad[16];
  double sum = 0, mn = INFINITY, mx = -INFINITY, bad = 0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = c[i];
    if (!(v > 0.0) || !isfinite(v)) {
      bad += 1;
      continue;
    }
    sum += v;
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_down(sum, off, 64);
    bad += __shfl_down(bad, off, 64);
    mn = fmin(mn, __shfl_down(mn, off, 64));
    mx = fmax(mx, __shfl_down(mx, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_sum[w] = sum;
    s_min[w] = mn;
    s_max[w] = mx;
    s_bad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      sum += s_sum[q];
      mn = fmin(mn, s_min[q]);
      mx = fmax(mx, s_max[q]);
      bad += s_bad[q];
    }
    out[0] = sum;
    out[1] = mn;
    out[2] = mx;
    out[3] = bad;
  }
}

__global__ void k_k2_nodes(const double* __restrict__ c, size_t n, double om2, double* __restrict__ k2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    k2[i] = om2 / (c[i] * c[i]);
}

__global__ void k_cell_average(const double* __restrict__ k2n, int n1, int n2, const int* __restrict__ x0,
                               const double* __restrict__ wx, const int* __restrict__ y0,
                               const double* __restrict__ wy, int nc2, double* __restrict__ k2c) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= nc2) return;
  double acc = 0;
  for (int a = 0; a < 3; ++a) {
    const double wa = wx[3 * p + a];
    if (wa == 0.0) continue;
    int gi = x0[p] + a;                       // node index 0..N1
    gi = gi < 1 ? 1 : (gi > n1 ? n1 : gi);    // edge value for Dirichlet nodes
    for (int b = 0; b < 3; ++b) {
      const double wb = wy[3 * q + b];
      if (wb == 0.0) continue;
      int gk = y0[q] + b;
      gk = gk < 1 ? 1 : (gk > n2 ? n2 : gk);
      acc += wa * wb * k2n[(size_t)(gi - 1) * n2 + (gk - 1)];
    }
  }
  k2c[(size_t)p * nc2 + q] = acc;
}

// Optimized finite-difference coefficients (App. A, Table (a)): 1/G_k and
// c_1, c_2, c_3 at the support points 1/G_k = 0, 0.04, ..., 0.40.
__constant__ double kOptTable2D[11][3] = {
    {0.61953, 0.45295, 0.77363}, {0.63691, 0.47535, 0.87242}, {0.62988, 0.48633, 0.86400},
    {0.62610, 0.48880, 0.84984}, {0.62289, 0.48759, 0.83017}, {0.62596, 0.47106, 0.80852},
    {0.62213, 0.46478, 0.78215}, {0.61036, 0.47016, 0.74857}, {0.59107, 0.48468, 0.70553},
    {0.56369, 0.50746, 0.65062}, {0.52412, 0.54163, 0.57676}};

__global__ void k_cell_coefs(const double* __restrict__ k2c, size_t n, double h_nom, double* __restrict__ coef) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    // 1/G = h k / (2 pi), clamped to the table range
    double g = h_nom * sqrt(k2c[i]) * (0.5 / M_PI);
    g = fmin(fmax(g, 0.0), 0.40);
    double s = g / 0.04;
    int j = (int)floor(s);
    if (j > 9) j = 9;
    const double t = s - j;
    for (int c = 0; c < 3; ++c) coef[3 * i + c] = (1.0 - t) * kOptTable2D[j][c] + t * kOptTable2D[j + 1][c];
  }
}

// Sponge layers (Sec. 2.1): k^2 -> k^2 (1 + i beta)^2 at the unknown nodes,
// beta = bx[i] + by[k]; k2 holds the real part on return, k2i the imaginary.
__global__ void k_sponge_k2(int n1, int n2, const double* __restrict__ bx, const double* __restrict__ by,
                            double* __restrict__ k2, double* __restrict__ k2i) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n2) return;
  const size_t id = (size_t)i * n2 + k;
  const double b = bx[i] + by[k], v = k2[id];
  k2[id] = v * (1.0 - b * b);
  k2i[id] = 2.0 * v * b;
}

__global__ void k_grad_m(int n1, int n2, double scale, const cd* __restrict__ ixn, const cd* __restrict__ iyn,
                         const cd* __restrict__ u, const cd* __restrict__ lam, double* __restrict__ g) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n2) return;
  const size_t id = (size_t)i * n2 + k;
  const cd w = conj(lam[id]) * (u[id] * (ixn[i + 1] * iyn[k + 1]));
  g[id] += scale * w.re;
}

// ---- batched Gram-Schmidt pieces: vector j of right-hand side z of a basis
// is V + bv.off(z) + j * ldj; blockIdx.z (or .y) selects z.
// Sum of NV complex values over the 256 threads of a block: thread q < NV
// returns the total of entry q.
template <int NV>
__device__ __forceinline__ cd block_sum_arr(cd (&v)[NV], cd* sh) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) {
      v[q].re += __shfl_xor(v[q].re, off, 64);
      v[q].im += __shfl_xor(v[q].im, off, 64);
    }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wv * NV + q] = v[q];
  __syncthreads();
  cd r = mk<double>(0, 0);
  if (t < NV)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w * NV + t];
  return r;
}

// Basis vectors j0 .. j0+kDotTile-1 (blockIdx.y tile) against w: w is read
// once per tile.
constexpr int kDotTile = 8;
constexpr int kUpdUnroll = 8;
constexpr int kDotElems = 2;  // elements per thread and iteration of k_bmultidot2
__global__ void __launch_bounds__(256) k_bmultidot(const cd* __restrict__ V, size_t ldj, BIdx bv, int cnt,
                                                   const cd* __restrict__ w, BIdx bw, size_t n,
                                                   cd* __restrict__ partial) {
  __shared__ cd sh[4 * kDotTile];
  const int z = blockIdx.z, j0 = blockIdx.y * kDotTile;
  const int jn = min(kDotTile, cnt - j0);
  const cd* v = V + bv.off(z) + (size_t)j0 * ldj;
  w += bw.off(z);
  cd acc[kDotTile];
#pragma unroll
  for (int q = 0; q < kDotTile; ++q) acc[q] = mk<double>(0, 0);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  if (jn == kDotTile) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
      const cd wi = w[i];
#pragma unroll
      for (int q = 0; q < kDotTile; ++q) cfma(acc[q], conj(v[(size_t)q * ldj + i]), wi);
    }
  } else {  // a partial tile: rows q >= jn repeat the last vector, never written out
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
      const cd wi = w[i];
#pragma unroll
      for (int q = 0; q < kDotTile; ++q) cfma(acc[q], conj(v[(size_t)(q < jn ? q : jn - 1) * ldj + i]), wi);
    }
  }
  const cd r = block_sum_arr<kDotTile>(acc, sh);
  if ((int)threadIdx.x < jn) partial[((size_t)z * cnt + j0 + threadIdx.x) * gridDim.x + blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_breduce(const cd* __restrict__ partial, int nb, int cnt,
                                                 cd* __restrict__ out, size_t ldo) {
  __shared__ cd sh[4];
  const int j = blockIdx.x, z = blockIdx.y;
  const cd* p = partial + ((size_t)z * cnt + j) * nb;
  cd acc = mk<double>(0, 0);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += p[b];
  cd r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(size_t)z * ldo + j] = r;
}

template <class TV>
__global__ void __launch_bounds__(256) k_bmultiaxpy(const cx<TV>* __restrict__ V, size_t ldj, BIdx bv, int cnt,
                                                    const cd* __restrict__ h, size_t ldh, cd* __restrict__ w,
                                                    BIdx bw, size_t n, int sub) {
  const int z = blockIdx.y;
  const cx<TV>* v = V + bv.off(z);
  const cd* hz = h + (size_t)z * ldh;
  w += bw.off(z);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    cd acc = mk<double>(0, 0);
    int j = 0;
    for (; j + kUpdUnroll <= cnt; j += kUpdUnroll) {  // kUpdUnroll loads in flight per step
      cx<TV> vq[kUpdUnroll];
#pragma unroll
      for (int q = 0; q < kUpdUnroll; ++q) vq[q] = v[(size_t)(j + q) * ldj + i];
#pragma unroll
      for (int q = 0; q < kUpdUnroll; ++q) cfma(acc, hz[j + q], cvt<double>(vq[q]));
    }
    for (; j < cnt; ++j) cfma(acc, hz[j], cvt<double>(v[(size_t)j * ldj + i]));
    w[i] = sub ? (w[i] - acc) : (w[i] + acc);
  }
}

// Delayed classical Gram-Schmidt, one projection pass: for basis vectors
// j < cnt of right-hand side z (slot cnt-1 holds the once-projected,
// unnormalised vector u), conj(V_zj) . u and conj(V_zj) . w; both read once.
// partial[((z 2 cnt) + q cnt + j) nblk + block], q = 0 (u) or 1 (w).  The
// basis is stored in TV (complex128, or complex64 for the mixed-precision
// solver); the products are formed in double.
template <class TV>
__global__ void __launch_bounds__(256) k_bmultidot2(const cx<TV>* __restrict__ V, size_t ldj, BIdx bv, int cnt,
                                                    const cd* __restrict__ w, BIdx bw, size_t n,
                                                    cd* __restrict__ partial) {
  __shared__ cd sh[4 * 2 * kDotTile];
  const int z = blockIdx.z, j0 = blockIdx.y * kDotTile;
  const int jn = min(kDotTile, cnt - j0);
  const cx<TV>* vz = V + bv.off(z);
  const cx<TV>* v = vz + (size_t)j0 * ldj;
  const cx<TV>* u = vz + (size_t)(cnt - 1) * ldj;
  w += bw.off(z);
  cd acc[2 * kDotTile];
#pragma unroll
  for (int q = 0; q < 2 * kDotTile; ++q) acc[q] = mk<double>(0, 0);
  // kDotElems elements per thread and iteration (blockDim apart, the last
  // clamped and weighted by zero); all loads of an iteration are
  // unconditional (rows q >= jn repeat the last vector of the tile and are
  // never written out), so that they are issued together rather than one
  // branch at a time
  constexpr int E = kDotElems;
  const size_t stride = (size_t)gridDim.x * blockDim.x * E;
  for (size_t i0 = blockIdx.x * (size_t)blockDim.x * E + threadIdx.x; i0 < n; i0 += stride) {
    cd ui[E], wi[E];
    cx<TV> vq[E][kDotTile];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t ie = i0 + (size_t)e * blockDim.x;
      const bool ok = ie < n;
      const size_t i = ok ? ie : n - 1;
      const cd uv = cvt<double>(u[i]), wv = w[i];
      ui[e] = mk<double>(ok ? uv.re : 0.0, ok ? uv.im : 0.0);
      wi[e] = mk<double>(ok ? wv.re : 0.0, ok ? wv.im : 0.0);
#pragma unroll
      for (int q = 0; q < kDotTile; ++q) vq[e][q] = v[(size_t)(q < jn ? q : jn - 1) * ldj + i];
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
      for (int q = 0; q < kDotTile; ++q) {
        const cd vj = conj(cvt<double>(vq[e][q]));
        cfma(acc[q], vj, ui[e]);
        cfma(acc[kDotTile + q], vj, wi[e]);
      }
  }
  const cd r = block_sum_arr<2 * kDotTile>(acc, sh);
  const int t = threadIdx.x;
  if (t < 2 * kDotTile) {
    const int q = t / kDotTile, jj = t - q * kDotTile;
    if (jj < jn) partial[(((size_t)z * 2 + q) * cnt + j0 + jj) * gridDim.x + blockIdx.x] = r;
  }
}

// Per right-hand side (one thread each) after k_bmultidot2 with cnt = k+1:
// d = hb + z ldh holds s_j = conj(v_j) . u (j < k), sigma = u . u (at k),
// then p_j = conj(v_j) . w (j < k) and pi = u . w (at cnt + k).  The
// reorthogonalised basis vector is v_k = (u - sum_j s_j v_j) / nu with
// nu^2 = sigma - |s|^2 (nu = 1 at k = 0, where u is already final), and
// h_kk = conj(v_k) . w = (pi - s^H p) / nu.  Writes nu and h_kk at d[off],
// d[off + 1].
__global__ void k_bdcgs_coef(cd* __restrict__ hb, size_t ldh, int k, int off, int nb) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nb) return;
  cd* d = hb + (size_t)z * ldh;
  const int cnt = k + 1;
  double ss = 0;
  cd sp = mk<double>(0, 0);
  for (int j = 0; j < k; ++j) {
    ss += abs2(d[j]);
    cfma(sp, conj(d[j]), d[cnt + j]);
  }
  double nu = 1.0;
  if (k > 0) nu = sqrt(fmax(d[k].re - ss, 1e-300));
  const cd pi = d[cnt + k];
  d[off] = mk<double>(nu, 0.0);
  d[off + 1] = mk<double>((pi.re - sp.re) / nu, (pi.im - sp.im) / nu);
}

// The update pass of the delayed Gram-Schmidt step: with s, p, nu, h_kk as
// above, v_k = (u - V s) / nu overwrites slot k and
// u' = w - V p - h_kk v_k (the next once-projected vector) goes to slot k+1,
// with the block partials of ||u'||^2.  Reads V (k vectors), u and w once.
// With a complex64 basis, v_k and u' are rounded before they are used, so
// that the recurrences see exactly the stored vectors.  Each thread takes
// kUpdElems elements per iteration (blockDim apart) so that more loads are in
// flight, and the two output vectors are written with non-temporal stores
// (no reuse before they are streamed again).
constexpr int kUpdElems = 2;
template <class T>
__device__ __forceinline__ void store_nt(cx<T>* p, cx<T> v) {
  __builtin_nontemporal_store(v.re, &p->re);
  __builtin_nontemporal_store(v.im, &p->im);
}
template <class TV>
__global__ void __launch_bounds__(256) k_bdcgs_update(cx<TV>* __restrict__ V, size_t ldj, BIdx bv, int k,
                                                      const cd* __restrict__ hb, size_t ldh, int off,
                                                      const cd* __restrict__ w, BIdx bw, size_t n,
                                                      cd* __restrict__ partial) {
  __shared__ cd sh[4];
  const int z = blockIdx.y;
  cx<TV>* vz = V + bv.off(z);
  const cd* d = hb + (size_t)z * ldh;
  const cd* sv = d;
  const cd* pv = d + (k + 1);
  const double inu = 1.0 / d[off].re;
  const cd hkk = d[off + 1];
  cx<TV>* u = vz + (size_t)k * ldj;
  cx<TV>* un = vz + (size_t)(k + 1) * ldj;
  w += bw.off(z);
  double nrm = 0;
  constexpr int E = kUpdElems;
  const size_t stride = (size_t)gridDim.x * blockDim.x * E;
  for (size_t i0 = blockIdx.x * (size_t)blockDim.x * E + threadIdx.x; i0 < n; i0 += stride) {
    size_t ii[E];
    cx<TV> ui[E];
    cd wi[E], t1[E], t2[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t ie = i0 + (size_t)e * blockDim.x;
      ii[e] = ie < n ? ie : n - 1;  // clamped: loads are unconditional
      ui[e] = u[ii[e]];
      wi[e] = w[ii[e]];
      t1[e] = mk<double>(0, 0);
      t2[e] = mk<double>(0, 0);
    }
    // kUpdUnroll basis vectors per round, the last round included: its
    // indices are clamped to k - 1 and the coefficients past k are zero, so
    // that no load waits behind a branch
    for (int j = 0; j < k; j += kUpdUnroll) {
      cx<TV> vq[E][kUpdUnroll];
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int q = 0; q < kUpdUnroll; ++q) vq[e][q] = vz[(size_t)min(j + q, k - 1) * ldj + ii[e]];
#pragma unroll
      for (int q = 0; q < kUpdUnroll; ++q) {
        const bool in = j + q < k;
        const int jq = min(j + q, k - 1);
        const cd sq = in ? sv[jq] : mk<double>(0, 0), pq = in ? pv[jq] : mk<double>(0, 0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cd vj = cvt<double>(vq[e][q]);
          cfma(t1[e], sq, vj);
          cfma(t2[e], pq, vj);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (i0 + (size_t)e * blockDim.x >= n) continue;
      const cx<TV> vks = cvt<TV>(inu * (cvt<double>(ui[e]) - t1[e]));
      cd wn = wi[e] - t2[e];
      cfma(wn, -hkk, cvt<double>(vks));
      const cx<TV> wns = cvt<TV>(wn);
      store_nt(u + ii[e], vks);
      store_nt(un + ii[e], wns);
      nrm += abs2(cvt<double>(wns));
    }
  }
  const cd r = block_sum(mk<double>(nrm, 0.0), sh);
  if (threadIdx.x == 0) partial[(size_t)z * gridDim.x + blockIdx.x] = r;
}

// w_z -= sum_j h[z ldh + j] V_zj, with the block partials of ||w_z||^2
__global__ void __launch_bounds__(256) k_bmultiaxpy_norm(const cd* __restrict__ V, size_t ldj, BIdx bv, int cnt,
                                                         const cd* __restrict__ h, size_t ldh, cd* __restrict__ w,
                                                         BIdx bw, size_t n, cd* __restrict__ partial) {
  __shared__ cd sh[4];
  const int z = blockIdx.y;
  const cd* v = V + bv.off(z);
  const cd* hz = h + (size_t)z * ldh;
  w += bw.off(z);
  double nrm = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    cd acc = mk<double>(0, 0);
    for (int j = 0; j < cnt; ++j) cfma(acc, hz[j], v[(size_t)j * ldj + i]);
    const cd wn = w[i] - acc;
    w[i] = wn;
    nrm += abs2(wn);
  }
  const cd r = block_sum(mk<double>(nrm, 0.0), sh);
  if (threadIdx.x == 0) partial[(size_t)z * gridDim.x + blockIdx.x] = r;
}

template <class TV>
__global__ void k_bnormalize(const cd* __restrict__ w, BIdx bw, const cd* __restrict__ nrm2, size_t ldn,
                             cx<TV>* __restrict__ v, BIdx bvv, size_t n) {
  const int z = blockIdx.y;
  const double s = 1.0 / sqrt(nrm2[(size_t)z * ldn].re);
  w += bw.off(z);
  v += bvv.off(z);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = cvt<TV>(s * w[i]);
}

inline int nblk(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b == 0 ? 1 : b));
}

// blocks per vector of a batched launch: about 2048 blocks in total
inline int nblk_batch(size_t n, int nb) {
  size_t b = (n + 255) / 256;
  size_t cap = (size_t)std::max(8, 2048 / std::max(nb, 1));
  return (int)(b > cap ? cap : (b == 0 ? 1 : b));
}

}  // namespace

template <class To, class Ti>
void launch_convert(const cx<Ti>* in, cx<To>* out, size_t n, int conjugate, hipStream_t s, int nb, BIdx bi,
                    BIdx bo) {
  if (nb < 1) return;
  hipLaunchKernelGGL((k_convert<To, Ti>), dim3(nb == 1 ? nblk(n) : nblk_batch(n, nb), nb), dim3(256), 0, s, in,
                     out, n, conjugate, bi, bo);
}
template void launch_convert<float, double>(const cd*, cf*, size_t, int, hipStream_t, int, BIdx, BIdx);
template void launch_convert<double, float>(const cf*, cd*, size_t, int, hipStream_t, int, BIdx, BIdx);
template void launch_convert<double, double>(const cd*, cd*, size_t, int, hipStream_t, int, BIdx, BIdx);
template void launch_convert<float, float>(const cf*, cf*, size_t, int, hipStream_t, int, BIdx, BIdx);

template <class T>
void launch_zero(cx<T>* v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_zero<T>), dim3(nblk(n)), dim3(256), 0, s, v, n);
}
template void launch_zero<double>(cd*, size_t, hipStream_t);
void launch_fill(cd* v, size_t n, cd value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, s, v, n, value);
}
template void launch_zero<float>(cf*, size_t, hipStream_t);

void launch_multiaxpy(const cd* V, size_t ldv, int m, const cd* h, cd* w, size_t n, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3(nblk(n)), dim3(256), 0, s, V, ldv, m, h, w, n, sub);
}
void launch_normalize(const cd* w, const cd* nrm2, cd* v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(nblk(n)), dim3(256), 0, s, w, nrm2, v, n);
}
// Blocks per right-hand side of the batched reductions: about 8192 blocks in
// total for the projection pass (times its tiles of basis vectors) and 16384
// for the update pass, so that a launch is many rounds of resident blocks and
// its last round is short, also when few right-hand sides are left.
// The projection pass ends every block with a reduction of 2 kDotTile
// sums, so its blocks keep at least 16 elements per thread.
int batch_dot_blocks(size_t n, int nb) {
  const size_t b = (n + 16 * 256 - 1) / (16 * 256), cap = (size_t)std::max(16, 8192 / std::max(nb, 1));
  static_assert(kDotElems <= 16, "a projection block must hold at least one iteration per thread");
  return (int)(b > cap ? cap : (b == 0 ? 1 : b));
}
int batch_upd_blocks(size_t n, int nb) {
  const size_t per = (size_t)256 * kUpdElems;
  const size_t b = (n + per - 1) / per, cap = (size_t)std::max(32, 16384 / std::max(nb, 1));
  return (int)(b > cap ? cap : (b == 0 ? 1 : b));
}
void launch_bmultidot(const cd* V, size_t ldj, BIdx bv, int cnt, const cd* w, BIdx bw, size_t n, cd* partial,
                      int nblocks, cd* out, size_t ldo, int nb, hipStream_t s) {
  if (nb < 1 || cnt < 1) return;
  const int tiles = (cnt + kDotTile - 1) / kDotTile;
  hipLaunchKernelGGL(k_bmultidot, dim3(nblocks, tiles, nb), dim3(256), 0, s, V, ldj, bv, cnt, w, bw, n, partial);
  hipLaunchKernelGGL(k_breduce, dim3(cnt, nb), dim3(256), 0, s, (const cd*)partial, nblocks, cnt, out, ldo);
}
template <class TV>
void launch_bmultiaxpy(const cx<TV>* V, size_t ldj, BIdx bv, int cnt, const cd* h, size_t ldh, cd* w, BIdx bw,
                       size_t n, int sub, int nb, hipStream_t s) {
  if (nb < 1 || cnt < 1) return;
  hipLaunchKernelGGL(k_bmultiaxpy<TV>, dim3(nblk_batch(n, nb), nb), dim3(256), 0, s, V, ldj, bv, cnt, h, ldh, w, bw,
                     n, sub);
}
template void launch_bmultiaxpy<double>(const cd*, size_t, BIdx, int, const cd*, size_t, cd*, BIdx, size_t, int, int,
                                        hipStream_t);
template void launch_bmultiaxpy<float>(const cf*, size_t, BIdx, int, const cd*, size_t, cd*, BIdx, size_t, int, int,
                                       hipStream_t);
void launch_bmultiaxpy_norm(const cd* V, size_t ldj, BIdx bv, int cnt, const cd* h, size_t ldh, cd* w, BIdx bw,
                            size_t n, cd* partial, int nblocks, cd* nrm2, size_t ldo, int nb, hipStream_t s) {
  if (nb < 1) return;
  hipLaunchKernelGGL(k_bmultiaxpy_norm, dim3(nblocks, nb), dim3(256), 0, s, V, ldj, bv, cnt, h, ldh, w, bw, n,
                     partial);
  hipLaunchKernelGGL(k_breduce, dim3(1, nb), dim3(256), 0, s, (const cd*)partial, nblocks, 1, nrm2, ldo);
}
template <class TV>
void launch_bdcgs_project(const cx<TV>* V, size_t ldj, BIdx bv, int k, const cd* w, BIdx bw, size_t n,
                          cd* partial, int nblocks, cd* hb, size_t ldh, int off, int nb, hipStream_t s) {
  if (nb < 1) return;
  const int cnt = k + 1;
  const int tiles = (cnt + kDotTile - 1) / kDotTile;
  hipLaunchKernelGGL(k_bmultidot2<TV>, dim3(nblocks, tiles, nb), dim3(256), 0, s, V, ldj, bv, cnt, w, bw, n,
                     partial);
  hipLaunchKernelGGL(k_breduce, dim3(2 * cnt, nb), dim3(256), 0, s, (const cd*)partial, nblocks, 2 * cnt, hb, ldh);
  hipLaunchKernelGGL(k_bdcgs_coef, dim3((nb + 63) / 64), dim3(64), 0, s, hb, ldh, k, off, nb);
}
template <class TV>
void launch_bdcgs_update(cx<TV>* V, size_t ldj, BIdx bv, int k, const cd* hb, size_t ldh, int off, const cd* w,
                         BIdx bw, size_t n, cd* partial, int nblocks, cd* nrm2, int nb, hipStream_t s) {
  if (nb < 1) return;
  hipLaunchKernelGGL(k_bdcgs_update<TV>, dim3(nblocks, nb), dim3(256), 0, s, V, ldj, bv, k, hb, ldh, off, w, bw, n,
                     partial);
  hipLaunchKernelGGL(k_breduce, dim3(1, nb), dim3(256), 0, s, (const cd*)partial, nblocks, 1, nrm2, ldh);
}
template <class TV>
void launch_bnormalize(const cd* w, BIdx bw, const cd* nrm2, size_t ldn, cx<TV>* v, BIdx bv, size_t n, int nb,
                       hipStream_t s) {
  if (nb < 1) return;
  hipLaunchKernelGGL(k_bnormalize<TV>, dim3(nblk_batch(n, nb), nb), dim3(256), 0, s, w, bw, nrm2, ldn, v, bv, n);
}
template void launch_bdcgs_project<double>(const cd*, size_t, BIdx, int, const cd*, BIdx, size_t, cd*, int, cd*,
                                           size_t, int, int, hipStream_t);
template void launch_bdcgs_project<float>(const cf*, size_t, BIdx, int, const cd*, BIdx, size_t, cd*, int, cd*,
                                          size_t, int, int, hipStream_t);
template void launch_bdcgs_update<double>(cd*, size_t, BIdx, int, const cd*, size_t, int, const cd*, BIdx, size_t,
                                          cd*, int, cd*, int, hipStream_t);
template void launch_bdcgs_update<float>(cf*, size_t, BIdx, int, const cd*, size_t, int, const cd*, BIdx, size_t,
                                         cd*, int, cd*, int, hipStream_t);
template void launch_bnormalize<double>(const cd*, BIdx, const cd*, size_t, cd*, BIdx, size_t, int, hipStream_t);
template void launch_bnormalize<float>(const cd*, BIdx, const cd*, size_t, cf*, BIdx, size_t, int, hipStream_t);
void launch_scale_rhs_arrays(int n1, int n2, double h2, const cd* ixn, const cd* iyn, const cd* f, cd* b,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rhs, dim3((n2 + 255) / 256, n1), dim3(256), 0, s, n1, n2, h2, ixn, iyn, f, b);
}
void launch_grad_m(int n1, int n2, double scale, const cd* ixn, const cd* iyn, const cd* u, const cd* lam, double* g,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_grad_m, dim3((n2 + 255) / 256, n1), dim3(256), 0, s, n1, n2, scale, ixn, iyn, u, lam, g);
}
void launch_stats(const double* c, size_t n, double* out4, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, s, c, n, out4);
}
void launch_k2_nodes(const double* c, size_t n, double omega, double* k2, hipStream_t s) {
  hipLaunchKernelGGL(k_k2_nodes, dim3(nblk(n)), dim3(256), 0, s, c, n, omega * omega, k2);
}
void launch_cell_average(const double* k2n, int n1, int n2, const int* x0, const double* wx, int nc1,
                         const int* y0, const double* wy, int nc2, double* k2c, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_average, dim3((nc2 + 255) / 256, nc1), dim3(256), 0, s, k2n, n1, n2, x0, wx, y0, wy,
                     nc2, k2c);
}
void launch_sponge_k2(int n1, int n2, const double* bx, const double* by, double* k2, double* k2i, hipStream_t s) {
  hipLaunchKernelGGL(k_sponge_k2, dim3((n2 + 255) / 256, n1), dim3(256), 0, s, n1, n2, bx, by, k2, k2i);
}
void launch_cell_coefs(const double* k2c, size_t ncell, double h_nom, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_coefs, dim3(nblk(ncell)), dim3(256), 0, s, k2c, ncell, h_nom, coef);
}

}  // namespace hsp
