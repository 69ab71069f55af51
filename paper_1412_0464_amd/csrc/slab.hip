// Slab subdomain factorization and the SubdomSolve stage kernels.
//
// A slab A^(j) (Sec. 2.1, subdomains) covers nl layers x n2 tangential nodes.
// Ordered with the tangential index t slowest it is block tridiagonal with
// nl x nl blocks: A_t x_{t-1} + B_t x_t + C_t x_{t+1} = f_t, the blocks being
// tridiagonal in the layer index (compact stencil).  Block LU along t:
//   S_0 = B_0,  S_t = B_t - A_t E_{t-1},  G_t = S_t^{-1},  E_t = G_t C_t.
// S_t is inverted in LDS by Gauss-Jordan with partial (row) pivoting; the
// pivot row is found by a wavefront max-reduction.  All slabs are factored in
// one launch (one workgroup per slab).  Pivoting stays inside each block, so
// the Schur complements S_t are not protected against growth: every slab
// reports its growth factor max_t |S_t|_max / max_t |B_t|_max, which the
// host compares with a limit (the factor loses about log10(growth) digits).
//
// The substitutions of this factorization are evaluated in parallel along t.
// Forward: y_t = G_t (f_t - A_t y_{t-1}) = c_t + M_t y_{t-1} with
// c_t = G_t f_t (independent matvecs) and M_t = -G_t A_t.  The t axis is cut
// into P chunks of m blocks; every chunk runs the chain from y = 0, a short
// chain over the chunk ends propagates the true boundary values through the
// chunk transfer matrices Y_t = M_t ... M_s (s = first block of the chunk),
// and every block adds Y_t y_{s-1}.  Backward: x_t = y_t - E_t x_{t+1}, the
// same with X_t = (-E_t) ... (-E_{e-1}) (e = one past the last block).  In
// exact arithmetic this is the sequential substitution of the same factors.
// All blocks are stored column major (a thread owning output row l reads
// them coalesced).
#include <algorithm>

#include "internal.h"
#include "sweep_dev.h"

namespace hsp {

namespace {

constexpr int kFactorThreads = 1024;

template <class T>
__global__ void __launch_bounds__(kFactorThreads) k_factor(const SlabDev* __restrict__ slabs, int n2, cx<T>* factors,
                                                cd* setup, cd* scratchE, int* status, double* growth,
                                                int dbg_singular) {
  extern __shared__ cd smem[];
  const SlabDev sd = slabs[blockIdx.x];
  const int nl = sd.nl;
  const size_t nb = (size_t)nl * nl;
  cd* S = smem;            // nl*nl, row major
  cd* cfs = S + nl * nl;   // [nl][9] stencil coefficients of the rows at t
  cd* colf = cfs + 9 * nl; // [nl]
  __shared__ int piv[kMaxSlabLayers];
  __shared__ int sh_p, sh_bad;
  cd* Ep = scratchE + (size_t)blockIdx.x * kMaxSlabLayers * kMaxSlabLayers;
  cx<T>* Gm = factors + sd.fac_off;
  cx<T>* Em = Gm + 2 * (size_t)n2 * nb;
  cx<T>* Am = Gm + 5 * (size_t)n2 * nb;
  cd* Gd = setup + sd.scr_off;             // FP64 copies for the transfer matrices
  cd* Ed = Gd + (size_t)n2 * nb;
  cd* Ad = Ed + (size_t)n2 * nb;           // couplings A_t, [t][3][nl]
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) sh_bad = 0;
  double mxB = 0.0, mxS = 0.0;  // largest |entry|^2 of the blocks B_t and of the Schur complements S_t
  // debugging aid: the first block of slab dbg_singular is replaced by zero
  const bool zero_block = (int)blockIdx.x == dbg_singular;

  for (int t = 0; t < n2; ++t) {
    for (int i = tid; i < nl; i += nt) {
      cd c[3][3];
      stencil_coefs(sd.op, i + 1, t + 1, c);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cfs[i * 9 + a * 3 + b] = c[a][b];
          if (b == 1) mxB = fmax(mxB, abs2(c[a][b]));
        }
        Ad[((size_t)t * 3 + a) * nl + i] = c[a][0];
        Am[((size_t)t * 3 + a) * nl + i] = cvt<T>(c[a][0]);
      }
    }
    __syncthreads();
    // S = B_t - A_t E_{t-1}
    for (int idx = tid; idx < nl * nl; idx += nt) {
      const int i = idx / nl, j = idx - (idx / nl) * nl;
      const int d = j - i;
      cd s = (d >= -1 && d <= 1) ? cfs[i * 9 + (d + 1) * 3 + 1] : mk<double>(0, 0);
      if (t > 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int m = i + a - 1;
          if (m < 0 || m >= nl) continue;
          s -= cfs[i * 9 + a * 3 + 0] * Ep[m * nl + j];
        }
      }
      if (zero_block && t == 0) s = mk<double>(0, 0);
      mxS = fmax(mxS, abs2(s));
      S[idx] = s;
    }
    __syncthreads();
    // in-place Gauss-Jordan inversion with partial pivoting
    for (int k = 0; k < nl; ++k) {
      if (tid < 64) {
        const int i = k + tid;
        double v = (i < nl) ? abs2(S[i * nl + k]) : -1.0;
        int id = i;
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(v, off, 64);
          const int oi = __shfl_xor(id, off, 64);
          if (ov > v || (ov == v && oi < id)) {
            v = ov;
            id = oi;
          }
        }
        if (tid == 0) {
          sh_p = id;
          piv[k] = id;
          if (!(v > 0.0) || !isfinite(v)) sh_bad = 1;
        }
      }
      __syncthreads();
      const int p = sh_p;
      if (p != k)
        for (int c = tid; c < nl; c += nt) {
          const cd tmp = S[k * nl + c];
          S[k * nl + c] = S[p * nl + c];
          S[p * nl + c] = tmp;
        }
      __syncthreads();
      const cd pv = S[k * nl + k];
      for (int i = tid; i < nl; i += nt) colf[i] = S[i * nl + k];
      __syncthreads();
      const cd inv = cinv(pv);
      for (int c = tid; c < nl; c += nt) S[k * nl + c] = (c == k) ? inv : S[k * nl + c] * inv;
      __syncthreads();
      for (int idx = tid; idx < nl * nl; idx += nt) {
        const int i = idx / nl, c = idx - (idx / nl) * nl;
        if (i == k) continue;
        const cd f = colf[i];
        if (c == k)
          S[idx] = -(f * S[k * nl + k]);
        else
          S[idx] -= f * S[k * nl + c];
      }
      __syncthreads();
    }
    for (int k = nl - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        for (int i = tid; i < nl; i += nt) {
          const cd tmp = S[i * nl + k];
          S[i * nl + k] = S[i * nl + p];
          S[i * nl + p] = tmp;
        }
      }
      __syncthreads();
    }
    // store G_t and E_t = G_t C_t (column major)
    for (int idx = tid; idx < nl * nl; idx += nt) {
      const int j = idx / nl, i = idx - (idx / nl) * nl;
      const cd gv = S[i * nl + j];
      Gm[(size_t)t * nb + idx] = cvt<T>(gv);
      Gd[(size_t)t * nb + idx] = gv;
      cd e = mk<double>(0, 0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int m = j + a - 1;
        if (m < 0 || m >= nl) continue;
        e += S[i * nl + m] * cfs[m * 9 + (j - m + 1) * 3 + 2];
      }
      Em[(size_t)t * nb + idx] = cvt<T>(e);
      Ed[(size_t)t * nb + idx] = e;
      Ep[i * nl + j] = e;
    }
    __syncthreads();
  }
  if (tid == 0 && sh_bad) atomicOr(status, 1);
  // growth factor of this slab
  __syncthreads();
  double* red = reinterpret_cast<double*>(S);
  red[tid] = mxB;
  red[nt + tid] = mxS;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (tid < off) {
      red[tid] = fmax(red[tid], red[tid + off]);
      red[nt + tid] = fmax(red[nt + tid], red[nt + tid + off]);
    }
    __syncthreads();
  }
  if (tid == 0) growth[blockIdx.x] = red[0] > 0.0 ? sqrt(red[nt] / red[0]) : 0.0;
}

// C = sign * A B for column-major nl x nl matrices in double (setup only).
__device__ __forceinline__ void matmul_cm(const cd* A, const cd* B, cd* C, int nl, double sign) {
  for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) {
    const int j = idx / nl, i = idx - (idx / nl) * nl;
    cd acc = mk<double>(0, 0);
    for (int k = 0; k < nl; ++k) cfma(acc, A[(size_t)k * nl + i], B[(size_t)j * nl + k]);
    C[idx] = sign * acc;
  }
}

// Per chunk (blockIdx.x) of a slab (blockIdx.y): M_t = -G_t A_t, the forward
// transfer matrices Y_t = M_t Y_{t-1} (Y_s = M_s), the backward transfer
// matrices X_t = -E_t X_{t+1} (X_{e-1} = -E_{e-1}) and W_t = Y_t - E_t W_{t+1}
// (W_{e-1} = Y_{e-1}), the chunk-local backward substitution of the columns
// of Y.  Products in double (W from the stored Y).
template <class T>
__global__ void __launch_bounds__(256) k_chunk_transfer(const SlabDev* __restrict__ slabs, int n2, int m,
                                                        cx<T>* factors, const cd* setup, cd* tmp) {
  const SlabDev sd = slabs[blockIdx.y];
  const int nl = sd.nl, p = blockIdx.x, P = gridDim.x;
  const size_t nb = (size_t)nl * nl;
  const int s = p * m, e = min(s + m, n2);
  if (s >= n2) return;
  const cd* Gd = setup + sd.scr_off;
  const cd* Ed = Gd + (size_t)n2 * nb;
  const cd* Ad = Ed + (size_t)n2 * nb;
  cx<T>* Mm = factors + sd.fac_off + (size_t)n2 * nb;
  cx<T>* Ym = factors + sd.fac_off + 3 * (size_t)n2 * nb;
  cx<T>* Xm = factors + sd.fac_off + 4 * (size_t)n2 * nb;
  cx<T>* Wm = factors + sd.fac_off + 5 * (size_t)n2 * nb + (size_t)3 * n2 * nl;
  cd* bufM = tmp + ((size_t)blockIdx.y * P + p) * 3 * kMaxSlabLayers * kMaxSlabLayers;
  cd* bufA = bufM + kMaxSlabLayers * kMaxSlabLayers;
  cd* bufB = bufA + kMaxSlabLayers * kMaxSlabLayers;
  // The first chunk has no forward transfer and the last no backward one;
  // their blocks are multiplied by zero in the chains over chunk ends and
  // must hold finite values.
  if (p == 0)
    for (size_t idx = threadIdx.x; idx < (size_t)(e - s) * nb; idx += blockDim.x) {
      Ym[(size_t)s * nb + idx] = mk<T>(0, 0);
      Wm[(size_t)s * nb + idx] = mk<T>(0, 0);
    }
  if (p == P - 1)
    for (size_t idx = threadIdx.x; idx < (size_t)(e - s) * nb; idx += blockDim.x)
      Xm[(size_t)s * nb + idx] = mk<T>(0, 0);
  for (int t = s; t < e; ++t) {
    // M_t = -G_t A_t; (G A)[i][j] = sum_a G[i][j-a+1] A_t[j-a+1 -> j]
    for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) {
      const int j = idx / nl, i = idx - (idx / nl) * nl;
      cd acc = mk<double>(0, 0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int k = j - a + 1;
        if (k < 0 || k >= nl) continue;
        cfma(acc, Gd[(size_t)t * nb + (size_t)k * nl + i], Ad[((size_t)t * 3 + a) * nl + k]);
      }
      bufM[idx] = -acc;
      Mm[(size_t)t * nb + idx] = cvt<T>(-acc);
    }
    __syncthreads();
    if (p > 0) {
      if (t == s) {
        for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) bufB[idx] = bufM[idx];
      } else {
        matmul_cm(bufM, bufA, bufB, nl, 1.0);
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) {
        Ym[(size_t)t * nb + idx] = cvt<T>(bufB[idx]);
        bufA[idx] = bufB[idx];
      }
      __syncthreads();
    }
  }
  if (p < P - 1) {
    for (int t = e - 1; t >= s; --t) {
      if (t == e - 1) {
        for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) bufB[idx] = -Ed[(size_t)t * nb + idx];
      } else {
        matmul_cm(Ed + (size_t)t * nb, bufA, bufB, nl, -1.0);
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) {
        Xm[(size_t)t * nb + idx] = cvt<T>(bufB[idx]);
        bufA[idx] = bufB[idx];
      }
      __syncthreads();
    }
  }
  if (p > 0) {
    for (int t = e - 1; t >= s; --t) {
      if (t == e - 1) {
        for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) bufB[idx] = mk<double>(0, 0);
      } else {
        matmul_cm(Ed + (size_t)t * nb, bufA, bufB, nl, -1.0);
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < nl * nl; idx += blockDim.x) {
        const cd wv = bufB[idx] + cvt<double>(Ym[(size_t)t * nb + idx]);
        Wm[(size_t)t * nb + idx] = cvt<T>(wv);
        bufA[idx] = wv;
      }
      __syncthreads();
    }
  }
}

// Row slice of a column-major block: entries (row lc, columns j0..j0+CW-1),
// unconditional loads from clamped (always valid) addresses, zero outside.
// (A load inside a divergent branch would make the compiler wait for every
// outstanding vector-memory operation at the join, draining the prefetch.)
template <class T, int CW>
__device__ __forceinline__ void fetch_slice(const cx<T>* __restrict__ blk, int nl, int lc, int j0, bool act,
                                            cx<T> (&dst)[CW]) {
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int j = j0 + c;
    const int jc = j < nl ? j : nl - 1;
    dst[c] = sel(act && j < nl, blk[(size_t)jc * nl + lc]);
  }
}

// Lane layout of the dependent chains (one wavefront): R row slots (32 when
// the slab has <= 32 layers, else 64) times NG = 64 / R column groups; lane
// (l, h) owns row l and columns [h CW, (h+1) CW) of every block.
template <int NB>
struct Layout {
  static constexpr int R = (NB <= 32) ? 32 : 64;
  static constexpr int NG = 64 / R;
  static constexpr int CW = (NB + NG - 1) / NG;
};

// Affine chain z_k = b_k + sigma M_k z_{k-1}, k = 0..count-1, z_{-1} = 0,
// run by the first wavefront of the workgroup (the other waves wait at the
// final barrier).  Step k uses index r = first + dir k: matrix M at
// mat + r * mstride, b_k at rows[r * nl + l]; z_k overwrites b_k.  The
// matrix slices and b of the next D steps are kept in a register ring so
// that the latency of the matrix stream overlaps the dependent steps.  Per
// step: the two column halves' partial products are combined by a
// cross-half shuffle, the row owners publish z_{k-1} in LDS, every lane forms
// its partial product of M_k z_{k-1}.
template <class T, int NB, int D>
__device__ __forceinline__ void chain_one_wave(const cx<T>* __restrict__ mat, long mstride, cx<T>* rows, int first,
                                               int dir, int count, int nl, T sigma, cx<T>* vs) {
  using LY = Layout<NB>;
  constexpr int R = LY::R, NG = LY::NG, CW = LY::CW;
  if (threadIdx.x < 64 && count > 0) {
    const int lane = threadIdx.x;
    const int l = lane % R, h = lane / R, j0 = h * CW;
    const bool act = l < nl;
    const bool own = act && h == 0;
    const int lc = l < nl ? l : nl - 1;
    cx<T> rg[D][CW], rb[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int r = first + dir * (d < count ? d : count - 1);
      fetch_slice<T, CW>(mat + r * mstride, nl, lc, j0, act, rg[d]);
      rb[d] = sel(act, rows[(size_t)r * nl + lc]);
    }
    cx<T> bprev = mk<T>(0, 0), part = mk<T>(0, 0);
    auto full_sum = [](cx<T> pv) {
      if constexpr (NG == 2) {
        pv.re += __shfl_xor(pv.re, 32, 64);
        pv.im += __shfl_xor(pv.im, 32, 64);
      }
      return pv;
    };
#define HSP_CHAIN_STEP(k, d)                                                              \
  {                                                                                       \
    cx<T> z = mk<T>(0, 0);                                                                \
    if ((k) > 0) {                                                                        \
      const cx<T> sm = full_sum(part);                                                    \
      z = mk<T>(bprev.re + sigma * sm.re, bprev.im + sigma * sm.im);                      \
      if (own) rows[(size_t)(first + dir * ((k) - 1)) * nl + l] = z;                      \
    }                                                                                     \
    if (h == 0 && l < NG * CW) vs[l] = sel(act, z);                                       \
    bprev = rb[d];                                                                        \
    wave_lds_sync();                                                                      \
    part = mk<T>(0, 0);                                                                   \
    _Pragma("unroll") for (int c = 0; c < CW; ++c) cfma(part, rg[d][c], vs[j0 + c]);      \
    wave_lds_sync();                                                                      \
  }
#define HSP_CHAIN_FETCH(kn, d)                                                            \
  {                                                                                       \
    const int r = first + dir * ((kn) < count ? (kn) : count - 1);                        \
    fetch_slice<T, CW>(mat + r * mstride, nl, lc, j0, act, rg[d]);                        \
    rb[d] = sel(act, rows[(size_t)r * nl + lc]);                                          \
  }
    int k0 = 0;
    for (; k0 + D <= count; k0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        HSP_CHAIN_STEP(k0 + d, d)
        HSP_CHAIN_FETCH(k0 + d + D, d)
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (k0 + d < count) HSP_CHAIN_STEP(k0 + d, d)
    }
#undef HSP_CHAIN_STEP
#undef HSP_CHAIN_FETCH
    const cx<T> sm = full_sum(part);
    if (own)
      rows[(size_t)(first + dir * (count - 1)) * nl + l] = mk<T>(bprev.re + sigma * sm.re, bprev.im + sigma * sm.im);
  }
  __syncthreads();
}


// The same chain for thick slabs (> 32 layers), run by the whole workgroup:
// 64 row slots times NT / 64 column groups, partial products summed through
// LDS, two workgroup barriers per step.
template <class T, int NB, int NT, int D>
__device__ __forceinline__ void chain_workgroup(const cx<T>* __restrict__ mat, long mstride, cx<T>* rows, int first,
                                                int dir, int count, int nl, T sigma, cx<T>* vs, cx<T>* ps) {
  constexpr int R = 64, NG = NT / R, CW = (NB + NG - 1) / NG;
  const int tid = threadIdx.x;
  const int l = tid % R, h = tid / R, j0 = h * CW;
  const bool act = l < nl;
  const bool own = act && h == 0;
  const int lc = l < nl ? l : nl - 1;
  if (count <= 0) return;
  cx<T> rg[D][CW], rb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int r = first + dir * (d < count ? d : count - 1);
    fetch_slice<T, CW>(mat + r * mstride, nl, lc, j0, act, rg[d]);
    rb[d] = sel(act, rows[(size_t)r * nl + lc]);
  }
  cx<T> bprev = mk<T>(0, 0);
#define HSP_CHAIN_STEP(k, d)                                                              \
  {                                                                                       \
    if ((k) > 0) {                                                                        \
      cx<T> sm = mk<T>(0, 0);                                                             \
      _Pragma("unroll") for (int q = 0; q < NG; ++q) sm = sm + ps[q * R + l];             \
      const cx<T> z = mk<T>(bprev.re + sigma * sm.re, bprev.im + sigma * sm.im);          \
      if (own) rows[(size_t)(first + dir * ((k) - 1)) * nl + l] = z;                      \
      if (h == 0 && l < NG * CW) vs[l] = sel(act, z);                                     \
    } else {                                                                              \
      if (h == 0 && l < NG * CW) vs[l] = mk<T>(0, 0);                                     \
    }                                                                                     \
    bprev = rb[d];                                                                        \
    __syncthreads();                                                                      \
    cx<T> part = mk<T>(0, 0);                                                             \
    _Pragma("unroll") for (int c = 0; c < CW; ++c) cfma(part, rg[d][c], vs[j0 + c]);      \
    ps[h * R + l] = sel(act, part);                                                       \
    __syncthreads();                                                                      \
  }
#define HSP_CHAIN_FETCH(kn, d)                                                            \
  {                                                                                       \
    const int r = first + dir * ((kn) < count ? (kn) : count - 1);                        \
    fetch_slice<T, CW>(mat + r * mstride, nl, lc, j0, act, rg[d]);                        \
    rb[d] = sel(act, rows[(size_t)r * nl + lc]);                                          \
  }
  int k0 = 0;
  for (; k0 + D <= count; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      HSP_CHAIN_STEP(k0 + d, d)
      HSP_CHAIN_FETCH(k0 + d + D, d)
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (k0 + d < count) HSP_CHAIN_STEP(k0 + d, d)
  }
#undef HSP_CHAIN_STEP
#undef HSP_CHAIN_FETCH
  if (own) {
    cx<T> sm = mk<T>(0, 0);
#pragma unroll
    for (int q = 0; q < NG; ++q) sm = sm + ps[q * R + l];
    rows[(size_t)(first + dir * (count - 1)) * nl + l] = mk<T>(bprev.re + sigma * sm.re, bprev.im + sigma * sm.im);
  }
  __syncthreads();
}

// Chain dispatcher: one wavefront for thin slabs, the workgroup otherwise.
template <class T, int NB, int NT, int D>
__device__ __forceinline__ void affine_chain(const cx<T>* __restrict__ mat, long mstride, cx<T>* rows, int first,
                                             int dir, int count, int nl, T sigma, cx<T>* vs, cx<T>* ps) {
  if constexpr (NB <= 32)
    chain_one_wave<T, NB, D>(mat, mstride, rows, first, dir, count, nl, sigma, vs);
  else
    chain_workgroup<T, NB, NT, D>(mat, mstride, rows, first, dir, count, nl, sigma, vs, ps);
}

// ---- stage kernel 1: right-hand side, c_t = G_t f_t, forward chain per
//      chunk, then (last workgroup) the chain over the chunk ends.
template <class T, int NB, int NT, int D>
__global__ void __launch_bounds__(NT) k_stage_fwd(const TaskDev* __restrict__ tasks, const SlabDev* __restrict__ slabs,
                                                  LevelDev G, const cx<T>* __restrict__ f, const cx<T>* __restrict__ g,
                                                  const cx<T>* __restrict__ bufs, cx<T>* __restrict__ scratch,
                                                  const cx<T>* __restrict__ factors, int nl_max, int m,
                                                  cx<T>* __restrict__ red, int* counters) {
  constexpr int MAXV = (kMaxChunk * NB + NT - 1) / NT;  // per-thread entries of c
  __shared__ cx<T> vs[64];
  __shared__ cx<T> ps[NT];
  const int task = blockIdx.y, p = blockIdx.x, P = gridDim.x;
  const TaskDev tk = tasks[task];
  const SlabDev sd = slabs[tk.slab];
  const int nl = sd.nl, n2 = G.n2;
  const int s = p * m, e = min(s + m, n2), cnt = e - s;
  const SlabFac<T> F(factors + sd.fac_off, n2, nl);
  cx<T>* y = scratch + (size_t)task * n2 * nl_max;
  cx<T>* tips = red + (size_t)task * 2 * (size_t)P * nl_max;  // [P][nl] forward tips
  const cx<T>* src = tk.src ? g : f;
  const cx<T>* Bif = bufs + (size_t)tk.bin_f * 2 * n2;
  const cx<T>* Bib = bufs + (size_t)tk.bin_b * 2 * n2;
  const int tid = threadIdx.x;
  // slab right-hand side of the chunk
  for (int idx = tid; idx < nl * cnt; idx += NT) {
    const int ll = idx / cnt, t = s + idx - (idx / cnt) * cnt;
    const int gl = sd.x0 + ll;
    cx<T> v = mk<T>(0, 0);
    if (tk.mode == 1) {
      v = src[(size_t)ll * n2 + t];
    } else {
      if (tk.a < gl && gl <= tk.b) v = src[(size_t)(gl - 1) * n2 + t];
      v = v + cvt<T>(transmission_rhs<T>(tk, G, gl, t, n2, Bif, Bib));
    }
    y[(size_t)t * nl + ll] = v;
  }
  __syncthreads();
  // c_t = G_t f_t (rows of the chunk in parallel), computed then written back
  cx<T> cv[MAXV];
#pragma unroll
  for (int q = 0; q < MAXV; ++q) {
    const int idx = tid + q * NT;
    cv[q] = mk<T>(0, 0);
    if (idx < nl * cnt) {
      const int t = s + idx / nl, l = idx - (idx / nl) * nl;
      const cx<T>* gb = F.G + (size_t)t * nl * nl + l;
      const cx<T>* fr = y + (size_t)t * nl;
      cx<T> acc = mk<T>(0, 0);
#pragma unroll 8
      for (int j = 0; j < nl; ++j) cfma(acc, gb[(size_t)j * nl], fr[j]);
      cv[q] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXV; ++q) {
    const int idx = tid + q * NT;
    if (idx < nl * cnt) y[(size_t)(s + idx / nl) * nl + (idx - (idx / nl) * nl)] = cv[q];
  }
  __syncthreads();
  // chunk-local forward chain y_t = c_t + M_t y_{t-1}
  affine_chain<T, NB, NT, D>(F.M, (long)nl * nl, y, s, 1, cnt, nl, T(1), vs, ps);
  for (int l = tid; l < nl; l += NT) tips[(size_t)p * nl + l] = y[(size_t)(e - 1) * nl + l];
  if (P == 1) return;
  if (!last_arrival(counters + 2 * task, P)) return;
  // true chunk-end values: tip_q = raw_q + Y_{e_q - 1} tip_{q-1}, q = 0..P-2
  affine_chain<T, NB, NT, D>(F.Y + (size_t)(m - 1) * nl * nl, (long)m * nl * nl, tips, 0, 1, P - 1, nl, T(1), vs,
                             ps);
}

// ---- stage kernel 2: forward fix-up y_t += Y_t tip_{p-1}, backward chain
//      per chunk, then (last workgroup) the chain over the chunk starts.
template <class T, int NB, int NT, int D>
__global__ void __launch_bounds__(NT) k_stage_mid(const TaskDev* __restrict__ tasks, const SlabDev* __restrict__ slabs,
                                                  int n2, cx<T>* __restrict__ scratch, const cx<T>* __restrict__ factors,
                                                  int nl_max, int m, cx<T>* __restrict__ red, int* counters) {
  __shared__ cx<T> vs[64];
  __shared__ cx<T> ps[NT];
  __shared__ cx<T> tv[kMaxSlabLayers];
  const int task = blockIdx.y, p = blockIdx.x, P = gridDim.x;
  const TaskDev tk = tasks[task];
  const SlabDev sd = slabs[tk.slab];
  const int nl = sd.nl;
  const int s = p * m, e = min(s + m, n2), cnt = e - s;
  const SlabFac<T> F(factors + sd.fac_off, n2, nl);
  cx<T>* y = scratch + (size_t)task * n2 * nl_max;
  cx<T>* tips = red + (size_t)task * 2 * (size_t)P * nl_max;
  cx<T>* heads = tips + (size_t)P * nl_max;  // [P][nl] backward heads
  const int tid = threadIdx.x;
  if (p > 0) {
    for (int l = tid; l < nl; l += NT) tv[l] = tips[(size_t)(p - 1) * nl + l];
    __syncthreads();
    for (int idx = tid; idx < nl * cnt; idx += NT) {
      const int t = s + idx / nl, l = idx - (idx / nl) * nl;
      const cx<T>* yb = F.Y + (size_t)t * nl * nl + l;
      cx<T> acc = y[(size_t)t * nl + l];
#pragma unroll 8
      for (int j = 0; j < nl; ++j) cfma(acc, yb[(size_t)j * nl], tv[j]);
      y[(size_t)t * nl + l] = acc;
    }
    __syncthreads();
  }
  // chunk-local backward chain x_t = y_t - E_t x_{t+1}
  affine_chain<T, NB, NT, D>(F.E, (long)nl * nl, y, e - 1, -1, cnt, nl, T(-1), vs, ps);
  for (int l = tid; l < nl; l += NT) heads[(size_t)p * nl + l] = y[(size_t)s * nl + l];
  if (P == 1) return;
  if (!last_arrival(counters + 2 * task + 1, P)) return;
  // true chunk-start values: head_q = raw_q + X_{s_q} head_{q+1}, q = P-1..1
  affine_chain<T, NB, NT, D>(F.X, (long)m * nl * nl, heads, P - 1, -1, P - 1, nl, T(1), vs, ps);
}

// ---- stage kernel 3: backward fix-up x_t += X_t head_{p+1}, then the
//      scatter-add into u and the outgoing transmission layers.
template <class T, int NT>
__global__ void __launch_bounds__(NT) k_stage_bwd(const TaskDev* __restrict__ tasks, const SlabDev* __restrict__ slabs,
                                                  int n2, cx<T>* __restrict__ u, cx<T>* __restrict__ bufs,
                                                  cx<T>* __restrict__ scratch, const cx<T>* __restrict__ factors,
                                                  int nl_max, int m, const cx<T>* __restrict__ red) {
  __shared__ cx<T> hv[kMaxSlabLayers];
  const int task = blockIdx.y, p = blockIdx.x, P = gridDim.x;
  const TaskDev tk = tasks[task];
  const SlabDev sd = slabs[tk.slab];
  const int nl = sd.nl;
  const int s = p * m, e = min(s + m, n2), cnt = e - s;
  const SlabFac<T> F(factors + sd.fac_off, n2, nl);
  cx<T>* y = scratch + (size_t)task * n2 * nl_max;
  const cx<T>* heads = red + (size_t)task * 2 * (size_t)P * nl_max + (size_t)P * nl_max;
  cx<T>* Bof = bufs + (size_t)tk.bout_f * 2 * n2;
  cx<T>* Bob = bufs + (size_t)tk.bout_b * 2 * n2;
  const int tid = threadIdx.x;
  if (p < P - 1) {
    for (int l = tid; l < nl; l += NT) hv[l] = heads[(size_t)(p + 1) * nl + l];
    __syncthreads();
    for (int idx = tid; idx < nl * cnt; idx += NT) {
      const int t = s + idx / nl, l = idx - (idx / nl) * nl;
      const cx<T>* xb = F.X + (size_t)t * nl * nl + l;
      cx<T> acc = y[(size_t)t * nl + l];
#pragma unroll 8
      for (int j = 0; j < nl; ++j) cfma(acc, xb[(size_t)j * nl], hv[j]);
      y[(size_t)t * nl + l] = acc;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nl * cnt; idx += NT) {
    const int ll = idx / cnt, t = s + idx - (idx / cnt) * cnt;
    const int gl = sd.x0 + ll;
    const cx<T> x = y[(size_t)t * nl + ll];
    if (tk.mode == 1) {
      u[(size_t)ll * n2 + t] = x;
      continue;
    }
    if (tk.at < gl && gl <= tk.bt) {
      const size_t id = (size_t)(gl - 1) * n2 + t;
      u[id] = u[id] + x;
    }
    if (tk.t2) {
      if (gl == tk.beta_out) Bof[t] = x;
      if (gl == tk.beta_out + 1) Bof[(size_t)n2 + t] = x;
    }
    if (tk.t4) {
      if (gl == tk.bt_out) Bob[t] = x;
      if (gl == tk.bt_out + 1) Bob[(size_t)n2 + t] = x;
    }
  }
}

}  // namespace

template <class T>
void launch_factor(const SlabDev* slabs_dev, int nslabs, int nl_max, int n2, int m, int P, cx<T>* factors,
                   cd* setup, cd* scratchE, cd* tmp, int* status, double* growth, int dbg_singular,
                   hipStream_t s) {
  // LDS: S, the row coefficients and one column; at least 2 x 256 doubles
  // for the growth reduction, which reuses S
  const size_t shm = std::max(((size_t)nl_max * nl_max + 10 * (size_t)nl_max) * sizeof(cd),
                              2 * (size_t)kFactorThreads * sizeof(double));
  hipLaunchKernelGGL((k_factor<T>), dim3(nslabs), dim3(kFactorThreads), shm, s, slabs_dev, n2, factors, setup, scratchE, status,
                     growth, dbg_singular);
  hipLaunchKernelGGL((k_chunk_transfer<T>), dim3(P, nslabs), dim3(256), 0, s, slabs_dev, n2, m, factors,
                     (const cd*)setup, tmp);
}

template <class T>
void launch_stage(const TaskDev* tasks_dev, int ntasks, const SlabDev* slabs_dev, const LevelDev& G,
                  const cx<T>* f, const cx<T>* g, cx<T>* u, cx<T>* bufs, cx<T>* scratch, const cx<T>* factors,
                  int nl_max, int nl_launch, int m, int P, cx<T>* red, int* counters, hipStream_t s) {
  const dim3 grd(P, ntasks);
  const int n2 = G.n2;
#define LAUNCH3(NB, NT, D)                                                                                    \
  do {                                                                                                        \
    hipLaunchKernelGGL((k_stage_fwd<T, NB, NT, D>), grd, dim3(NT), 0, s, tasks_dev, slabs_dev, G, f, g,        \
                       (const cx<T>*)bufs, scratch, factors, nl_max, m, red, counters);                       \
    hipLaunchKernelGGL((k_stage_mid<T, NB, NT, D>), grd, dim3(NT), 0, s, tasks_dev, slabs_dev, n2, scratch,    \
                       factors, nl_max, m, red, counters);                                                    \
    hipLaunchKernelGGL((k_stage_bwd<T, NT>), grd, dim3(NT), 0, s, tasks_dev, slabs_dev, n2, u, bufs, scratch,  \
                       factors, nl_max, m, (const cx<T>*)red);                                                \
  } while (0)
  // prefetch depth of the chains: thin slabs run on one wavefront with 16
  // columns per lane, thick slabs on 512 threads with 5-8 columns per thread
  constexpr int DS = sizeof(T) == 4 ? 6 : 3;
  constexpr int DW = sizeof(T) == 4 ? 4 : 2;
  if (nl_launch <= 16)
    LAUNCH3(16, 128, DS);
  else if (nl_launch <= 32)
    LAUNCH3(32, 256, DS);
  else if (nl_launch <= 40)
    LAUNCH3(40, 512, DW);
  else if (nl_launch <= 48)
    LAUNCH3(48, 512, DW);
  else
    LAUNCH3(64, 512, DW);
#undef LAUNCH3
}

template void launch_factor<double>(const SlabDev*, int, int, int, int, int, cd*, cd*, cd*, cd*, int*, double*, int,
                                    hipStream_t);
template void launch_factor<float>(const SlabDev*, int, int, int, int, int, cf*, cd*, cd*, cd*, int*, double*, int,
                                   hipStream_t);
template void launch_stage<double>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cd*, const cd*, cd*,
                                   cd*, cd*, const cd*, int, int, int, int, cd*, int*, hipStream_t);
template void launch_stage<float>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cf*, const cf*, cf*,
                                  cf*, cf*, const cf*, int, int, int, int, cf*, int*, hipStream_t);

}  // namespace hsp
