// Three-dimensional slabs: factorization of the dense blocks and the
// SubdomSolve stage (Sec. 2.1 subdomains, Sec. 2.2 helper algorithms).
//
// A 3-D slab A^(j) (nl x-layers of m2 x m3 nodes) is block tridiagonal along
// y with dense n x n blocks, n = nl m3 (the unknowns of one y-plane):
//   L_t x_{t-1} + D_t x_t + U_t x_{t+1} = f_t,
// where D_t is the 9-point (x, z) stencil of the plane and L_t, U_t the
// couplings to the neighbouring planes.  Block LU along y (pivoting inside
// each block only, as the paper's direct slab solves assume a non-singular
// slab): S_0 = D_0, S_t = D_t - L_t E_{t-1}, G_t = S_t^{-1}, E_t = G_t U_t.
// The factors kept for the solves are W_t = [G_t | M_t] with M_t = -G_t L_t
// and E_t, so that both substitutions are plain dense matrix-vector
// products:
//   forward  y_t = G_t f_t + M_t y_{t-1},   backward  x_t = y_t - E_t x_{t+1}.
//
// S_t is inverted in place by blocked Gauss-Jordan elimination with partial
// (row) pivoting, 32 columns per panel: the panel is eliminated by one
// workgroup (rows in registers, argmax pivot search by wavefront shuffles),
// the row interchanges are applied to the other columns, and the rest of
// the matrix takes the rank-32 update R <- R + P' B_K (P' the eliminated
// panel, B_K the pivot rows of R) as a complex product on the FP32 matrix
// cores (v_mfma_f32_32x32x2f32, four real products per complex one, FP32
// accumulation).  The row interchanges turn into a column permutation of
// the computed inverse, applied when the factors are stored.  Everything is
// complex64; all slabs of a level are processed by the same launches.
#include <algorithm>
#include <cmath>

#include "d3.h"

namespace hsp {
namespace d3 {

namespace {

constexpr int kNB = 32;        // panel width
constexpr int kPanelT = 1024;  // threads of the panel kernel

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

inline int nblk(size_t n, int t = 256) { return (int)std::min<size_t>((n + t - 1) / t, (size_t)1 << 20); }

// padded row length (even, so that rows of complex64 start 16-byte aligned)
__host__ __device__ inline int padded(int n) { return n + (n & 1); }

// Factor block pointers of slab sl at block t: W_t (n x 2n) then E_t
// (n x padded(n)).
__device__ __forceinline__ size_t block_elems(int n) { return (size_t)2 * n * n + (size_t)n * padded(n); }
__device__ __forceinline__ cf* Wblk(cf* fac, const Slab3& sl, int t) {
  return fac + sl.fac_off + (size_t)t * block_elems(sl.n);
}
__device__ __forceinline__ const cf* Wblk(const cf* fac, const Slab3& sl, int t) {
  return fac + sl.fac_off + (size_t)t * block_elems(sl.n);
}

__device__ __forceinline__ void atomic_max_pos(double* a, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(a), (unsigned long long)__double_as_longlong(v));
}

// Block reduction of a non-negative value into *a (max).
__device__ __forceinline__ void block_max_into(double v, double* a) {
  __shared__ double sh[32];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) m = fmax(m, sh[w]);
    if (m > 0) atomic_max_pos(a, m);
  }
}

// ---- setup -----------------------------------------------------------------

// Coefficient rows of block t of every slab: coef[q][27] for the rows
// q = x_l m3 + z of the plane y = t + 1; the running max of |D_t| entries.
__global__ void __launch_bounds__(256) k3_coef(Setup3 Su, int t) {
  const Slab3 sl = Su.slabs[blockIdx.y];
  const int q = blockIdx.x * 256 + threadIdx.x;
  double mx = 0;
  if (q < sl.n) {
    const int m3 = sl.op.m3;
    const int xl = q / m3, z = q - (q / m3) * m3;
    cd c[27];
    coefs27(sl.op, xl + 1, t + 1, z + 1, c);
    cf* o = Su.coef + ((size_t)blockIdx.y * Su.n_max + q) * 27;
#pragma unroll
    for (int a = 0; a < 27; ++a) {
      o[a] = cvt<float>(c[a]);
      if ((a / 3) % 3 == 1) mx = fmax(mx, abs2(c[a]));
    }
  }
  block_max_into(mx, Su.gmax + 2 * blockIdx.y);
}

// S_t = D_t - L_t E_{t-1} (S_0 = D_0), row stride n_max.
__global__ void __launch_bounds__(256) k3_schur(Setup3 Su, int t) {
  const Slab3 sl = Su.slabs[blockIdx.y];
  const int n = sl.n;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  double mx = 0;
  if (idx < (size_t)n * n) {
    const int i = (int)(idx / n), j = (int)(idx - (idx / n) * n);
    const int m3 = sl.op.m3, nl = sl.nl;
    const int xi = i / m3, zi = i - (i / m3) * m3;
    const int xj = j / m3, zj = j - (j / m3) * m3;
    const cf* ci = Su.coef + ((size_t)blockIdx.y * Su.n_max + i) * 27;
    cf s = mk<float>(0, 0);
    const int dx = xj - xi, dz = zj - zi;
    if (dx >= -1 && dx <= 1 && dz >= -1 && dz <= 1) s = ci[(dx + 1) * 9 + 3 + (dz + 1)];
    if (t > 0) {
      const cf* E = Wblk(Su.factors, sl, t - 1) + (size_t)2 * n * n;
      const int ldE = padded(n);
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int xr = xi + a;
        if (xr < 0 || xr >= nl) continue;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
          const int zr = zi + b;
          if (zr < 0 || zr >= m3) continue;
          const cf l = ci[(a + 1) * 9 + 0 + (b + 1)];
          const cf e = E[(size_t)(xr * m3 + zr) * ldE + j];
          s.re -= l.re * e.re - l.im * e.im;
          s.im -= l.re * e.im + l.im * e.re;
        }
      }
    }
    if ((int)blockIdx.y == Su.dbg_singular && t == 0) s = mk<float>(0, 0);
    mx = abs2(cvt<double>(s));
    Su.S[((size_t)blockIdx.y * Su.n_max + i) * Su.n_max + j] = s;
  }
  block_max_into(mx, Su.gmax + 2 * blockIdx.y + 1);
}

// ---- dense partial Gauss-Jordan elimination (GJob) -------------------------
// Gauss-Jordan elimination of the panel columns k0..k0+31 over the rows
// 0..s-1 of every job, one workgroup of T threads per job.  Row r < T lives
// in the registers of thread r; with T = 1024, rows 1024.. (at most
// kPanelLds of them) in LDS, handled by thread r - 1024.  The scaled pivot
// row of every step goes to spr, for the rows >= s (kg_replay).
constexpr int kPanelLds = kGJMaxPivots - kPanelT;

__device__ __forceinline__ void pivot_better(float& best, int& bi, float v, int r) {
  if (v > best || (v == best && r < bi)) {
    best = v;
    bi = r;
  }
}

template <int T>
__global__ void __launch_bounds__(T) kg_panel(const GJob* __restrict__ jobs, int k0, int* status) {
  const GJob jb = jobs[blockIdx.x];
  const int n = jb.s;
  if (k0 >= n) return;
  const int nbv = min(kNB, n - k0);
  const int ld = jb.ld;
  cf* S = jb.F;
  constexpr int kL = (T == kPanelT) ? kPanelLds : 1;  // rows held in LDS
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ cf prow[kNB], srow[kNB], spr[kNB];
  __shared__ cf P2[kL][kNB + 1];
  __shared__ float wbest[T / 64];
  __shared__ int widx[T / 64];
  __shared__ int sh_p;
  const int r1 = tid, r2 = T + tid;  // the thread's rows
  const bool has1 = r1 < n, has2 = T == kPanelT && tid < kPanelLds && r2 < n;
  cf P[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) P[c] = (has1 && c < nbv) ? S[(size_t)r1 * ld + k0 + c] : mk<float>(0, 0);
  if (T == kPanelT && tid < kPanelLds)
    for (int c = 0; c < kNB; ++c) P2[tid][c] = (has2 && c < nbv) ? S[(size_t)r2 * ld + k0 + c] : mk<float>(0, 0);
  bool bad = false;
#pragma clang loop unroll(full)
  for (int c = 0; c < kNB; ++c) {
    if (c < nbv) {  // uniform
      const int gc = k0 + c;
      // pivot: largest |entry| of column gc among the rows not yet pivotal
      float best = -1.0f;
      int bi = n;
      if (has1 && r1 >= gc) pivot_better(best, bi, P[c].re * P[c].re + P[c].im * P[c].im, r1);
      if (has2 && r2 >= gc) pivot_better(best, bi, abs2(P2[tid][c]), r2);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        pivot_better(best, bi, ov, oi);
      }
      if (lane == 0) {
        wbest[wv] = best;
        widx[wv] = bi;
      }
      __syncthreads();
      if (tid < 64) {
        float b2 = tid < T / 64 ? wbest[tid] : -1.0f;
        int i2 = tid < T / 64 ? widx[tid] : n;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const float ov = __shfl_xor(b2, off, 64);
          const int oi = __shfl_xor(i2, off, 64);
          pivot_better(b2, i2, ov, oi);
        }
        if (tid == 0) {
          if (!(b2 > 0.0f) || !isfinite(b2) || i2 >= n) {
            bad = true;
            i2 = gc;
          }
          sh_p = i2;
          jb.piv[gc] = i2;
        }
      }
      __syncthreads();
      const int p = sh_p;
      // interchange rows gc and p of the panel (through LDS)
      if (r1 == p) {
#pragma unroll
        for (int q = 0; q < kNB; ++q) prow[q] = P[q];
      }
      if (has2 && r2 == p)
        for (int q = 0; q < kNB; ++q) prow[q] = P2[tid][q];
      if (p != gc) {
        if (r1 == gc) {
#pragma unroll
          for (int q = 0; q < kNB; ++q) srow[q] = P[q];
        }
        if (has2 && r2 == gc)
          for (int q = 0; q < kNB; ++q) srow[q] = P2[tid][q];
      }
      __syncthreads();
      if (tid < kNB) {
        // scaled pivot row: entries / pivot, the pivot entry replaced by 1 / pivot
        const cf pv = prow[c];
        const float d = 1.0f / (pv.re * pv.re + pv.im * pv.im);
        const cf inv = mk<float>(pv.re * d, -pv.im * d);
        const cf v = (tid == c) ? inv : prow[tid] * inv;
        spr[tid] = v;
        jb.spr[c * kNB + tid] = v;
      }
      if (p != gc) {
        if (r1 == p) {
#pragma unroll
          for (int q = 0; q < kNB; ++q) P[q] = srow[q];
        }
        if (has2 && r2 == p)
          for (int q = 0; q < kNB; ++q) P2[tid][q] = srow[q];
      }
      __syncthreads();
      // elimination of column gc from every other row
      if (has1) {
        if (r1 == gc) {
#pragma unroll
          for (int q = 0; q < kNB; ++q) P[q] = spr[q];
        } else {
          const cf f = P[c];
#pragma unroll
          for (int q = 0; q < kNB; ++q) {
            const cf base = (q == c) ? mk<float>(0, 0) : P[q];
            const cf sp = spr[q];
            P[q] = mk<float>(base.re - (f.re * sp.re - f.im * sp.im), base.im - (f.re * sp.im + f.im * sp.re));
          }
        }
      }
      if (has2) {
        if (r2 == gc) {
          for (int q = 0; q < kNB; ++q) P2[tid][q] = spr[q];
        } else {
          const cf f = P2[tid][c];
          for (int q = 0; q < kNB; ++q) {
            const cf base = (q == c) ? mk<float>(0, 0) : P2[tid][q];
            const cf sp = spr[q];
            P2[tid][q] = mk<float>(base.re - (f.re * sp.re - f.im * sp.im), base.im - (f.re * sp.im + f.im * sp.re));
          }
        }
      }
      __syncthreads();  // prow / spr are rewritten by the next column
    }
  }
  if (has1) {
#pragma unroll
    for (int c = 0; c < kNB; ++c)
      if (c < nbv) S[(size_t)r1 * ld + k0 + c] = P[c];
  }
  if (has2)
    for (int c = 0; c < nbv; ++c) S[(size_t)r2 * ld + k0 + c] = P2[tid][c];
  if (bad) atomicOr(status, 1);
}

// The panel steps replayed on the rows s..nf-1 (never pivot candidates):
// the same eliminations with the scaled pivot rows kg_panel recorded.
__global__ void __launch_bounds__(256) kg_replay(const GJob* __restrict__ jobs, int k0) {
  const GJob jb = jobs[blockIdx.y];
  if (k0 >= jb.s) return;
  const int nbv = min(kNB, jb.s - k0);
  __shared__ cf sp[kNB][kNB];
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int c = e / kNB, q = e - (e / kNB) * kNB;
    sp[c][q] = (c < nbv && q < nbv) ? jb.spr[e] : mk<float>(0, 0);
  }
  __syncthreads();
  const int r = jb.s + blockIdx.x * 256 + threadIdx.x;
  if (r >= jb.nf) return;
  cf* row = jb.F + (size_t)r * jb.ld + k0;
  cf P[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) P[c] = c < nbv ? row[c] : mk<float>(0, 0);
#pragma unroll
  for (int c = 0; c < kNB; ++c) {
    if (c < nbv) {
      const cf f = P[c];
#pragma unroll
      for (int q = 0; q < kNB; ++q) {
        const cf base = (q == c) ? mk<float>(0, 0) : P[q];
        const cf v = sp[c][q];
        P[q] = mk<float>(base.re - (f.re * v.re - f.im * v.im), base.im - (f.re * v.im + f.im * v.re));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kNB; ++c)
    if (c < nbv) row[c] = P[c];
}

// Row interchanges of the panel applied to the other columns, and the pivot
// rows of those columns copied to brow[c][j] (zero in the panel columns).
__global__ void __launch_bounds__(256) kg_swap(const GJob* __restrict__ jobs, int k0) {
  const GJob jb = jobs[blockIdx.y];
  if (k0 >= jb.s) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= jb.nf) return;
  const int nbv = min(kNB, jb.s - k0);
  const int ld = jb.ld;
  cf* S = jb.F;
  const bool panel = j >= k0 && j < k0 + nbv;
  for (int c = 0; c < kNB; ++c) {
    cf v = mk<float>(0, 0);
    if (c < nbv && !panel) {
      const int gc = k0 + c, p = jb.piv[gc];
      if (p != gc) {
        const cf a = S[(size_t)gc * ld + j];
        v = S[(size_t)p * ld + j];
        S[(size_t)p * ld + j] = a;
        S[(size_t)gc * ld + j] = v;
      } else {
        v = S[(size_t)gc * ld + j];
      }
    }
    jb.brow[(size_t)c * ld + j] = v;
  }
}

// R <- R + P' B_K over the columns outside the panel (all nf rows), with
// the pivot rows of R replaced (not incremented).  64 x 64 output tile per
// workgroup, a 32 x 32 tile per wavefront on the FP32 matrix cores.
__global__ void __launch_bounds__(256) kg_update(const GJob* __restrict__ jobs, int k0, int tiles) {
  const GJob jb = jobs[blockIdx.y];
  const int n = jb.nf;
  if (k0 >= jb.s) return;
  const int nbv = min(kNB, jb.s - k0);
  const int ti = blockIdx.x / tiles, tj = blockIdx.x - (blockIdx.x / tiles) * tiles;
  const int i0 = ti * 64, j0 = tj * 64;
  if (i0 >= n || j0 >= n) return;
  const int ld = jb.ld;
  cf* S = jb.F;
  const cf* B = jb.brow;
  __shared__ cf sA[64][kNB + 1];
  __shared__ cf sB[kNB][64];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * kNB; e += 256) {
    const int r = e / kNB, c = e - (e / kNB) * kNB;
    const int i = i0 + r;
    sA[r][c] = (i < n && c < nbv) ? S[(size_t)i * ld + k0 + c] : mk<float>(0, 0);
  }
  for (int e = tid; e < 64 * kNB; e += 256) {
    const int c = e / 64, q = e - (e / 64) * 64;
    const int j = j0 + q;
    sB[c][q] = (j < n && c < nbv) ? B[(size_t)c * ld + j] : mk<float>(0, 0);
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;
  floatx16 are, aim;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    are[v] = 0.0f;
    aim[v] = 0.0f;
  }
  // operand layout of v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32]
  // and B[l / 32][l % 32] of the 32 x 2 and 2 x 32 factors
#pragma unroll
  for (int kk = 0; kk < kNB / 2; ++kk) {
    const cf a = sA[rb + (lane & 31)][2 * kk + (lane >> 5)];
    const cf b = sB[2 * kk + (lane >> 5)][cb + (lane & 31)];
    are = __builtin_amdgcn_mfma_f32_32x32x2f32(a.re, b.re, are, 0, 0, 0);
    are = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.im, b.im, are, 0, 0, 0);
    aim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.re, b.im, aim, 0, 0, 0);
    aim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.im, b.re, aim, 0, 0, 0);
  }
  // result layout: lane l, register v holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]
  const int j = j0 + cb + (lane & 31);
  const bool colok = j < n && !(j >= k0 && j < k0 + nbv);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + rb + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (colok && i < n) {
      const bool pivrow = i >= k0 && i < k0 + nbv;
      const cf old = pivrow ? mk<float>(0, 0) : S[(size_t)i * ld + j];
      S[(size_t)i * ld + j] = mk<float>(old.re + are[v], old.im + aim[v]);
    }
  }
}

// Column permutation of the eliminated columns: the row interchanges in
// reverse order become column interchanges; col[j] = the column of the
// eliminated matrix that is column j of F11^{-1}.
__global__ void __launch_bounds__(64) kg_colperm(const GJob* __restrict__ jobs) {
  const GJob jb = jobs[blockIdx.x];
  const int n = jb.s;
  for (int j = threadIdx.x; j < n; j += 64) jb.col[j] = j;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = n - 1; c >= 0; --c) {
      const int p = jb.piv[c];
      if (p != c) {
        const int a = jb.col[c];
        jb.col[c] = jb.col[p];
        jb.col[p] = a;
      }
    }
}

// Store G_t, M_t = -G_t L_t and E_t = G_t U_t of block t.
__global__ void __launch_bounds__(256) k3_store(Setup3 Su, int t) {
  const Slab3 sl = Su.slabs[blockIdx.y];
  const int n = sl.n;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx - (idx / n) * n);
  const int m3 = sl.op.m3, nl = sl.nl;
  const int ld = Su.n_max;
  const cf* Sr = Su.S + ((size_t)blockIdx.y * ld + i) * ld;
  const int* col = Su.col + (size_t)blockIdx.y * Su.n_max;
  const cf* cfs = Su.coef + (size_t)blockIdx.y * Su.n_max * 27;
  cf* W = Wblk(Su.factors, sl, t);
  cf* E = W + (size_t)2 * n * n;
  const int xj = j / m3, zj = j - (j / m3) * m3;
  const cf g = Sr[col[j]];
  cf mv = mk<float>(0, 0), ev = mk<float>(0, 0);
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
    const int xr = xj - a;
    if (xr < 0 || xr >= nl) continue;
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      const int zr = zj - b;
      if (zr < 0 || zr >= m3) continue;
      const int r = xr * m3 + zr;  // row r of block t couples to column j of the neighbour planes
      const cf gr = Sr[col[r]];
      const cf l = cfs[(size_t)r * 27 + (a + 1) * 9 + 0 + (b + 1)];
      const cf u = cfs[(size_t)r * 27 + (a + 1) * 9 + 6 + (b + 1)];
      mv.re -= gr.re * l.re - gr.im * l.im;
      mv.im -= gr.re * l.im + gr.im * l.re;
      ev.re += gr.re * u.re - gr.im * u.im;
      ev.im += gr.re * u.im + gr.im * u.re;
    }
  }
  W[(size_t)i * 2 * n + j] = g;
  W[(size_t)i * 2 * n + n + j] = mv;
  E[(size_t)i * padded(n) + j] = ev;
}

__global__ void k3_growth(Setup3 Su, double* growth) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Su.nslabs) return;
  const double b = Su.gmax[2 * s], a = Su.gmax[2 * s + 1];
  growth[s] = b > 0 ? sqrt(a / b) : 0.0;
}

// ---- sweep stage ---------------------------------------------------------------

// Slab right-hand side of every task: f_d = J(j, a, b) f (or g) plus the
// transmission terms (T B, T~ B) on the four incoming layers; slab-layout
// input for mode 1.  fs[task][t][q], block stride padded(n_max).
__global__ void __launch_bounds__(256) k3s_prep(Stage3 st) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const Slab3 sl = st.slabs[tk.slab];
  const int m2 = st.G.m2, m3 = st.G.m3, n = sl.n;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  if (idx >= (size_t)m2 * n) return;
  const int t = (int)(idx / n), q = (int)(idx - (idx / n) * n);
  const int xl = q / m3, z = q - (q / m3) * m3;
  const int gl = sl.x0 + xl;
  const size_t pl = (size_t)m2 * m3;
  cd v = mk<double>(0, 0);
  if (tk.mode == 1) {
    v = cvt<double>(st.f[((size_t)xl * m2 + t) * m3 + z]);
  } else {
    const cf* src = tk.src ? st.g : st.f;
    if (gl > tk.a && gl <= tk.b) v = cvt<double>(src[((size_t)(gl - 1) * m2 + t) * m3 + z]);
    const bool inF = tk.t1 && (gl == tk.beta_in || gl == tk.beta_in + 1);
    const bool inB = tk.t3 && (gl == tk.bt_in || gl == tk.bt_in + 1);
    if (inF || inB) {
      cd c[27];
      coefs27(st.G, gl, t + 1, z + 1, c);
      for (int side = 0; side < 2; ++side) {
        if (side == 0 && !inF) continue;
        if (side == 1 && !inB) continue;
        const cf* Bi = st.bufs + (size_t)(side == 0 ? tk.bin_f : tk.bin_b) * 2 * pl;
        const int s = side == 0 ? (gl == tk.beta_in ? 1 : 0) : (gl == tk.bt_in ? 1 : 0);
        const int dxc = s == 1 ? 2 : 0;  // coupling to layer gl + 1 or gl - 1
        cd a = mk<double>(0, 0);
        for (int dy = -1; dy <= 1; ++dy) {
          const int tt = t + dy;
          if (tt < 0 || tt >= m2) continue;
          for (int dz = -1; dz <= 1; ++dz) {
            const int zz = z + dz;
            if (zz < 0 || zz >= m3) continue;
            cfma(a, c[dxc * 9 + (dy + 1) * 3 + (dz + 1)], cvt<double>(Bi[(size_t)s * pl + (size_t)tt * m3 + zz]));
          }
        }
        // T adds +A_{b,b+1} B[1] on layer b and -A_{b+1,b} B[0] on b+1; T~ the opposite signs
        const bool plus = (side == 0) ? (s == 1) : (s == 0);
        v = plus ? v + a : v - a;
      }
    }
  }
  st.fs[(size_t)blockIdx.y * m2 * padded(st.n_max) + (size_t)t * padded(st.n_max) + q] = cvt<float>(v);
}

// One block step of the substitutions of every task (one launch per step:
// the steps depend on each other through the whole vector y_{t-1} or
// x_{t+1}).  Each wavefront forms one row, four rows per workgroup; every
// lane issues all of its loads of the row (pairs of complex entries, 16
// bytes each) at once, before the input vector is staged in LDS, so that a
// step keeps its whole factor block in flight.
//   forward  (FWD): y_t = [G_t | M_t] [f_t ; y_{t-1}]
//   backward:       x_t = y_t - E_t x_{t+1}   (in place over y_t)
constexpr int kRowsPerBlock = 4;

// Pairs c < npair of the row (pair c = entries 2c, 2c + 1; an odd row
// length reads one entry past the row, which meets a zero of the staged
// input vector).
template <int NP>
__device__ __forceinline__ void load_row(floatx4 (&a)[NP], const cf* row, int npair, int lane) {
  const floatx4* w = reinterpret_cast<const floatx4*>(row) + lane;
#pragma unroll
  for (int k = 0; k < NP; ++k)
    a[k] = (lane + 64 * k < npair) ? __builtin_nontemporal_load(w + 64 * k) : floatx4{0.f, 0.f, 0.f, 0.f};
}

template <int NP>
__device__ __forceinline__ cf row_dot(const floatx4 (&a)[NP], const cf* vin, int npair, int lane) {
  const floatx4* vv = reinterpret_cast<const floatx4*>(vin) + lane;
  float ar = 0, ai = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (lane + 64 * k < npair) {
      const floatx4 x = vv[64 * k];
      ar += a[k].x * x.x - a[k].y * x.y + a[k].z * x.z - a[k].w * x.w;
      ai += a[k].x * x.y + a[k].y * x.x + a[k].z * x.w + a[k].w * x.z;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  return mk<float>(ar, ai);
}

// NP: pairs of complex entries per lane and row (rows of up to 128 NP
// entries: [G_t | M_t] has 2n, E_t has n).
template <bool FWD, int NP>
__global__ void __launch_bounds__(256) k3s_step(Stage3 st, int t) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const Slab3 sl = st.slabs[tk.slab];
  const int n = sl.n, m2 = st.G.m2;
  const int i0 = blockIdx.x * kRowsPerBlock;
  if (i0 >= n) return;
  const int ldv = padded(st.n_max);
  const cf* fs = st.fs + (size_t)blockIdx.y * m2 * ldv;
  cf* ys = st.ys + (size_t)blockIdx.y * m2 * ldv;
  __shared__ __align__(16) cf vin[128 * NP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = i0 + wv;
  const bool ok = r < n;
  const int rr = ok ? r : 0;
  floatx4 a[NP];
  const int nin = (FWD && t > 0) ? 2 * n : n;
  const int npair = (nin + 1) / 2;
  if (FWD)
    load_row(a, Wblk(st.factors, sl, t) + (size_t)rr * 2 * n, npair, lane);
  else
    load_row(a, Wblk(st.factors, sl, t) + (size_t)2 * n * n + (size_t)rr * padded(n), npair, lane);
  for (int e = tid; e < 2 * npair; e += 256) {
    cf v = mk<float>(0, 0);
    if (FWD) {
      if (e < n)
        v = fs[(size_t)t * ldv + e];
      else if (e < 2 * n && t > 0)
        v = ys[(size_t)(t - 1) * ldv + e - n];
    } else if (e < n) {
      v = ys[(size_t)(t + 1) * ldv + e];
    }
    vin[e] = v;
  }
  __syncthreads();
  const cf d = row_dot(a, vin, npair, lane);
  if (lane == 0 && ok) {
    cf* y = ys + (size_t)t * ldv + r;
    if (FWD) {
      *y = d;
    } else {
      const cf o = *y;
      *y = mk<float>(o.re - d.re, o.im - d.im);
    }
  }
}

// u += J(j, a~, b~)^T x over the layers a~+1..b~, outgoing transmission
// layers, or the slab-layout result (mode 1).
__global__ void __launch_bounds__(256) k3s_fin(Stage3 st) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const Slab3 sl = st.slabs[tk.slab];
  const int m2 = st.G.m2, m3 = st.G.m3, n = sl.n;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  if (idx >= (size_t)m2 * n) return;
  const int t = (int)(idx / n), q = (int)(idx - (idx / n) * n);
  const int xl = q / m3, z = q - (q / m3) * m3;
  const int gl = sl.x0 + xl;
  const size_t pl = (size_t)m2 * m3;
  const cf x = st.ys[(size_t)blockIdx.y * m2 * padded(st.n_max) + (size_t)t * padded(st.n_max) + q];
  if (tk.mode == 1) {
    st.u[((size_t)xl * m2 + t) * m3 + z] = x;
    return;
  }
  if (gl > tk.at && gl <= tk.bt) {
    cf* up = st.u + ((size_t)(gl - 1) * m2 + t) * m3 + z;
    *up = *up + x;
  }
  const size_t o = (size_t)t * m3 + z;
  if (tk.t2) {
    cf* Bo = st.bufs + (size_t)tk.bout_f * 2 * pl;
    if (gl == tk.beta_out) Bo[o] = x;
    if (gl == tk.beta_out + 1) Bo[pl + o] = x;
  }
  if (tk.t4) {
    cf* Bo = st.bufs + (size_t)tk.bout_b * 2 * pl;
    if (gl == tk.bt_out) Bo[o] = x;
    if (gl == tk.bt_out + 1) Bo[pl + o] = x;
  }
}

}  // namespace

void launch_gauss_jordan(const GJob* jobs, int njobs, int s_max, int b_max, int nf_max, int* status,
                         hipStream_t s) {
  if (njobs < 1 || s_max < 1) return;
  const int tiles = (nf_max + 63) / 64;
  for (int k0 = 0; k0 < s_max; k0 += kNB) {
    if (s_max > 256)
      hipLaunchKernelGGL(kg_panel<kPanelT>, dim3(njobs), dim3(kPanelT), 0, s, jobs, k0, status);
    else
      hipLaunchKernelGGL(kg_panel<256>, dim3(njobs), dim3(256), 0, s, jobs, k0, status);
    if (b_max > 0) hipLaunchKernelGGL(kg_replay, dim3((b_max + 255) / 256, njobs), dim3(256), 0, s, jobs, k0);
    hipLaunchKernelGGL(kg_swap, dim3((nf_max + 255) / 256, njobs), dim3(256), 0, s, jobs, k0);
    hipLaunchKernelGGL(kg_update, dim3(tiles * tiles, njobs), dim3(256), 0, s, jobs, k0, tiles);
  }
  hipLaunchKernelGGL(kg_colperm, dim3(njobs), dim3(64), 0, s, jobs);
}

size_t setup3_scratch_bytes(int nslabs, int n_max) {
  const size_t nm = (size_t)n_max;
  // eight arrays, each 256-byte aligned
  return nslabs * (nm * nm * sizeof(cf) + nm * 27 * sizeof(cf) + kNB * nm * sizeof(cf) + kNB * kNB * sizeof(cf) +
                   2 * nm * sizeof(int) + sizeof(GJob) + 2 * sizeof(double)) + 8 * 256;
}

void setup3_jobs(const Setup3& Su, const int* n, GJob* jobs) {
  const size_t nm = (size_t)Su.n_max;
  for (int sl = 0; sl < Su.nslabs; ++sl) {
    GJob& jb = jobs[sl];
    jb.F = Su.S + (size_t)sl * nm * nm;
    jb.nf = jb.s = n[sl];
    jb.ld = Su.n_max;
    jb.piv = Su.piv + (size_t)sl * nm;
    jb.col = Su.col + (size_t)sl * nm;
    jb.brow = Su.brow + (size_t)sl * kNB * nm;
    jb.spr = Su.spr + (size_t)sl * kNB * kNB;
  }
}

void launch_factor3(const Setup3& Su, hipStream_t s) {
  const int ns = Su.nslabs, nm = Su.n_max;
  const size_t nn = (size_t)nm * nm;
  for (int t = 0; t < Su.m2; ++t) {
    hipLaunchKernelGGL(k3_coef, dim3((nm + 255) / 256, ns), dim3(256), 0, s, Su, t);
    hipLaunchKernelGGL(k3_schur, dim3(nblk(nn), ns), dim3(256), 0, s, Su, t);
    launch_gauss_jordan(Su.jobs, ns, nm, 0, nm, Su.status, s);
    hipLaunchKernelGGL(k3_store, dim3(nblk(nn), ns), dim3(256), 0, s, Su, t);
  }
}

void finish_growth3(const Setup3& Su, double* growth, hipStream_t s) {
  hipLaunchKernelGGL(k3_growth, dim3((Su.nslabs + 63) / 64), dim3(64), 0, s, Su, growth);
}

hipError_t launch_stage3(const Stage3& st, hipStream_t s) {
  if (st.ntasks < 1) return hipSuccess;
  const size_t cnt = (size_t)st.G.m2 * st.n_max;
  const int m2 = st.G.m2;
  hipLaunchKernelGGL(k3s_prep, dim3(nblk(cnt), st.ntasks), dim3(256), 0, s, st);
  if (st.nd) {
    launch_nd_solve(st, *st.nd, *st.nd_lv, s);
    hipLaunchKernelGGL(k3s_fin, dim3(nblk(cnt), st.ntasks), dim3(256), 0, s, st);
    return hipGetLastError();
  }
  const dim3 grd((st.n_max + kRowsPerBlock - 1) / kRowsPerBlock, st.ntasks);
  // pairs per lane: n_max (forward rows of 2 n_max entries), n_max / 2 (backward)
  const int npf = (st.n_max + 63) / 64, npb = (st.n_max + 127) / 128;
#define FWD_STEPS(NP)                                                                                 \
  for (int t = 0; t < m2; ++t) hipLaunchKernelGGL((k3s_step<true, NP>), grd, dim3(256), 0, s, st, t)
#define BWD_STEPS(NP)                     \
  for (int t = m2 - 2; t >= 0; --t) hipLaunchKernelGGL((k3s_step<false, NP>), grd, dim3(256), 0, s, st, t)
  if (npf <= 8)
    FWD_STEPS(8);
  else if (npf <= 16)
    FWD_STEPS(16);
  else if (npf <= 20)
    FWD_STEPS(20);
  else
    FWD_STEPS(24);
  if (npb <= 4)
    BWD_STEPS(4);
  else if (npb <= 8)
    BWD_STEPS(8);
  else
    BWD_STEPS(12);
#undef FWD_STEPS
#undef BWD_STEPS
  hipLaunchKernelGGL(k3s_fin, dim3(nblk(cnt), st.ntasks), dim3(256), 0, s, st);
  return hipGetLastError();
}


}  // namespace d3
}  // namespace hsp
