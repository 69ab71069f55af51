// Batched SubdomSolve stages: the slab solves of one sweep stage applied to
// many right-hand sides at once (the multi-RHS pipelining of Sec. 5, where
// the factors of a slab are shared by every source).
//
// Work items are (task of the stage, chunk of the tangential axis, tile of
// RB right-hand sides); every launch covers all of them, so one stage is two
// launches whatever the number of right-hand sides.  Within a tile the block
// substitutions act on nl x RB blocks:
//   forward   y_t = G_t (f_t - A_t y_{t-1})         (A_t: coupling to t-1),
//   backward  x_t = y_t - E_t x_{t+1},
// chunked: each work item runs both chunk-local chains from zero, the forward
// one on its right-hand side and the backward one on the forward result, so
// that with c_{p-1} the true forward value at the end of the previous chunk
// and d_{p+1} the true backward value at the start of the next one,
//   x_t = x_t(local) + W_t c_{p-1} + X_t d_{p+1}
// (W_t: the local backward chain applied to the forward transfer matrices
// Y_t).  The last work item of a slot to arrive runs the chain over the chunk
// ends (c through Y), corrects the chunk starts by W, and runs the chain over
// the chunk starts (d through X); the second launch applies both terms to
// every block and scatters.  The factor blocks of a chunk are read
// once per tile; the tiles of one chunk are placed on the same XCD so that
// they share its L2.
//
// Scratch per (task, tile) slot: y [n2][RB][nl] (right-hand side, then the
// solution), chunk tips and heads [2][P][RB][nl], an arrival counter (of
// two reserved).  Where a chunk's slice of y fits in 64 KB of LDS, each work
// item keeps it there within a launch: y in global memory then only carries
// the chunk-local solution from the forward to the backward launch.
#include "internal.h"
#include "sweep_dev.h"

namespace hsp {

namespace {

// Pointers taken from the segment table are generic (flat) to the compiler;
// flat loads count against the LDS wait counter too, so every LDS wait of a
// chain step would also wait for the loads prefetched for later steps.
// Casting them to the global address space keeps the two counters apart.
// (The host pass of the same source only parses the kernels; there the
// qualifier is left out.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GAS __attribute__((address_space(1)))
#define CAS __attribute__((address_space(4)))
#else
#define GAS
#define CAS
#endif
template <class X>
__device__ __forceinline__ GAS X* gp(X* p) {
  return (GAS X*)p;
}
template <class X>
__device__ __forceinline__ const GAS X* gp(const X* p) {
  return (const GAS X*)p;
}
// Task and slab descriptors are read-only for the whole launch and the same
// for every thread of a workgroup: read them as constants (scalar loads, so
// that the index arithmetic derived from them stays scalar).
template <class X>
__device__ __forceinline__ X cload(const X* p, int i) {
  return ((const CAS X*)p)[i];
}

// Thread layout of a 256-thread workgroup for slabs of up to NC <= NB
// layers, NB (32 or 64) the row lanes.  Product phase: thread (l, g),
// l = tid % NB, owns row l and the CW columns [g CW, (g+1) CW) of a block, the
// first NC columns split over the NG groups (NC < NB trims the work of slabs
// that are thinner than NB).  Reduction phase: thread (l, g) owns row l of
// the right-hand sides g, g + NG, ... (RC of them).  The product input q has
// QN = max(NB, NG CW) rows, the rows from nl on kept zero.
template <int NB, int RB, int NC = NB>
struct BLay {
  static_assert(NC <= NB && 64 % NB == 0, "row lanes must divide the wavefront");
  static constexpr int NT = 256;
  static constexpr int NG = NT / NB;
  static constexpr int CW = (NC + NG - 1) / NG;
  static constexpr int QR = NG * CW;
  static constexpr int QN = QR > NB ? QR : NB;
  static constexpr int RC = (RB + NG - 1) / NG;
};

template <class T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v, int width) {
  return mk<T>(__shfl_up(v.re, 1, width), __shfl_up(v.im, 1, width));
}
template <class T>
__device__ __forceinline__ cx<T> shfl_down1(cx<T> v, int width) {
  return mk<T>(__shfl_down(v.re, 1, width), __shfl_down(v.im, 1, width));
}

// Block chain over the RB columns of a tile, by the whole workgroup.  Step k
// (k = 0..count-1) uses the index r = first + dir k:
//   GD = false:  Z_k = B_k + sigma Mat_r Z_{k-1}
//   GD = true:   Z_k = Mat_r (B_k - Cpl_r Z_{k-1})
// with Z_{-1} = 0, Mat_r the column-major nl x nl block at mat + r mstride
// and Cpl_r the tridiagonal coupling (Cpl Z)[l] = sum_a cpl[r][a][l] Z[l+a-1].
// B_k is read from, and Z_k written to, rows[((r - rbase) RB + c) nl + l]
// (rows in global memory or a chunk's slice in LDS).  The matrix
// slices (and B, couplings) of the next D steps are held in a register ring;
// loads are unconditional from clamped addresses.  LDS: q [NB][RB] holds the
// product input, ps [NG][RB][NB] the partial products.
template <class T, int NB, int RB, int D, bool GD, int NC = NB, class R>
__device__ __forceinline__ void bchain(const GAS cx<T>* __restrict__ mat, long mstride,
                                       const GAS cx<T>* __restrict__ cpl, R rows, int rbase, int first, int dir,
                                       int count, int nl, T sigma, cx<T>* q, cx<T>* ps) {
  using LY = BLay<NB, RB, NC>;
  constexpr int NG = LY::NG, CW = LY::CW, RC = LY::RC, QR = LY::QR;
  if (count <= 0) return;
  const int tid = threadIdx.x;
  const int l = tid % NB, g = tid / NB;
  const bool act = l < nl;
  const int lc = act ? l : nl - 1;
  cx<T> rm[D][CW];
  cx<T> rb[D][RC];
  cx<T> ra[D][3];
  // Ring slot d of step kk holds Mat_{r_kk} and what the reduction of step kk
  // needs: GD: B and couplings of step kk+1 (the next input); else B_kk.
  // The loads are plain loads from clamped (valid) addresses; masks are
  // applied where the values are consumed, so that no wait for a load is
  // placed right after it.  Matrix entries of columns j >= nl meet zero
  // product inputs (q rows >= nl are kept zero), rows l >= nl are masked.
#define BCH_FETCH(kk, d)                                                                         \
  {                                                                                              \
    const int kc = (kk) < count ? (kk) : count - 1;                                              \
    const GAS cx<T>* Mk = mat + (long)(first + dir * kc) * mstride;                                  \
    _Pragma("unroll") for (int cc = 0; cc < CW; ++cc) {                                          \
      const int j = g * CW + cc;                                                                 \
      const int jc = j < nl ? j : nl - 1;                                                        \
      rm[d][cc] = Mk[(size_t)jc * nl + lc];                                                      \
    }                                                                                            \
    const int kb = GD ? ((kk) + 1 < count ? (kk) + 1 : count - 1) : kc;                          \
    const int rbi = first + dir * kb;                                                            \
    _Pragma("unroll") for (int i = 0; i < RC; ++i) {                                             \
      const int c = g + NG * i;                                                                  \
      const int ccl = c < RB ? c : RB - 1;                                                       \
      rb[d][i] = rows[((size_t)(rbi - rbase) * RB + ccl) * nl + lc];                             \
    }                                                                                            \
    if constexpr (GD) {                                                                          \
      _Pragma("unroll") for (int a = 0; a < 3; ++a) ra[d][a] = cpl[((size_t)rbi * 3 + a) * nl + lc]; \
    }                                                                                            \
  }
#define BCH_STEP(k, d)                                                                           \
  {                                                                                              \
    {                                                                                            \
      cx<T> part[RB];                                                                            \
      _Pragma("unroll") for (int c = 0; c < RB; ++c) part[c] = mk<T>(0, 0);                      \
      _Pragma("unroll") for (int cc = 0; cc < CW; ++cc) {                                        \
        const cx<T>* qr = q + (g * CW + cc) * RB;                                                \
        _Pragma("unroll") for (int c = 0; c < RB; ++c) cfma(part[c], rm[d][cc], qr[c]);          \
      }                                                                                          \
      _Pragma("unroll") for (int c = 0; c < RB; ++c) ps[(g * RB + c) * NB + l] = part[c];        \
    }                                                                                            \
    __syncthreads();                                                                             \
    const int rk = first + dir * (k);                                                            \
    _Pragma("unroll") for (int i = 0; i < RC; ++i) {                                             \
      const int c = g + NG * i;                                                                  \
      const int ccl = c < RB ? c : RB - 1;                                                       \
      cx<T> s = mk<T>(0, 0);                                                                     \
      _Pragma("unroll") for (int gg = 0; gg < NG; ++gg) s += ps[(gg * RB + ccl) * NB + l];       \
      cx<T> zk;                                                                                  \
      if constexpr (GD)                                                                          \
        zk = s;                                                                                  \
      else                                                                                       \
        zk = mk<T>(rb[d][i].re + sigma * s.re, rb[d][i].im + sigma * s.im);                      \
      zk = sel(act && c < RB, zk);                                                               \
      if (act && c < RB) rows[((size_t)(rk - rbase) * RB + c) * nl + l] = zk;                    \
      cx<T> qn = zk;                                                                             \
      if constexpr (GD) {                                                                        \
        const cx<T> zl = sel(l > 0, shfl_up1(zk, NB));                                           \
        const cx<T> zr = sel(l + 1 < nl, shfl_down1(zk, NB));                                    \
        qn = rb[d][i];                                                                           \
        cfma(qn, -ra[d][0], zl);                                                                 \
        cfma(qn, -ra[d][1], zk);                                                                 \
        cfma(qn, -ra[d][2], zr);                                                                 \
        qn = sel(act && c < RB, qn);                                                             \
      }                                                                                          \
      if (c < RB) q[l * RB + c] = qn;                                                            \
    }                                                                                            \
    __syncthreads();                                                                             \
  }
  // first input: B_0 (GD) or zero; rows past NB of the product input (when
  // NG CW > NB) stay zero for the whole chain
  if constexpr (QR > NB) {
    for (int idx = tid; idx < (QR - NB) * RB; idx += 256) q[NB * RB + idx] = mk<T>(0, 0);
  }
#pragma unroll
  for (int i = 0; i < RC; ++i) {
    const int c = g + NG * i;
    const int ccl = c < RB ? c : RB - 1;
    cx<T> v = mk<T>(0, 0);
    if constexpr (GD) v = sel(act && c < RB, rows[((size_t)(first - rbase) * RB + ccl) * nl + lc]);
    if (c < RB) q[l * RB + c] = v;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) BCH_FETCH(d, d)
  __syncthreads();
  int k0 = 0;
  for (; k0 + D <= count; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      BCH_STEP(k0 + d, d)
      BCH_FETCH(k0 + d + D, d)
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (k0 + d < count) BCH_STEP(k0 + d, d)
  }
#undef BCH_STEP
#undef BCH_FETCH
}

// rows_{t - rbase} += Mat_t v for t in [s, e), v = LDS [nl][RB]; one (t, row) pair per
// thread and all RB columns at once.  The row of Mat_t is fetched in blocks
// of JB entries (unconditional loads from clamped addresses) so that each
// block costs one memory round trip.
template <class T, int RB, class R>
__device__ __forceinline__ void bfixup(const GAS cx<T>* __restrict__ mat, R rows, int rbase, int s, int e, int nl,
                                       const cx<T>* v) {
  constexpr int JB = sizeof(T) == 4 ? 32 : 16;
  const int cnt = e - s;
  for (int idx = threadIdx.x; idx < cnt * nl; idx += blockDim.x) {
    const int t = s + idx / nl, l = idx - (idx / nl) * nl;
    const GAS cx<T>* mb = mat + (size_t)t * nl * nl + l;
    const R o = rows + (size_t)(t - rbase) * RB * nl + l;
    cx<T> acc[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) acc[c] = o[(size_t)c * nl];
    for (int j0 = 0; j0 < nl; j0 += JB) {
      cx<T> mv[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj;
        const int jc = j < nl ? j : nl - 1;
        mv[jj] = sel(j < nl, mb[(size_t)jc * nl]);
      }
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj;
        if (j < nl) {  // the same for every thread: padding columns are skipped
#pragma unroll
          for (int c = 0; c < RB; ++c) cfma(acc[c], mv[jj], v[j * RB + c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RB; ++c) o[(size_t)c * nl] = acc[c];
  }
}

// rows_{t - rbase} += Mat1_t v1 + Mat2_t v2 for t in [s, e): both fix-ups of a block
// in one pass, the rows of the two matrices fetched together (one memory
// round trip per block of JB entries of both).
template <class T, int RB, class R>
__device__ __forceinline__ void bfixup2(const GAS cx<T>* __restrict__ m1, const cx<T>* v1,
                                        const GAS cx<T>* __restrict__ m2, const cx<T>* v2, R rows, int rbase,
                                        int s, int e, int nl) {
  constexpr int JB = sizeof(T) == 4 ? 32 : 16;
  const int cnt = e - s;
  for (int idx = threadIdx.x; idx < cnt * nl; idx += blockDim.x) {
    const int t = s + idx / nl, l = idx - (idx / nl) * nl;
    const GAS cx<T>* mb1 = m1 + (size_t)t * nl * nl + l;
    const GAS cx<T>* mb2 = m2 + (size_t)t * nl * nl + l;
    const R o = rows + (size_t)(t - rbase) * RB * nl + l;
    cx<T> acc[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) acc[c] = o[(size_t)c * nl];
    for (int j0 = 0; j0 < nl; j0 += JB) {
      cx<T> mv1[JB], mv2[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj;
        const int jc = j < nl ? j : nl - 1;
        mv1[jj] = sel(j < nl, mb1[(size_t)jc * nl]);
        mv2[jj] = sel(j < nl, mb2[(size_t)jc * nl]);
      }
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj;
        if (j < nl) {  // the same for every thread
#pragma unroll
          for (int c = 0; c < RB; ++c) {
            cfma(acc[c], mv1[jj], v1[j * RB + c]);
            cfma(acc[c], mv2[jj], v2[j * RB + c]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RB; ++c) o[(size_t)c * nl] = acc[c];
  }
}

// Chunk starts corrected for the true forward values of the previous chunk:
// heads_q += W_{s_q} tips_{q-1} for q = 1..P-1 (s_q = q m), by the whole
// workgroup.  The tip vectors are staged in buf (cap complex values) for as
// many chunks at a time as fit; one (chunk, row) pair per thread.
template <class T, int RB>
__device__ __forceinline__ void bheads_fix(const GAS cx<T>* __restrict__ W, GAS cx<T>* heads,
                                           const GAS cx<T>* tips, int P, int m, int nl, cx<T>* buf, int cap) {
  constexpr int JB = sizeof(T) == 4 ? 32 : 16;
  const int per = RB * nl;
  const int qg = cap / per > 0 ? cap / per : 1;
  for (int q0 = 1; q0 < P; q0 += qg) {
    const int q1 = min(P, q0 + qg);
    for (int idx = threadIdx.x; idx < (q1 - q0) * per; idx += blockDim.x) {
      const int qq = idx / per, rem = idx - qq * per;
      const int c = rem / nl, j = rem - c * nl;
      buf[qq * per + j * RB + c] = tips[((size_t)(q0 + qq - 1) * RB + c) * nl + j];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < (q1 - q0) * nl; idx += blockDim.x) {
      const int qq = idx / nl, l = idx - qq * nl;
      const GAS cx<T>* wr = W + (size_t)(q0 + qq) * m * nl * nl + l;
      GAS cx<T>* o = heads + (size_t)(q0 + qq) * RB * nl + l;
      const cx<T>* v = buf + qq * per;
      cx<T> acc[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] = o[(size_t)c * nl];
      for (int j0 = 0; j0 < nl; j0 += JB) {
        cx<T> mv[JB];
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
          const int j = j0 + jj;
          const int jc = j < nl ? j : nl - 1;
          mv[jj] = sel(j < nl, wr[(size_t)jc * nl]);
        }
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
          const int j = j0 + jj;
          if (j < nl) {  // the same for every thread
#pragma unroll
            for (int c = 0; c < RB; ++c) cfma(acc[c], mv[jj], v[j * RB + c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < RB; ++c) o[(size_t)c * nl] = acc[c];
    }
    __syncthreads();
  }
}

// Work item of block b: blocks are dealt to the 8 XCDs in turn, so block b
// takes item (b mod 8) per + b / 8; the tiles of one (task, chunk) pair are
// consecutive items and so share an XCD and its L2.  The segment is found by
// a scan over the (few) problems of the launch.
struct BWork {
  int q, p, tile;
};
__device__ __forceinline__ bool decode_work(const BSeg* __restrict__ segs, int nseg, int nitems, BSeg& S,
                                            BWork& w) {
  const int per = (nitems + 7) / 8;
  const int id = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (id >= nitems) return false;
  int k = nseg - 1;
  while (k > 0 && segs[k].item0 > id) --k;
  S = segs[k];
  const int local = id - S.item0;
  w.tile = local % S.ntiles;
  const int rest = local / S.ntiles;
  w.p = rest % S.P;
  w.q = rest / S.P;
  return true;
}

// Decomposition of a flat index i = (c nl + l) cnt + t (t fastest) that
// follows i -> i + 256 by carries instead of divisions.
struct IdxWalk {
  int c, l, t;
  int dc, dl, dt, cnt, nl;
  __device__ IdxWalk(int i, int cnt_, int nl_) : cnt(cnt_), nl(nl_) {
    const int row = i / cnt;
    t = i - row * cnt;
    c = row / nl;
    l = row - c * nl;
    const int drow = 256 / cnt;
    dt = 256 - drow * cnt;
    dc = drow / nl;
    dl = drow - dc * nl;
  }
  __device__ __forceinline__ void step() {
    t += dt;
    const int ct = t >= cnt;
    t -= ct ? cnt : 0;
    l += dl + ct;
    const int cl = l >= nl;
    l -= cl ? nl : 0;
    c += dc + cl;
  }
};

// Dynamic LDS of the stage kernels: with LY, the work item's chunk of the
// slab scratch, [cnt][RB][nl], for the whole launch (the forward launch
// writes it to y once at its end, the backward launch reads it once at its
// start); without, both kernels work on y in global memory.
extern __shared__ __align__(16) unsigned char bst_lds[];

// The rows of a work item's chunk: y_t at yrows<LY>(..)[((t - base) RB + c) nl + l],
// base = s in LDS, 0 in global memory.
template <bool LY, class T>
__device__ __forceinline__ auto yrows(GAS cx<T>* y) {
  if constexpr (LY)
    return reinterpret_cast<cx<T>*>(bst_lds);
  else
    return y;
}

template <class T, int NB, int RB, int D, int NC, bool LY>
__global__ void __launch_bounds__(256) k_bstage_fwd(const BSeg* __restrict__ segs, int nseg, int nitems) {
  __shared__ cx<T> q[BLay<NB, RB, NC>::QN * RB];
  __shared__ cx<T> ps[256 * RB];
  BWork w;
  BSeg A;
  if (!decode_work(segs, nseg, nitems, A, w)) return;
  const GAS cx<T>* __restrict__ f = gp(static_cast<const cx<T>*>(A.f));
  const GAS cx<T>* __restrict__ g = gp(static_cast<const cx<T>*>(A.g));
  const GAS cx<T>* __restrict__ bufs = gp(static_cast<const cx<T>*>(A.bufs));
  GAS cx<T>* __restrict__ scratch = gp(static_cast<cx<T>*>(A.scratch));
  const cx<T>* __restrict__ factors = static_cast<const cx<T>*>(A.factors);
  GAS cx<T>* __restrict__ red = gp(static_cast<cx<T>*>(A.red));
  int* counters = A.counters;
  const int P = A.P, m = A.m, n2 = A.G.n2;
  const int slot = w.q * A.ntiles + w.tile, r0 = w.tile * RB;
  const int nr = min(RB, A.nact - r0);
  const TaskDev tk = cload(A.tasks, w.q);
  const SlabDev sd = cload(A.slabs, tk.slab);
  const int nl = sd.nl;
  const int s = w.p * m, e = min(s + m, n2), cnt = e - s;
  const SlabFac<T> F(factors + sd.fac_off, n2, nl);
  GAS cx<T>* y = scratch + (size_t)slot * n2 * A.nl_max * RB;
  const auto yr = yrows<LY, T>(y);
  const int yb = LY ? s : 0;
  GAS cx<T>* tips = red + (size_t)slot * 2 * P * A.nl_max * RB;
  const GAS cx<T>* src = tk.src ? g : f;
  // slab right-hand side of the chunk, t fastest (coalesced level reads);
  // U entries per thread and round: all loads first, then the stores.  The
  // (at most four) incoming transmission layers are left to a second pass,
  // so that their coefficient evaluation runs only where it is needed.
  auto trans_layer = [&](int gl) {
    return (tk.t1 && (gl == tk.beta_in || gl == tk.beta_in + 1)) || (tk.t3 && (gl == tk.bt_in || gl == tk.bt_in + 1));
  };
  {
    constexpr int U = 4;
    IdxWalk it(threadIdx.x, cnt, nl);
    for (int base = threadIdx.x; base < RB * nl * cnt; base += 256 * U) {
      cx<T> val[U];
      int dst[U];
      bool st[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int gl = sd.x0 + it.l;
        const int cc = it.c < nr ? it.c : 0;
        const bool inside = it.c < nr && tk.a < gl && gl <= tk.b;
        const int glc = inside ? gl : tk.b;
        const cx<T> v = src[(size_t)(r0 + cc) * A.ld + (size_t)(glc - 1) * n2 + s + it.t];
        val[q] = sel(inside, v);
        dst[q] = ((s + it.t - yb) * RB + it.c) * nl + it.l;
        st[q] = it.c < RB && !trans_layer(gl);
        it.step();
      }
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (st[q]) yr[dst[q]] = val[q];
    }
  }
  // transmission layers from the precomputed coefficients: slot k < 2 is
  // layer beta_in + k, k >= 2 layer bt_in + k - 2; a layer that is listed
  // twice is written once (with both terms), one outside the slab not at all
  {
    const GAS cd* tc = gp(A.tcoef) + (size_t)w.q * trans_coef_elems(n2);
    auto slot_gl = [&](int kk) {
      return kk < 2 ? (tk.t1 ? tk.beta_in + kk : -1) : (tk.t3 ? tk.bt_in + kk - 2 : -1);
    };
    const int tot = RB * 4 * cnt;
    for (int idx = threadIdx.x; idx < tot; idx += 256) {
      const int c = idx / (4 * cnt), rem = idx - c * (4 * cnt);
      const int k = rem / cnt, t = s + rem - k * cnt;
      const int gl = slot_gl(k);
      bool use = gl >= sd.x0 && gl < sd.x0 + nl;
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2)
        if (k2 < k && slot_gl(k2) == gl) use = false;
      if (!use) continue;
      cx<T> v = mk<T>(0, 0);
      if (c < nr) {
        if (tk.a < gl && gl <= tk.b) v = src[(size_t)(r0 + c) * A.ld + (size_t)(gl - 1) * n2 + t];
        const GAS cx<T>* bz = bufs + (size_t)(r0 + c) * A.nbuf * 2 * n2;
        cd acc = mk<double>(0, 0);
        for (int k2 = k; k2 < 4; ++k2) {
          if (slot_gl(k2) != gl) continue;
          const GAS cx<T>* Bk = bz + (size_t)(k2 < 2 ? tk.bin_f : tk.bin_b) * 2 * n2 + ((k2 & 1) ? 0 : n2);
          const GAS cd* ck = tc + ((size_t)k2 * n2 + t) * 3;
#pragma unroll
          for (int dt = 0; dt < 3; ++dt) {
            const int tt = min(max(t + dt - 1, 0), n2 - 1);
            cfma(acc, ck[dt], cvt<double>(Bk[tt]));
          }
        }
        v = v + cvt<T>(acc);
      }
      yr[((size_t)(t - yb) * RB + c) * nl + (gl - sd.x0)] = v;
    }
  }
  __syncthreads();
  // chunk-local forward substitution y_t = G_t (f_t - A_t y_{t-1}) from zero
  bchain<T, NB, RB, D, true, NC>(gp(F.G), (long)nl * nl, gp(F.A), yr, yb, s, 1, cnt, nl, T(1), q, ps);
  GAS cx<T>* heads = tips + (size_t)P * A.nl_max * RB;
  for (int idx = threadIdx.x; idx < RB * nl; idx += 256) {
    const int c = idx / nl, l = idx - c * nl;
    tips[((size_t)w.p * RB + c) * nl + l] = yr[((size_t)(e - 1 - yb) * RB + c) * nl + l];
  }
  // chunk-local backward substitution x_t = y_t - E_t x_{t+1} on the local
  // forward values (bchain passes a barrier before its first write, so the
  // tips above are read before y is overwritten)
  bchain<T, NB, RB, D, false, NC>(gp(F.E), (long)nl * nl, nullptr, yr, yb, e - 1, -1, cnt, nl, T(-1), q, ps);
  for (int idx = threadIdx.x; idx < RB * nl; idx += 256) {
    const int c = idx / nl, l = idx - c * nl;
    heads[((size_t)w.p * RB + c) * nl + l] = yr[((size_t)(s - yb) * RB + c) * nl + l];
  }
  // the chunk's local solution to y for the backward launch (bchain ends on
  // a barrier, so every row is in place)
  if constexpr (LY) {
    GAS cx<T>* yo = y + (size_t)s * RB * nl;
    for (int idx = threadIdx.x; idx < cnt * RB * nl; idx += 256) yo[idx] = yr[idx];
  }
  if (P == 1) return;
  if (!last_arrival(counters + 2 * slot, P)) return;
  // true chunk-end values: tip_q = raw_q + Y_{e_q - 1} tip_{q-1}
  bchain<T, NB, RB, D, false, NC>(gp(F.Y) + (size_t)(m - 1) * nl * nl, (long)m * nl * nl, nullptr, tips, 0,
                                  0, 1, P - 1, nl, T(1), q, ps);
  // chunk starts of the backward chains on the true forward values
  bheads_fix<T, RB>(gp(F.W), heads, tips, P, m, nl, ps, 256 * RB);
  // true chunk-start values: head_q = raw_q + X_{s_q} head_{q+1}
  bchain<T, NB, RB, D, false, NC>(gp(F.X), (long)m * nl * nl, nullptr, heads, 0, P - 1, -1, P - 1, nl, T(1),
                                  q, ps);
}

template <class T, int NB, int RB, bool LY>
__global__ void __launch_bounds__(256) k_bstage_bwd(const BSeg* __restrict__ segs, int nseg, int nitems) {
  __shared__ cx<T> hv[NB * RB], cv[NB * RB];
  BWork w;
  BSeg A;
  if (!decode_work(segs, nseg, nitems, A, w)) return;
  GAS cx<T>* __restrict__ u = gp(static_cast<cx<T>*>(A.u));
  GAS cx<T>* __restrict__ bufs = gp(static_cast<cx<T>*>(A.bufs));
  GAS cx<T>* __restrict__ scratch = gp(static_cast<cx<T>*>(A.scratch));
  const cx<T>* __restrict__ factors = static_cast<const cx<T>*>(A.factors);
  const GAS cx<T>* __restrict__ red = gp(static_cast<const cx<T>*>(A.red));
  const int P = A.P, m = A.m, n2 = A.G.n2;
  const int slot = w.q * A.ntiles + w.tile, r0 = w.tile * RB;
  const int nr = min(RB, A.nact - r0);
  const TaskDev tk = cload(A.tasks, w.q);
  const SlabDev sd = cload(A.slabs, tk.slab);
  const int nl = sd.nl;
  const int s = w.p * m, e = min(s + m, n2), cnt = e - s;
  const SlabFac<T> F(factors + sd.fac_off, n2, nl);
  GAS cx<T>* y = scratch + (size_t)slot * n2 * A.nl_max * RB;
  const auto yr = yrows<LY, T>(y);
  const int yb = LY ? s : 0;
  const GAS cx<T>* tips = red + (size_t)slot * 2 * P * A.nl_max * RB;
  const GAS cx<T>* heads = tips + (size_t)P * A.nl_max * RB;
  if constexpr (LY) {
    const GAS cx<T>* yi = y + (size_t)s * RB * nl;
    for (int idx = threadIdx.x; idx < cnt * RB * nl; idx += 256) yr[idx] = yi[idx];
    __syncthreads();
  }
  // x_t += W_t c_{p-1} + X_t d_{p+1} (the true values at the neighbouring
  // chunk ends; absent at the first and last chunk)
  if (w.p > 0 || w.p < P - 1) {
    for (int idx = threadIdx.x; idx < RB * nl; idx += 256) {
      const int c = idx / nl, l = idx - c * nl;
      if (w.p > 0) cv[l * RB + c] = tips[((size_t)(w.p - 1) * RB + c) * nl + l];
      if (w.p < P - 1) hv[l * RB + c] = heads[((size_t)(w.p + 1) * RB + c) * nl + l];
    }
    __syncthreads();
    if (w.p > 0 && w.p < P - 1)
      bfixup2<T, RB>(gp(F.W), cv, gp(F.X), hv, yr, yb, s, e, nl);
    else if (w.p > 0)
      bfixup<T, RB>(gp(F.W), yr, yb, s, e, nl, cv);
    else
      bfixup<T, RB>(gp(F.X), yr, yb, s, e, nl, hv);
    __syncthreads();
  }
  // u += J^T x over the task's layers, outgoing transmission layers; U
  // entries per thread and round, loads first
  constexpr int U = 4;
  const int tot = nr * nl * cnt;
  IdxWalk it(threadIdx.x, cnt, nl);
  for (int base = threadIdx.x; base < tot; base += 256 * U) {
    cx<T> xv[U], uv[U];
    size_t uid[U];
    int cq[U], lq[U], tq[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int c = it.c < nr ? it.c : nr - 1;
      const int ll = it.l, t = s + it.t;
      const int gl = sd.x0 + ll;
      const int glc = (tk.at < gl && gl <= tk.bt) ? gl : tk.bt;
      xv[q] = yr[((size_t)(t - yb) * RB + c) * nl + ll];
      uid[q] = (size_t)(r0 + c) * A.ld + (size_t)(glc - 1) * n2 + t;
      uv[q] = u[uid[q]];
      cq[q] = it.c;
      lq[q] = ll;
      tq[q] = t;
      it.step();
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (cq[q] >= nr) continue;
      const int c = cq[q], ll = lq[q], t = tq[q];
      const int gl = sd.x0 + ll;
      const cx<T> x = xv[q];
      if (tk.at < gl && gl <= tk.bt) u[uid[q]] = uv[q] + x;
      GAS cx<T>* bz = bufs + (size_t)(r0 + c) * A.nbuf * 2 * n2;
      if (tk.t2) {
        GAS cx<T>* Bo = bz + (size_t)tk.bout_f * 2 * n2;
        if (gl == tk.beta_out) Bo[t] = x;
        if (gl == tk.beta_out + 1) Bo[(size_t)n2 + t] = x;
      }
      if (tk.t4) {
        GAS cx<T>* Bo = bz + (size_t)tk.bout_b * 2 * n2;
        if (gl == tk.bt_out) Bo[t] = x;
        if (gl == tk.bt_out + 1) Bo[(size_t)n2 + t] = x;
      }
    }
  }
}

// One thread per (task, slot, t): the coupling of the incoming transmission
// layer to the buffer nodes t-1, t, t+1 (row beta+1 of the global operator
// towards beta for the first layer of a pair, row beta towards beta+1 for
// the second), signed as in the transmission operators T and T~ of Sec. 2.2.
__global__ void __launch_bounds__(256) k_trans_coef(const TaskDev* __restrict__ tasks, int ntasks,
                                                     const SlabDev* __restrict__ slabs, LevelDev G,
                                                     cd* __restrict__ out) {
  const int n2 = G.n2;
  const long total = (long)ntasks * 4 * n2;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const int t = (int)(i % n2), k = (int)((i / n2) % 4), q = (int)(i / (4L * n2));
    const TaskDev tk = tasks[q];
    const int gl = k < 2 ? tk.beta_in + k : tk.bt_in + k - 2;
    const int x0 = slabs[tk.slab].x0, nl = slabs[tk.slab].nl;
    const bool on = (k < 2 ? tk.t1 : tk.t3) && gl >= x0 && gl < x0 + nl;
    cd* o = out + (size_t)i * 3;
    cd c[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) c[a][b] = mk<double>(0, 0);
    if (on) stencil_coefs(G, gl, t + 1, c);
    // slots 0 and 3 add the term, slots 1 and 2 subtract it
    const double sg = (k == 0 || k == 3) ? 1.0 : -1.0;
#pragma unroll
    for (int dt = 0; dt < 3; ++dt) {
      const int tt = t + dt - 1;
      const cd cc = (k & 1) ? c[0][dt] : c[2][dt];
      o[dt] = (on && tt >= 0 && tt < n2) ? mk<double>(sg * cc.re, sg * cc.im) : mk<double>(0, 0);
    }
  }
}

}  // namespace

void launch_trans_coef(const TaskDev* tasks, int ntasks, const SlabDev* slabs, const LevelDev& G, cd* out,
                       hipStream_t s) {
  if (ntasks < 1) return;
  const long total = (long)ntasks * 4 * G.n2;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_trans_coef, dim3(blocks), dim3(256), 0, s, tasks, ntasks, slabs, G, out);
}

// LDS per workgroup of the stage kernels with the chunk scratch in LDS: at
// most 64 KB (no launch attribute needed; two workgroups still share a CU)
constexpr size_t kStageLdsCap = 64 << 10;

template <class T>
void launch_stage_group(const BSeg* segs_dev, int nseg, int nitems, int nl_launch, int m_launch, int rb,
                        hipStream_t s) {
  if (nseg < 1 || nitems < 1) return;
  const dim3 grd(8 * ((nitems + 7) / 8));
#define BLAUNCH(NB, RB, D, NC)                                                                                 \
  do {                                                                                                         \
    const size_t ylds = (size_t)m_launch * RB * nl_launch * sizeof(cx<T>);                                     \
    const size_t stat = (size_t)(BLay<NB, RB, NC>::QN * RB + 256 * RB) * sizeof(cx<T>);                        \
    if (stat + ylds <= kStageLdsCap) {                                                                         \
      hipLaunchKernelGGL((k_bstage_fwd<T, NB, RB, D, NC, true>), grd, dim3(256), ylds, s, segs_dev, nseg,     \
                         nitems);                                                                              \
      hipLaunchKernelGGL((k_bstage_bwd<T, NB, RB, true>), grd, dim3(256), ylds, s, segs_dev, nseg, nitems);   \
    } else {                                                                                                   \
      hipLaunchKernelGGL((k_bstage_fwd<T, NB, RB, D, NC, false>), grd, dim3(256), 0, s, segs_dev, nseg,       \
                         nitems);                                                                              \
      hipLaunchKernelGGL((k_bstage_bwd<T, NB, RB, false>), grd, dim3(256), 0, s, segs_dev, nseg, nitems);     \
    }                                                                                                          \
  } while (0)
  constexpr int D32 = sizeof(T) == 4 ? 2 : 2;
  constexpr int D64 = sizeof(T) == 4 ? 2 : 1;
#define BRB(NB, D, NC)                      \
  do {                                      \
    switch (rb) {                           \
      case 1: BLAUNCH(NB, 1, D, NC); break; \
      case 2: BLAUNCH(NB, 2, D, NC); break; \
      case 4: BLAUNCH(NB, 4, D, NC); break; \
      default: BLAUNCH(NB, 8, D, NC); break; \
    }                                       \
  } while (0)
  // thin slabs on 32 row lanes; thicker ones on 64, with the product columns
  // trimmed to 40 where the slab allows it
  if (nl_launch <= 32)
    BRB(32, D32, 32);
  else if (nl_launch <= 40)
    BRB(64, D64, 40);
  else
    BRB(64, D64, 64);
#undef BRB
#undef BLAUNCH
}

template void launch_stage_group<double>(const BSeg*, int, int, int, int, int, hipStream_t);
template void launch_stage_group<float>(const BSeg*, int, int, int, int, int, hipStream_t);

#undef GAS
#undef CAS

}  // namespace hsp
