// Slab subdomain factorization and the fused SubdomSolve stage kernel.
//
// A slab A^(j) (Sec. 2.1, subdomains) covers nl layers x n2 tangential nodes.
// Ordered with the tangential index t slowest it is block tridiagonal with
// nl x nl blocks: A_t x_{t-1} + B_t x_t + C_t x_{t+1} = f_t, the blocks being
// tridiagonal in the layer index (compact stencil).  Block LU along t:
//   S_0 = B_0,  S_t = B_t - A_t E_{t-1},  G_t = S_t^{-1},  E_t = G_t C_t,
// solved by  y_t = G_t (f_t - A_t y_{t-1})  and  x_t = y_t - E_t x_{t+1}.
// S_t is inverted in LDS by Gauss-Jordan with partial (row) pivoting; the
// pivot row is found by a wavefront max-reduction.  All slabs are factored
// in one launch (one workgroup per slab).  G_t and E_t are stored column
// major so that a lane owning output row l reads them coalesced.
#include "internal.h"

namespace hsp {

namespace {

template <class T>
__global__ void __launch_bounds__(256) k_factor(const SlabDev* __restrict__ slabs, int n2, cx<T>* factors,
                                                cd* scratchE, int* status) {
  extern __shared__ cd smem[];
  const SlabDev sd = slabs[blockIdx.x];
  const int nl = sd.nl;
  cd* S = smem;            // nl*nl, row major
  cd* cfs = S + nl * nl;   // [nl][9] stencil coefficients of the rows at t
  cd* colf = cfs + 9 * nl; // [nl]
  __shared__ int piv[kMaxSlabLayers];
  __shared__ int sh_p, sh_bad;
  cd* Ep = scratchE + (size_t)blockIdx.x * kMaxSlabLayers * kMaxSlabLayers;
  cx<T>* Gm = factors + sd.fac_off;
  cx<T>* Em = Gm + (size_t)n2 * nl * nl;
  cx<T>* Am = Em + (size_t)n2 * nl * nl;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) sh_bad = 0;

  for (int t = 0; t < n2; ++t) {
    for (int i = tid; i < nl; i += nt) {
      cd c[3][3];
      stencil_coefs(sd.op, i + 1, t + 1, c);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) cfs[i * 9 + a * 3 + b] = c[a][b];
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
    // store G_t (column major) and E_t = G_t C_t
    for (int idx = tid; idx < nl * nl; idx += nt) {
      const int j = idx / nl, i = idx - (idx / nl) * nl;
      Gm[((size_t)t * nl + j) * nl + i] = cvt<T>(S[i * nl + j]);
      cd e = mk<double>(0, 0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int m = j + a - 1;
        if (m < 0 || m >= nl) continue;
        e += S[i * nl + m] * cfs[m * 9 + (j - m + 1) * 3 + 2];
      }
      Em[((size_t)t * nl + j) * nl + i] = cvt<T>(e);
      Ep[i * nl + j] = e;
    }
    __syncthreads();
  }
  if (tid == 0 && sh_bad) atomicOr(status, 1);
}

// Transmission right-hand side of row gl at tangential node t (Sec. 2.2,
// discrete transmission): T^(j) B adds +A_{b,b+1} B[1] to layer b and
// -A_{b+1,b} B[0] to layer b+1 (b = beta_{j-1}); T~^(j) B adds
// -A_{b,b+1} B[1] and +A_{b+1,b} B[0] (b = beta~_j).  A is the global
// level operator, so the couplings are its (tridiagonal in t) blocks.
template <class T>
__device__ __forceinline__ cd transmission_rhs(const TaskDev& tk, const LevelDev& G, int gl, int t, int n2,
                                               const cx<T>* Bif, const cx<T>* Bib) {
  cd acc = mk<double>(0, 0);
  const bool inF = tk.t1 && (gl == tk.beta_in || gl == tk.beta_in + 1);
  const bool inB = tk.t3 && (gl == tk.bt_in || gl == tk.bt_in + 1);
  if (!inF && !inB) return acc;
  cd c[3][3];
  stencil_coefs(G, gl, t + 1, c);
  if (inF) {
    const int s = (gl == tk.beta_in) ? 1 : 0;
    cd a = mk<double>(0, 0);
#pragma unroll
    for (int dt = -1; dt <= 1; ++dt) {
      const int tt = t + dt;
      if (tt < 0 || tt >= n2) continue;
      const cd cc = (s == 1) ? c[2][dt + 1] : c[0][dt + 1];
      cfma(a, cc, cvt<double>(Bif[(size_t)s * n2 + tt]));
    }
    acc = (s == 1) ? acc + a : acc - a;
  }
  if (inB) {
    const int s = (gl == tk.bt_in) ? 1 : 0;
    cd a = mk<double>(0, 0);
#pragma unroll
    for (int dt = -1; dt <= 1; ++dt) {
      const int tt = t + dt;
      if (tt < 0 || tt >= n2) continue;
      const cd cc = (s == 1) ? c[2][dt + 1] : c[0][dt + 1];
      cfma(a, cc, cvt<double>(Bib[(size_t)s * n2 + tt]));
    }
    acc = (s == 1) ? acc - a : acc + a;
  }
  return acc;
}

// Register-ring fetches of the stage kernel (no address-taken locals, so
// nothing lands in private scratch: a scratch load would be a vector-memory
// operation and waiting for it would drain the whole prefetch ring).
template <class T, int CW>
__device__ __forceinline__ void fetch_block(const cx<T>* __restrict__ base, int t, int nl, int lc, int j0, bool act,
                                            cx<T> (&dst)[CW]) {
  // lc is the row clamped into the slab; loads are unconditional (addresses
  // always valid) and out-of-slab entries are replaced by zeros with a select.
  const cx<T>* p = base + (size_t)t * nl * nl + lc;
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int j = j0 + c;
    const int jc = j < nl ? j : nl - 1;
    const cx<T> v = p[(size_t)jc * nl];
    const bool ok = act && j < nl;
    dst[c] = mk<T>(ok ? v.re : T(0), ok ? v.im : T(0));
  }
}

template <class T>
__device__ __forceinline__ cx<T> sel(bool ok, cx<T> v) {
  return mk<T>(ok ? v.re : T(0), ok ? v.im : T(0));
}

// Fused SubdomSolve (Table 2) for one slab per workgroup.
//   prologue  (parallel): f_d = J(j,a,b) f + transmission terms -> scratch [t][l]
//   forward   (sequential in t): y_t = G_t (f_t - A_t y_{t-1})
//   backward  (sequential in t): x_t = y_t - E_t x_{t+1}
//   epilogue  (parallel): u += J(j,a~,b~)^T x, outgoing layers -> B buffers.
// Thread layout: R row slots (32 when the slab has <= 32 layers, else 64)
// times NG = NT / R column groups; thread (l, h) owns row l and columns
// [h CW, (h+1) CW) of every block, so it keeps only CW entries of a block.
// The blocks of the next D steps are held in a register ring (prefetch
// distance D) so that the HBM / last-level-cache latency of the factor
// stream overlaps the sequential recurrence.  Two LDS barriers per step:
// the row owners publish the right-hand side v_t, every thread forms its
// partial products, and the row owners sum them at the start of the next
// step.
template <class T, int NB, int NT, int D>
__global__ void __launch_bounds__(NT) k_stage(const TaskDev* __restrict__ tasks, const SlabDev* __restrict__ slabs,
                                              LevelDev G, const cx<T>* __restrict__ f, const cx<T>* __restrict__ g,
                                              cx<T>* __restrict__ u, cx<T>* __restrict__ bufs,
                                              cx<T>* __restrict__ scratch, const cx<T>* __restrict__ factors,
                                              int nl_max) {
  constexpr int R = (NB <= 32) ? 32 : 64;
  constexpr int NG = NT / R;
  constexpr int CW = (NB + NG - 1) / NG;
  const TaskDev tk = tasks[blockIdx.x];
  const SlabDev sd = slabs[tk.slab];
  const int nl = sd.nl, n2 = G.n2;
  const int tid = threadIdx.x;
  const int l = tid % R, h = tid / R, j0 = h * CW;
  const bool act = l < nl;
  const bool own = act && h == 0;
  const cx<T>* Gm = factors + sd.fac_off;
  const cx<T>* Em = Gm + (size_t)n2 * nl * nl;
  const cx<T>* Am = Em + (size_t)n2 * nl * nl;
  cx<T>* y = scratch + (size_t)blockIdx.x * n2 * nl_max;  // [t][l]
  const cx<T>* src = tk.src ? g : f;
  const cx<T>* Bif = bufs + (size_t)tk.bin_f * 2 * n2;
  const cx<T>* Bib = bufs + (size_t)tk.bin_b * 2 * n2;
  cx<T>* Bof = bufs + (size_t)tk.bout_f * 2 * n2;
  cx<T>* Bob = bufs + (size_t)tk.bout_b * 2 * n2;
  __shared__ cx<T> vs[NG * CW];
  __shared__ cx<T> ps[NG][R + 2];  // partial sums, rows shifted by one (halo)

  // ---- prologue: slab right-hand side -----------------------------------
  for (int idx = tid; idx < nl * n2; idx += NT) {
    const int ll = idx / n2, t = idx - (idx / n2) * n2;
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
  for (int i = tid; i < NG * CW; i += NT) vs[i] = mk<T>(0, 0);
  for (int i = tid; i < NG * (R + 2); i += NT) ps[i / (R + 2)][i % (R + 2)] = mk<T>(0, 0);
  __syncthreads();

  // register ring: factor slices, right-hand side rows and couplings
  const int lc = l < nl ? l : nl - 1;
  cx<T> rg[D][CW], rf[D], ra[D][3];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int tc = d < n2 ? d : n2 - 1;
    fetch_block<T, CW>(Gm, tc, nl, lc, j0, act, rg[d]);
    rf[d] = sel(act, y[(size_t)tc * nl + lc]);
#pragma unroll
    for (int a = 0; a < 3; ++a) ra[d][a] = sel(act, Am[((size_t)tc * 3 + a) * nl + lc]);
  }

  // ---- forward substitution ---------------------------------------------
  // step t: (a) row owners sum the partial products of step t-1 into
  // y_{t-1} (their row and its two neighbours), store y_{t-1} and publish
  // v_t = f_t - A_t y_{t-1}; (b) every thread forms its partial products of
  // G_t v_t.  Then the ring slot of step t is refilled with step t + D.
#define HSP_FWD_STEP(t, d)                                                         \
  {                                                                                \
    cx<T> ym = mk<T>(0, 0), yc = mk<T>(0, 0), yp = mk<T>(0, 0);                    \
    _Pragma("unroll") for (int q = 0; q < NG; ++q) {                               \
      ym = ym + ps[q][l];                                                          \
      yc = yc + ps[q][l + 1];                                                      \
      yp = yp + ps[q][l + 2];                                                      \
    }                                                                              \
    if (own && (t) > 0) y[(size_t)((t) - 1) * nl + l] = yc;                        \
    cx<T> ay = mk<T>(0, 0);                                                        \
    cfma(ay, ra[d][0], ym);                                                        \
    cfma(ay, ra[d][1], yc);                                                        \
    cfma(ay, ra[d][2], yp);                                                        \
    if (h == 0 && l < NG * CW) vs[l] = sel(act, rf[d] - ay);                       \
    __syncthreads();                                                               \
    cx<T> part = mk<T>(0, 0);                                                      \
    _Pragma("unroll") for (int c = 0; c < CW; ++c) cfma(part, rg[d][c], vs[j0 + c]); \
    ps[h][l + 1] = sel(act, part);                                                 \
    __syncthreads();                                                               \
  }
#define HSP_FWD_FETCH(tn, d)                                                       \
  {                                                                                \
    const int tc = (tn) < n2 ? (tn) : n2 - 1;                                      \
    fetch_block<T, CW>(Gm, tc, nl, lc, j0, act, rg[d]);                            \
    rf[d] = sel(act, y[(size_t)tc * nl + lc]);                                     \
    _Pragma("unroll") for (int a = 0; a < 3; ++a) ra[d][a] = sel(act, Am[((size_t)tc * 3 + a) * nl + lc]); \
  }
  int t0 = 0;
  for (; t0 + D <= n2; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      HSP_FWD_STEP(t0 + d, d)
      HSP_FWD_FETCH(t0 + d + D, d)
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (t0 + d < n2) HSP_FWD_STEP(t0 + d, d)
  }
#undef HSP_FWD_STEP
#undef HSP_FWD_FETCH
  if (own) {
    cx<T> yc = mk<T>(0, 0);
#pragma unroll
    for (int q = 0; q < NG; ++q) yc = yc + ps[q][l + 1];
    y[(size_t)(n2 - 1) * nl + l] = yc;
  }
  __syncthreads();

  // ---- back substitution --------------------------------------------------
  // ring slot d holds E_t and y_{t+1} for t = n2-1-(k D + d); step t: (a)
  // owners form x_{t+1} = y_{t+1} - (partials of step t+1), store it and
  // publish it; (b) partial products of E_t x_{t+1}.
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int t = n2 - 1 - d;
    const int tc = t >= 0 ? t : 0;
    fetch_block<T, CW>(Em, tc, nl, lc, j0, act, rg[d]);
    rf[d] = sel(act, y[(size_t)(tc + 1 < n2 ? tc + 1 : tc) * nl + lc]);
  }
#define HSP_BWD_STEP(t, d)                                                         \
  {                                                                                \
    cx<T> xn = mk<T>(0, 0);                                                        \
    if ((t) < n2 - 1) {                                                            \
      cx<T> sm = mk<T>(0, 0);                                                      \
      _Pragma("unroll") for (int q = 0; q < NG; ++q) sm = sm + ps[q][l + 1];       \
      xn = rf[d] - sm;                                                             \
      if (own) y[(size_t)((t) + 1) * nl + l] = xn;                                 \
    }                                                                              \
    if (h == 0 && l < NG * CW) vs[l] = sel(act, xn);                               \
    __syncthreads();                                                               \
    cx<T> part = mk<T>(0, 0);                                                      \
    _Pragma("unroll") for (int c = 0; c < CW; ++c) cfma(part, rg[d][c], vs[j0 + c]); \
    ps[h][l + 1] = sel(act, part);                                                 \
    __syncthreads();                                                               \
  }
#define HSP_BWD_FETCH(tn, d)                                                       \
  {                                                                                \
    const int tc = (tn) >= 0 ? (tn) : 0;                                           \
    fetch_block<T, CW>(Em, tc, nl, lc, j0, act, rg[d]);                            \
    rf[d] = sel(act, y[(size_t)(tc + 1) * nl + lc]);                               \
  }
  int k0 = 0;
  for (; k0 + D <= n2; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      HSP_BWD_STEP(n2 - 1 - (k0 + d), d)
      HSP_BWD_FETCH(n2 - 1 - (k0 + d) - D, d)
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (k0 + d < n2) HSP_BWD_STEP(n2 - 1 - (k0 + d), d)
  }
#undef HSP_BWD_STEP
#undef HSP_BWD_FETCH
  if (own) {
    cx<T> sm = mk<T>(0, 0);
#pragma unroll
    for (int q = 0; q < NG; ++q) sm = sm + ps[q][l + 1];
    y[l] = y[l] - sm;  // x_0 = y_0 - E_0 x_1
  }
  __syncthreads();

  // ---- epilogue: scatter-add and outgoing transmission layers ------------
  for (int idx = tid; idx < nl * n2; idx += NT) {
    const int ll = idx / n2, t = idx - (idx / n2) * n2;
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
void launch_factor(const SlabDev* slabs_dev, int nslabs, int nl_max, int n2, cx<T>* factors, cd* scratch,
                   int* status, hipStream_t s) {
  const size_t shm = ((size_t)nl_max * nl_max + 10 * (size_t)nl_max) * sizeof(cd);
  hipLaunchKernelGGL((k_factor<T>), dim3(nslabs), dim3(256), shm, s, slabs_dev, n2, factors, scratch, status);
}

template <class T>
void launch_stage(const TaskDev* tasks_dev, int ntasks, const SlabDev* slabs_dev, const LevelDev& G,
                  const cx<T>* f, const cx<T>* g, cx<T>* u, cx<T>* bufs, cx<T>* scratch, const cx<T>* factors,
                  int nl_max, int nl_launch, hipStream_t s) {
#define LAUNCH(NB, NT, D)                                                                                  \
  hipLaunchKernelGGL((k_stage<T, NB, NT, D>), dim3(ntasks), dim3(NT), 0, s, tasks_dev, slabs_dev, G, f, g, u, bufs, \
                     scratch, factors, nl_max)
  // prefetch depth: deeper for complex64 (half the registers per entry)
  constexpr int DS = sizeof(T) == 4 ? 8 : 4;   // thin slabs
  constexpr int DW = sizeof(T) == 4 ? 4 : 2;   // thick slabs
  if (nl_launch <= 16)
    LAUNCH(16, 128, DS);
  else if (nl_launch <= 32)
    LAUNCH(32, 256, DS);
  else if (nl_launch <= 40)
    LAUNCH(40, 512, DW);
  else if (nl_launch <= 48)
    LAUNCH(48, 512, DW);
  else
    LAUNCH(64, 512, DW);
#undef LAUNCH
}

template void launch_factor<double>(const SlabDev*, int, int, int, cd*, cd*, int*, hipStream_t);
template void launch_factor<float>(const SlabDev*, int, int, int, cf*, cd*, int*, hipStream_t);
template void launch_stage<double>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cd*, const cd*, cd*,
                                   cd*, cd*, const cd*, int, int, hipStream_t);
template void launch_stage<float>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cf*, const cf*, cf*,
                                  cf*, cf*, const cf*, int, int, hipStream_t);

}  // namespace hsp
