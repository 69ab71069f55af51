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

// Global coupling coefficient of row (i, t+1) of the level operator toward
// layer i + dl and tangential node t+1+dt.
__device__ __forceinline__ void row_coefs(const LevelDev& G, int i, int t, cd c[3][3]) {
  stencil_coefs(G, i, t + 1, c);
}

template <class T>
__global__ void __launch_bounds__(64) k_stage(const TaskDev* __restrict__ tasks, const SlabDev* __restrict__ slabs,
                                              LevelDev G, const cx<T>* __restrict__ f, const cx<T>* __restrict__ g,
                                              cx<T>* __restrict__ u, cx<T>* __restrict__ bufs,
                                              cx<T>* __restrict__ scratch, const cx<T>* __restrict__ factors,
                                              int nl_max) {
  const TaskDev tk = tasks[blockIdx.x];
  const SlabDev sd = slabs[tk.slab];
  const int nl = sd.nl, n2 = G.n2, l = threadIdx.x;
  const bool act = l < nl;
  const int gl = sd.x0 + l;
  const cx<T>* Gm = factors + sd.fac_off;
  const cx<T>* Em = Gm + (size_t)n2 * nl * nl;
  const cx<T>* Am = Em + (size_t)n2 * nl * nl;
  cx<T>* y = scratch + (size_t)blockIdx.x * n2 * nl_max;
  const cx<T>* src = tk.src ? g : f;
  const cx<T>* Bif = bufs + (size_t)tk.bin_f * 2 * n2;
  const cx<T>* Bib = bufs + (size_t)tk.bin_b * 2 * n2;
  cx<T>* Bof = bufs + (size_t)tk.bout_f * 2 * n2;
  cx<T>* Bob = bufs + (size_t)tk.bout_b * 2 * n2;
  __shared__ cx<T> sv[kWave];
  __shared__ cx<T> sp[kWave + 2];
  const cx<T> zero = mk<T>(0, 0);
  sv[l] = zero;
  sp[l + 1] = zero;
  if (l == 0) {
    sp[0] = zero;
    sp[kWave + 1] = zero;
  }
  __syncthreads();

  // forward substitution, gathering the right-hand side on the fly
  for (int t = 0; t < n2; ++t) {
    cx<T> v = zero;
    if (act) {
      if (tk.mode == 1) {
        v = src[(size_t)l * n2 + t];
      } else {
        if (tk.a < gl && gl <= tk.b) v = src[(size_t)(gl - 1) * n2 + t];
        // (J_in)^t T^(j) B : +A_{b,b+1} B[1] on layer b, -A_{b+1,b} B[0] on layer b+1
        if (tk.t1 && (gl == tk.beta_in || gl == tk.beta_in + 1)) {
          cd c[3][3];
          row_coefs(G, gl, t, c);
          const int s = (gl == tk.beta_in) ? 1 : 0;
          cd acc = mk<double>(0, 0);
#pragma unroll
          for (int dt = -1; dt <= 1; ++dt) {
            const int tt = t + dt;
            if (tt < 0 || tt >= n2) continue;
            cfma(acc, c[s == 1 ? 2 : 0][dt + 1], cvt<double>(Bif[(size_t)s * n2 + tt]));
          }
          v = (s == 1) ? v + cvt<T>(acc) : v - cvt<T>(acc);
        }
        // (J~_in)^t T~^(j) B : -A_{b,b+1} B[1] on layer b, +A_{b+1,b} B[0] on layer b+1
        if (tk.t3 && (gl == tk.bt_in || gl == tk.bt_in + 1)) {
          cd c[3][3];
          row_coefs(G, gl, t, c);
          const int s = (gl == tk.bt_in) ? 1 : 0;
          cd acc = mk<double>(0, 0);
#pragma unroll
          for (int dt = -1; dt <= 1; ++dt) {
            const int tt = t + dt;
            if (tt < 0 || tt >= n2) continue;
            cfma(acc, c[s == 1 ? 2 : 0][dt + 1], cvt<double>(Bib[(size_t)s * n2 + tt]));
          }
          v = (s == 1) ? v - cvt<T>(acc) : v + cvt<T>(acc);
        }
      }
      const cx<T>* ar = Am + (size_t)t * 3 * nl;
      cx<T> ay = zero;
      cfma(ay, ar[l], sp[l]);
      cfma(ay, ar[nl + l], sp[l + 1]);
      cfma(ay, ar[2 * nl + l], sp[l + 2]);
      v = v - ay;
    }
    sv[l] = v;
    __syncthreads();
    cx<T> acc = zero;
    if (act) {
      const cx<T>* gt = Gm + (size_t)t * nl * nl + l;
      for (int j = 0; j < nl; ++j) cfma(acc, gt[(size_t)j * nl], sv[j]);
      y[(size_t)t * nl + l] = acc;
    }
    sp[l + 1] = act ? acc : zero;
    __syncthreads();
  }

  // back substitution, scattering the solution and the outgoing layers
  sv[l] = zero;
  __syncthreads();
  for (int t = n2 - 1; t >= 0; --t) {
    cx<T> x = zero;
    if (act) {
      cx<T> acc = zero;
      if (t < n2 - 1) {
        const cx<T>* et = Em + (size_t)t * nl * nl + l;
        for (int j = 0; j < nl; ++j) cfma(acc, et[(size_t)j * nl], sv[j]);
      }
      x = y[(size_t)t * nl + l] - acc;
    }
    __syncthreads();
    sv[l] = x;
    if (act) {
      if (tk.mode == 1) {
        u[(size_t)l * n2 + t] = x;
      } else {
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
    __syncthreads();
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
                  int nl_max, hipStream_t s) {
  hipLaunchKernelGGL((k_stage<T>), dim3(ntasks), dim3(kWave), 0, s, tasks_dev, slabs_dev, G, f, g, u, bufs, scratch,
                     factors, nl_max);
}

template void launch_factor<double>(const SlabDev*, int, int, int, cd*, cd*, int*, hipStream_t);
template void launch_factor<float>(const SlabDev*, int, int, int, cf*, cd*, int*, hipStream_t);
template void launch_stage<double>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cd*, const cd*, cd*,
                                   cd*, cd*, const cd*, int, hipStream_t);
template void launch_stage<float>(const TaskDev*, int, const SlabDev*, const LevelDev&, const cf*, const cf*, cf*,
                                  cf*, cf*, const cf*, int, hipStream_t);

}  // namespace hsp
