// Device helpers shared by the single and the batched SubdomSolve stage
// kernels: the discrete transmission right-hand side, predicated values and
// the last-arrival pattern of the chunk-parallel substitutions.
#pragma once

#include "internal.h"

namespace hsp {

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

template <class T>
__device__ __forceinline__ cx<T> sel(bool ok, cx<T> v) {
  return mk<T>(ok ? v.re : T(0), ok ? v.im : T(0));
}

// LDS ordering between the lanes of one wavefront: the LDS executes a
// wave's instructions in order, so only the compiler must be kept from
// reordering (wavefront-scope fences) - no s_barrier is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The last workgroup of a (chunk-parallel) launch to arrive continues with
// the chain over the chunk ends.  Release the block's results device-wide,
// count arrivals, and make the other blocks' results visible to the last.
__device__ __forceinline__ bool last_arrival(int* counter, int nblocks) {
  __shared__ int sh_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int old = atomicAdd(counter, 1);
    sh_last = (old == nblocks - 1) ? 1 : 0;
    if (sh_last) atomicExch(counter, 0);  // ready for the next launch
  }
  __syncthreads();
  const bool last = sh_last != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace hsp
