// Internal interfaces between the host orchestration (hsp_api.hip) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include "common.h"

namespace hsp {

constexpr int kMaxSlabLayers = 56;   // 2-D slab thickness limit (LDS sized)
constexpr int kMaxChunk = 64;        // longest chunk of the parallel substitutions
constexpr int kWave = 64;

// Batch addressing: vector z of a batch starts at base + off(z), with
// off(z) = (map ? map[z] : z) * ld.  A default BIdx (ld = 0) addresses the
// same vector for every z; single-vector calls use nb = 1.
// dyn (optional) adds an element offset read from device memory, so that a
// captured launch sequence can be pointed at another vector without
// re-capturing it.
struct BIdx {
  size_t ld = 0;
  const int* map = nullptr;
  const long long* dyn = nullptr;
  __device__ __forceinline__ size_t off(int z) const {
    return (size_t)(map ? map[z] : z) * ld + (dyn ? (size_t)*dyn : 0);
  }
};

// ---- stencil kernels (stencil.hip) ---------------------------------------
// y = A x                         (mode 0)
// y = b - A x                     (mode 1)
// y = x + w D^{-1} (b - A x)      (mode 2; x == nullptr means x = 0)
// Tx/Tb/Ty are the storage types of x, b, y; Ta the arithmetic type.
template <class Ta, class Tx, class Tb, class Ty>
void launch_stencil(const LevelDev& L, int mode, const cx<Tx>* x, const cx<Tb>* b, cx<Ty>* y,
                    double w, hipStream_t s, int nb = 1, BIdx bx = {}, BIdx bb = {}, BIdx by = {});

// ---- transfers (transfer.hip) ---------------------------------------------
struct TransferDev {
  int nf1, nf2, nc1, nc2;
  const int* rx;      // [nc1][3] fine x unknown (0-based) per coarse x unknown, -1 = none
  const double* rwx;  // [nc1][3] weights
  const int* ry;
  const double* rwy;
  const int* px;      // [nf1][2] coarse x unknown (0-based) per fine x unknown, -1 = none
  const double* pwx;  // [nf1][2]
  const int* py;
  const double* pwy;
};
template <class Tin, class Tout>
void launch_restrict(const TransferDev& T, const cx<Tin>* rf, cx<Tout>* rc, hipStream_t s, int nb = 1,
                     BIdx bi = {}, BIdx bo = {});
template <class Tc, class Tf>
void launch_prolong_add(const TransferDev& T, const cx<Tc>* ec, cx<Tf>* xf, hipStream_t s, int nb = 1,
                        BIdx bi = {}, BIdx bo = {});

// ---- fused smoothing phases, complex64 smoother on a 5-point fine level ----
// (smooth.hip)
// pre:  xo = x_nu of nu Jacobi steps from 0, res = r - A x_nu (complex128)
// post: x_0 = xin + P ec, nu Jacobi steps, zo = x_nu (complex128)
bool smooth_fused_ok(const LevelDev& L, int nu);
// (r is complex128 or complex64: TR = double or float)
template <class TR>
void launch_smooth_pre(const LevelDev& L, int nu, double w, const cx<TR>* r, BIdx br, cf* xo, BIdx bxo, cd* res,
                       BIdx bres, int nb, hipStream_t s);
template <class TR, class TZ>
void launch_smooth_post(const LevelDev& L, const TransferDev& Tr, int nu, double w, const cx<TR>* r, BIdx br,
                        const cf* xin, BIdx bxin, const cf* ec, BIdx bec, cx<TZ>* zo, BIdx bzo, int nb, hipStream_t s);

// ---- slab factorization and sweep stages (slab.hip) ------------------------
struct SlabDev {
  int x0;          // first global layer (1-based)
  int nl;          // layers
  LevelDev op;     // the slab operator A^(j)
  size_t fac_off;  // element offset of this slab's factors
  size_t scr_off;  // element offset (complex double) of its setup scratch
};

struct TaskDev {
  int slab;                  // 0-based slab
  int a, b;                  // f_d = J(j, a, b) f : global layers a+1..b
  int at, bt;                // u += J(j, a~, b~)^T u_d
  int t1, t2, t3, t4;        // transmission flags (in fwd, out fwd, in bwd, out bwd)
  int bin_f, bin_b;          // buffer read by t1 / t3
  int bout_f, bout_b;        // buffer written by t2 / t4
  int beta_in, bt_in;        // beta_{j-1} (t1 layers) and beta~_j (t3 layers)
  int beta_out, bt_out;      // beta_j (t2 layers) and beta~_{j-1} (t4 layers)
  int src;                   // 0: read the sweep input f, 1: read the residual g
  int mode;                  // 0: subdomain solve on level vectors, 1: slab-layout solve
};

// Factor storage per slab (elements of cx<T>), column-major nl x nl blocks:
// G_t, M_t = -G_t A_t, E_t, the chunk transfer matrices Y_t and X_t, each
// [n2][nl][nl], then the couplings to the previous tangential node,
// A_t[a][l] = coefficient of x_{t-1}[l+a-1] in row l, as [n2][3][nl], then
// W_t [n2][nl][nl]: the chunk-local backward substitution applied to Y
// (the batched stages run the backward chains on the forward values before
// the forward fix-up).
inline size_t slab_factor_elems(int nl, int n2) {
  return (size_t)6 * n2 * nl * nl + (size_t)3 * n2 * nl;
}

// Factor block pointers of a slab.
template <class T>
struct SlabFac {
  const cx<T>* G;
  const cx<T>* M;
  const cx<T>* E;
  const cx<T>* Y;
  const cx<T>* X;
  const cx<T>* A;
  const cx<T>* W;
  __device__ SlabFac(const cx<T>* base, int n2, int nl) {
    const size_t sz = (size_t)n2 * nl * nl;
    G = base;
    M = base + sz;
    E = base + 2 * sz;
    Y = base + 3 * sz;
    X = base + 4 * sz;
    A = base + 5 * sz;
    W = A + (size_t)3 * n2 * nl;
  }
};
// Setup scratch per slab (complex double): G_t, E_t and the couplings A_t.
inline size_t slab_setup_elems(int nl, int n2) {
  return (size_t)2 * n2 * nl * nl + (size_t)3 * n2 * nl;
}
// Temporaries of the transfer-matrix kernel per (chunk, slab), complex double.
constexpr size_t kTransferTmpElems = (size_t)3 * kMaxSlabLayers * kMaxSlabLayers;

template <class T>
void launch_factor(const SlabDev* slabs_dev, int nslabs, int nl_max, int n2, int m, int P,
                   cx<T>* factors, cd* setup, cd* scratchE, cd* tmp, int* status, double* growth, int dbg_singular,
                  hipStream_t s);

// One SubdomSolve stage (ntasks slabs at once), as three launches over
// (P chunks) x (ntasks).  red: per task 2 P nl_max complex (chunk tips and
// heads); counters: 2 ints per task, zero between launches.
template <class T>
void launch_stage(const TaskDev* tasks_dev, int ntasks, const SlabDev* slabs_dev,
                  const LevelDev& G, const cx<T>* f, const cx<T>* g, cx<T>* u, cx<T>* bufs,
                  cx<T>* scratch, const cx<T>* factors, int nl_max, int nl_launch, int m, int P,
                  cx<T>* red, int* counters, hipStream_t s);

// The same stage for many right-hand sides of several problems (batch.hip).
// One segment per problem taking part in the launch: its tasks of this
// stage, its level vectors f, g, u ([nact][ld], right-hand side z at offset
// z ld, storage type of the launch), transmission buffers [nact][nbuf][2][n2],
// scratch ntasks ceil(nact/rb) rb n2 nl_max, chunk tips / heads
// ntasks ceil(nact/rb) 2 P nl_max rb, counters 2 ntasks ceil(nact/rb) ints
// (zero between launches).  Work items of a segment: (task, chunk, tile of rb
// right-hand sides); item0 is the segment's first item in the launch.
struct BSeg {
  const TaskDev* tasks;
  const SlabDev* slabs;
  LevelDev G;
  const void* f;
  const void* g;
  void* u;
  void* bufs;
  void* scratch;
  const void* factors;
  void* red;
  int* counters;
  const cd* tcoef;  // transmission coefficients of the segment's first task
  size_t ld;
  int ntasks, ntiles, nact, nl_max, m, P, item0, nbuf;  // nbuf: transmission buffers per right-hand side
};
// Incoming transmission terms of a task as a table, [4][n2][3] complex
// double per task: slot k of the (up to) four incoming transmission layers
// (beta_{j-1}, beta_{j-1} + 1, beta~_j, beta~_j + 1), tangential node t, and
// the coupling to buffer node t + dt - 1 with the sign of the transmission
// operator folded in (zero where the flag is off or t + dt - 1 is outside).
__host__ __device__ inline size_t trans_coef_elems(int n2) {
  return (size_t)4 * n2 * 3;
}
void launch_trans_coef(const TaskDev* tasks, int ntasks, const SlabDev* slabs, const LevelDev& G, cd* out,
                       hipStream_t s);
// segs_dev: nseg segments in device memory, nitems work items in total,
// nl_launch the thickest slab, m_launch the longest chunk, rb in {1, 2, 4, 8}.
template <class T>
void launch_stage_group(const BSeg* segs_dev, int nseg, int nitems, int nl_launch, int m_launch, int rb,
                        hipStream_t s);

// ---- BLAS-1 and utilities (blas.hip) ---------------------------------------
template <class To, class Ti>
void launch_convert(const cx<Ti>* in, cx<To>* out, size_t n, int conjugate, hipStream_t s, int nb = 1,
                    BIdx bi = {}, BIdx bo = {});
template <class T>
void launch_zero(cx<T>* v, size_t n, hipStream_t s);
// v[i] = value for i < n
void launch_fill(cd* v, size_t n, cd value, hipStream_t s);
// w -= sum_j h[j] V_j   (h on device)
void launch_multiaxpy(const cd* V, size_t ldv, int m, const cd* h, cd* w, size_t n, int sub,
                      hipStream_t s);
// v = w / sqrt(re(nrm2[0]))
void launch_normalize(const cd* w, const cd* nrm2, cd* v, size_t n, hipStream_t s);
// Batched forms over nb right-hand sides z (vector j of z: V + bv.off(z) + j ldj):
// out[z ldo + j] = conj(V_zj) . w_z, j < cnt (partial: nb cnt nblocks entries)
int batch_dot_blocks(size_t n, int nb);
// blocks per right-hand side of launch_bdcgs_update (partial: nb nblocks)
int batch_upd_blocks(size_t n, int nb);
void launch_bmultidot(const cd* V, size_t ldj, BIdx bv, int cnt, const cd* w, BIdx bw, size_t n, cd* partial,
                      int nblocks, cd* out, size_t ldo, int nb, hipStream_t s);
// w_z -= (or +=) sum_j h[z ldh + j] V_zj (V complex128 or complex64)
template <class TV>
void launch_bmultiaxpy(const cx<TV>* V, size_t ldj, BIdx bv, int cnt, const cd* h, size_t ldh, cd* w, BIdx bw,
                       size_t n, int sub, int nb, hipStream_t s);
// the same with nrm2[z ldo] = ||w_z||^2 after the update (partial: nb nblocks)
void launch_bmultiaxpy_norm(const cd* V, size_t ldj, BIdx bv, int cnt, const cd* h, size_t ldh, cd* w, BIdx bw,
                            size_t n, cd* partial, int nblocks, cd* nrm2, size_t ldo, int nb, hipStream_t s);
// Delayed classical Gram-Schmidt (one projection pass and one update pass
// per Arnoldi step).  Slot k of right-hand side z holds the once-projected
// vector u_k.  project: hb[z ldh + (0..k)] = V^H u_k, hb[.. + k+1 + (0..k)] =
// V^H w, then nu and h_kk at hb[.. + off], hb[.. + off + 1].  update: slot k
// <- v_k (final), slot k+1 <- u_{k+1} = w - V p - h_kk v_k, ||u_{k+1}||^2 at
// nrm2[z ldh].
// The basis is complex128 (TV = double) or complex64 (TV = float; the
// products and sums are still formed in double).
template <class TV>
void launch_bdcgs_project(const cx<TV>* V, size_t ldj, BIdx bv, int k, const cd* w, BIdx bw, size_t n,
                          cd* partial, int nblocks, cd* hb, size_t ldh, int off, int nb, hipStream_t s);
template <class TV>
void launch_bdcgs_update(cx<TV>* V, size_t ldj, BIdx bv, int k, const cd* hb, size_t ldh, int off, const cd* w,
                         BIdx bw, size_t n, cd* partial, int nblocks, cd* nrm2, int nb, hipStream_t s);
// v_z = w_z / sqrt(re(nrm2[z ldn])), rounded to TV
template <class TV>
void launch_bnormalize(const cd* w, BIdx bw, const cd* nrm2, size_t ldn, cx<TV>* v, BIdx bv, size_t n, int nb,
                       hipStream_t s);
// b = h2 * f / (alpha_1(x_i) alpha_2(y_k)); ixn, iyn = 1/alpha at nodes 0..n+1
void launch_scale_rhs_arrays(int n1, int n2, double h2, const cd* ixn, const cd* iyn, const cd* f, cd* b,
                             hipStream_t s);
// g += scale * Re(conj(lam) u / (alpha_1 alpha_2)) on the fine unknowns
void launch_grad_m(int n1, int n2, double scale, const cd* ixn, const cd* iyn, const cd* u, const cd* lam, double* g,
                   hipStream_t s);
// statistics of a real array: [sum, min, max, count of non-finite or <= 0]
void launch_stats(const double* c, size_t n, double* out4, hipStream_t s);
// per-node medium arrays
void launch_k2_nodes(const double* c, size_t n, double omega, double* k2, hipStream_t s);
// cell k2 = W1 (k2 nodes padded) W2^T with per-axis 3-tap weights
void launch_cell_average(const double* k2n, int n1, int n2, const int* x0, const double* wx,
                         int nc1, const int* y0, const double* wy, int nc2, double* k2c,
                         hipStream_t s);
void launch_cell_coefs(const double* k2c, size_t ncell, double h_nom, double* coef,
                       hipStream_t s);
// sponge layers: k2 -> real part of k2 (1 + i (bx[i] + by[k]))^2, k2i its
// imaginary part, at the n1 x n2 unknown nodes
void launch_sponge_k2(int n1, int n2, const double* bx, const double* by, double* k2, double* k2i, hipStream_t s);

}  // namespace hsp
