// Host-side state shared by the translation units of the library: the
// size plan of a workspace, the sweep schedule, event timing and the handle.
// Not part of the public ABI.
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "../../include/hsp.h"
#include "internal.h"

namespace hsp {

// Records msg as the calling thread's last error and returns st.
hsp_status fail(hsp_status st, const std::string& msg);

// Debugging knobs of hsp_debug_set (process-wide).
struct DebugKnobs {
  int singular_slab = -1;     // slab whose first block is replaced by zero at setup
  double growth_limit = 0.0;  // > 0: replaces the default growth limit
};
DebugKnobs& debug_knobs();
// Growth limit for slab factors stored with tsize bytes per complex value:
// the factorization is refused when fewer than two significant digits of the
// factor precision would survive a growth of the Schur complements.
double growth_limit(size_t tsize);

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return hsp::fail(HSP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

using cplx = std::complex<double>;

inline cd to_cd(cplx z) { return mk<double>(z.real(), z.imag()); }

// PML damping sigma(x): C (lo - x)^2 left of lo, C (x - hi)^2 right of hi.
struct Sigma {
  double lo = 0, hi = 0, C = 0;
  bool left = false, right = false;
  double operator()(double x) const {
    double s = 0;
    if (left && x < lo) s = C * (lo - x) * (lo - x);
    if (right && x > hi) s = C * (x - hi) * (x - hi);
    return s;
  }
};

inline cplx alpha_of(double sigma, double omega) { return 1.0 / cplx(1.0, sigma / omega); }

// One axis of a level: node coordinates and the outer PML.
struct AxisH {
  std::vector<double> x;  // nodes 0..N
  Sigma sig;
  double h_nom = 0;
  int n() const { return (int)x.size() - 2; }  // unknowns
};

// Partition beta_0..beta_J of n1 layers: outer-PML layers join the first and
// last cores, interior layers split evenly.
std::vector<int> partition(int n1, int w_outer, int J);
// PML-aware coarsening of an axis with N cells and w PML cells per side: the
// fine node of every coarse node (ifp) and which coarse cells are refined.
void coarse_map(int N, int w, std::vector<int>& ifp, std::vector<char>& ref);

inline hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    const size_t o = off;
    off += bytes;
    return o;
  }
};

// Everything that depends on sizes only.
struct Plan {
  int nf1 = 0, nf2 = 0, Nf1 = 0, Nf2 = 0;  // fine unknowns / cells
  int two_grid = 0;
  int nc1 = 0, nc2 = 0;                   // coarse unknowns
  std::vector<int> ifp1, ifp2;            // coarse -> fine node maps
  std::vector<char> ref1, ref2;           // refined coarse cells
  int dd_kind = 5, dd_n1 = 0, dd_n2 = 0;  // DD level
  int fine_kind = 5;
  std::vector<int> beta, bt, x0, x1;
  int nl_max = 0;
  int chunk = 0, nchunk = 0;              // parallel substitution: chunk length m, count P
  int nbuf = 2, maxtask = 2;              // transmission buffers; most slab solves in one stage
  int sponge = 0;                         // outer layers are sponge layers (no PML)
  size_t o_k2i = 0, o_bx = 0, o_by = 0, o_ck2ci = 0;  // sponge: imaginary k^2, beta per node
  size_t tsize = 16;                      // bytes per preconditioner complex
  int m = 0;                              // FGMRES restart
  // workspace offsets
  size_t o_fxA, o_fxB, o_fyA, o_fyB, o_k2n, o_fk2c, o_fcoef, o_ixn, o_iyn;
  size_t o_cxA, o_cxB, o_cyA, o_cyB, o_ck2c, o_ccoef;
  size_t o_avgx0, o_avgwx, o_avgy0, o_avgwy;
  size_t o_rx, o_rwx, o_ry, o_rwy, o_px, o_pwx, o_py, o_pwy;
  size_t o_slabs, o_slabA, o_slabB, o_xmap, o_fac, o_facscr, o_status, o_growth, o_tasks, o_tcoef;
  size_t o_swf, o_swg, o_swu, o_swB, o_swscr;
  size_t o_tgx0, o_tgx1, o_tgres, o_tgrc, o_tgec, o_cvin, o_cvout;
  size_t o_V, o_Z, o_w, o_part, o_hbuf, o_stats, o_bconj;
  size_t o_red, o_ctr, o_setup, o_ttmp;  // chunk tips/heads, arrival counters, setup scratch (aliases V, Z)
  size_t n_slabA = 0, n_xmap = 0, n_fac = 0, n_tasks = 0;
  size_t total = 0;
};

constexpr int kPartBlocks = 512;

struct Stage {
  int residual;
  int first, ntasks;
  int nl;        // thickest slab among the stage's tasks
  double bytes;  // algorithmic bytes per complex unit (times sizeof(T) at launch)
  double fac;    // the factor part of bytes (shared by all right-hand sides of a batch)
};

// Event-pair timing per kernel class.
struct Prof {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[HSP_PROF_NCLASS];
  size_t used[HSP_PROF_NCLASS] = {};
  double bytes[HSP_PROF_NCLASS] = {};
  long long n[HSP_PROF_NCLASS] = {};
};

}  // namespace hsp

namespace hsp {
struct D3Ctx;  // the three-dimensional path (hsp3d.hip)
void destroy_d3(D3Ctx* d);
}  // namespace hsp

struct hsp_ctx {
  hsp::Plan P;
  hsp::D3Ctx* d3 = nullptr;  // set for dim = 3
  hsp_grid grid;
  hsp_options opt;
  int J = 0;
  double omega = 0, c_pml = 0, h = 0;
  char* ws = nullptr;
  hsp::LevelDev fine{}, coarse{}, dd{};
  hsp::TransferDev tr{};
  hsp::SlabDev* slabs_dev = nullptr;
  std::vector<hsp::SlabDev> slabs_host;
  std::vector<hsp::Stage> stages;
  hsp::TaskDev* tasks_dev = nullptr;
  std::vector<hsp::TaskDev> tasks_host;
  void* factors = nullptr;
  const hsp::cd* tcoef = nullptr;  // transmission coefficients per task (batched stages)
  hsp::Prof prof;
  double growth = 0;   // largest growth factor of the slab factorization
  int tuned_rb = 0;    // right-hand-side tile chosen by hsp_tune_batch (0: none)
  int tuned_nact = 0;  // batch size it was chosen for
  ~hsp_ctx() {
    if (d3) hsp::destroy_d3(d3);
    for (int c = 0; c < HSP_PROF_NCLASS; ++c)
      for (auto& e : prof.ev[c]) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
  template <class T>
  hsp::cx<T>* at(size_t off) const {
    return reinterpret_cast<hsp::cx<T>*>(ws + off);
  }
  template <class X>
  X* raw(size_t off) const {
    return reinterpret_cast<X*>(ws + off);
  }
};

namespace hsp {

// Event-pair timing of one kernel class around the launches in between
// (no-ops unless timing is enabled on the handle).
void prof_begin(hsp_ctx* C, int cls, hipStream_t s);
void prof_end(hsp_ctx* C, int cls, hipStream_t s, double bytes);

// Size plan of a 2-D setup workspace (validates the arguments).
hsp_status make_plan(const hsp_grid* g, int J, const hsp_options* o, Plan& P);
// Task list and stages of the sweep of Table 3 (X, UD or NX) from the
// partition in C->P (beta, bt, x0, x1) and C->J, C->opt.sweep, C->opt.ncell.
void build_schedule(hsp_ctx* C);
// Groups of the NX-sweep: jc[0..N] (jc[0] = 0, jc[N] = J + 1) and the centres
// jm[1..N] (jm[0] unused); HSP_EINVAL when a group would hold no slab.
hsp_status nx_cells(int J, int N, std::vector<int>& jc, std::vector<int>& jm);
// Transmission buffers and the largest number of slab solves in one stage of
// the sweep selected by the options (HSP_EINVAL for a bad NX grouping).
hsp_status sweep_shape(int J, const hsp_options* o, int* nbuf, int* maxtask);

// ---- the three-dimensional path (hsp3d.hip) --------------------------------
hsp_status d3_workspace_size(const hsp_grid* g, int J, const hsp_options* o, size_t* bytes);
hsp_status d3_setup(const double* c_dev, double omega, const hsp_grid* g, int J, const hsp_options* o, void* ws,
                    size_t ws_bytes, hipStream_t s, hsp_ctx** out);
void d3_precond(hsp_ctx* C, const cd* r, cd* z, hipStream_t s);
// fine operator: y = A x (mode 0) or y = b - A x (mode 1), complex128
void d3_fine_apply(hsp_ctx* C, int mode, const cd* x, const cd* b, cd* y, hipStream_t s);
hsp_status d3_rhs(hsp_ctx* C, const cd* f, cd* b, hipStream_t s);
hsp_status d3_apply_level_operator(hsp_ctx* C, int level, const cd* x, cd* y, hipStream_t s);
hsp_status d3_restrict(hsp_ctx* C, const cd* rf, cd* rc, hipStream_t s);
hsp_status d3_prolong_add(hsp_ctx* C, const cd* ec, cd* xf, hipStream_t s);
hsp_status d3_smooth(hsp_ctx* C, const cd* r, cd* x, int steps, hipStream_t s);
hsp_status d3_sweep(hsp_ctx* C, const cd* f, cd* u, hipStream_t s);
hsp_status d3_slab_solve(hsp_ctx* C, int j, const cd* b, cd* x, hipStream_t s);
void d3_info(const hsp_ctx* C, hsp_info* info);
// Reports a failed stage launch since the last check.
hsp_status d3_check(hsp_ctx* C);

}  // namespace hsp
