// Host side of the library: the C ABI of include/hsp.h, workspace planning,
// setup (PML profiles, PML-aware coarse mesh, slab partition and slab
// operators), the sweep schedules of Table 3, the two-grid cycle of Sec. 4
// and right-preconditioned FGMRES.  All vector work runs in the kernels of
// stencil.hip, transfer.hip, slab.hip and blas.hip.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hsp.h"
#include "internal.h"

using namespace hsp;

namespace {

thread_local std::string g_err = "no error";

hsp_status fail(hsp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(HSP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
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

// Per-axis level arrays (see LevelDev in common.h).
void axis_arrays(const AxisH& ax, int kind, double omega, const std::vector<double>* sig_override_x,
                 std::vector<cd>& A, std::vector<cd>& B) {
  (void)sig_override_x;
  const int N = (int)ax.x.size() - 1;
  if (kind == 5) {
    A.resize(N);
    B.resize(N + 1);
    for (int p = 0; p < N; ++p) A[p] = to_cd(alpha_of(ax.sig(0.5 * (ax.x[p] + ax.x[p + 1])), omega));
    for (int i = 0; i <= N; ++i) B[i] = to_cd(1.0 / alpha_of(ax.sig(ax.x[i]), omega));
  } else {
    A.resize(N);
    B.resize(N);
    for (int p = 0; p < N; ++p) {
      const double hp = ax.x[p + 1] - ax.x[p];
      const cplx al = alpha_of(ax.sig(0.5 * (ax.x[p] + ax.x[p + 1])), omega);
      A[p] = to_cd(al / hp);
      B[p] = to_cd(hp / al);
    }
  }
}

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
  size_t tsize = 16;                      // bytes per preconditioner complex
  int m = 0;                              // FGMRES restart
  // workspace offsets
  size_t o_fxA, o_fxB, o_fyA, o_fyB, o_k2n, o_fk2c, o_fcoef, o_ixn, o_iyn;
  size_t o_cxA, o_cxB, o_cyA, o_cyB, o_ck2c, o_ccoef;
  size_t o_avgx0, o_avgwx, o_avgy0, o_avgwy;
  size_t o_rx, o_rwx, o_ry, o_rwy, o_px, o_pwx, o_py, o_pwy;
  size_t o_slabs, o_slabA, o_slabB, o_xmap, o_fac, o_facscr, o_status, o_tasks;
  size_t o_swf, o_swg, o_swu, o_swB, o_swscr;
  size_t o_tgx0, o_tgx1, o_tgres, o_tgrc, o_tgec, o_cvin, o_cvout;
  size_t o_V, o_Z, o_w, o_part, o_hbuf, o_stats, o_bconj;
  size_t o_red, o_ctr, o_setup, o_ttmp;  // chunk tips/heads, arrival counters, setup scratch (aliases V, Z)
  size_t n_slabA = 0, n_xmap = 0, n_fac = 0, n_tasks = 0;
  size_t total = 0;
};

constexpr int kPartBlocks = 512;

hsp_status validate(const hsp_grid* g, int J, const hsp_options* o) {
  if (!g || !o) return fail(HSP_EINVAL, "null grid or options");
  if (g->dim != 2) return fail(HSP_EINVAL, "only dim = 2 is supported");
  for (int a = 0; a < 2; ++a) {
    if (g->n[a] < 1) return fail(HSP_EINVAL, "n must be >= 1");
    if (g->pml[a] < 0) return fail(HSP_EINVAL, "pml must be >= 0");
  }
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(HSP_EINVAL, "h must be positive and finite");
  if (J < 1) return fail(HSP_EINVAL, "J must be >= 1");
  if (o->w_dd < 1) return fail(HSP_EINVAL, "w_dd must be >= 1");
  if (o->nu < 0) return fail(HSP_EINVAL, "nu must be >= 0");
  if (o->restart < 1) return fail(HSP_EINVAL, "restart must be >= 1");
  if (o->fine_stencil != 5 && o->fine_stencil != 9) return fail(HSP_EINVAL, "fine_stencil must be 5 or 9");
  if (o->sweep != HSP_SWEEP_X && o->sweep != HSP_SWEEP_UD) return fail(HSP_EINVAL, "bad sweep");
  if (o->precision != HSP_FP64 && o->precision != HSP_MIXED) return fail(HSP_EINVAL, "bad precision");
  if (!std::isfinite(o->omega_jac)) return fail(HSP_EINVAL, "bad omega_jac");
  if (o->chunk < 0 || o->chunk > kMaxChunk) return fail(HSP_EINVAL, "chunk must be in 0..64");
  return HSP_OK;
}

// Partition beta_0..beta_J of n1 layers: outer-PML layers join the first and
// last cores, interior layers split evenly (integer arithmetic).
std::vector<int> partition(int n1, int w_outer, int J) {
  std::vector<int> b(J + 1);
  const int n_int = n1 - 2 * w_outer;
  b[0] = 0;
  for (int j = 1; j < J; ++j) b[j] = w_outer + (int)(((long long)j * n_int + J / 2) / J);
  b[J] = n1;
  return b;
}

void coarse_map(int N, int w, std::vector<int>& ifp, std::vector<char>& ref) {
  ifp.clear();
  for (int i = 0; i <= w; ++i) ifp.push_back(i);
  const int nint = N - 2 * w;
  for (int m = 1; m <= nint / 2; ++m) ifp.push_back(w + 2 * m);
  for (int q = 1; q <= w; ++q) ifp.push_back(N - w + q);
  ref.resize(ifp.size() - 1);
  for (size_t p = 0; p + 1 < ifp.size(); ++p) ref[p] = (ifp[p + 1] - ifp[p]) == 2;
}

hsp_status make_plan(const hsp_grid* g, int J, const hsp_options* o, Plan& P) {
  hsp_status st = validate(g, J, o);
  if (st != HSP_OK) return st;
  P.Nf1 = g->n[0] + 1 + 2 * g->pml[0];
  P.Nf2 = g->n[1] + 1 + 2 * g->pml[1];
  P.nf1 = P.Nf1 - 1;
  P.nf2 = P.Nf2 - 1;
  P.two_grid = o->two_grid ? 1 : 0;
  P.fine_kind = o->fine_stencil;
  P.tsize = (o->precision == HSP_MIXED) ? sizeof(cf) : sizeof(cd);
  P.m = o->restart;
  int w_dd_outer;
  if (P.two_grid) {
    for (int a = 0; a < 2; ++a) {
      const int N = a == 0 ? P.Nf1 : P.Nf2;
      if ((N - 2 * g->pml[a]) % 2 != 0 || N - 2 * g->pml[a] < 2)
        return fail(HSP_EINVAL, "two-grid needs an even, positive interior cell count per axis");
    }
    coarse_map(P.Nf1, g->pml[0], P.ifp1, P.ref1);
    coarse_map(P.Nf2, g->pml[1], P.ifp2, P.ref2);
    P.nc1 = (int)P.ifp1.size() - 2;
    P.nc2 = (int)P.ifp2.size() - 2;
    P.dd_kind = 9;
    P.dd_n1 = P.nc1;
    P.dd_n2 = P.nc2;
  } else {
    P.dd_kind = P.fine_kind;
    P.dd_n1 = P.nf1;
    P.dd_n2 = P.nf2;
  }
  w_dd_outer = g->pml[0];
  if (P.dd_n1 - 2 * w_dd_outer < J) return fail(HSP_EINVAL, "too many slabs for the interior layers");
  P.beta = partition(P.dd_n1, w_dd_outer, J);
  P.bt = P.beta;
  for (int j = 1; j < J; ++j) P.bt[j] = P.beta[j] - 1;
  P.x0.resize(J);
  P.x1.resize(J);
  P.nl_max = 0;
  for (int j = 1; j <= J; ++j) {
    if (P.beta[j] - P.beta[j - 1] < 3) return fail(HSP_EINVAL, "a core is thinner than 3 layers");
    P.x0[j - 1] = (j == 1) ? 1 : P.beta[j - 1] - o->w_dd;
    P.x1[j - 1] = (j == J) ? P.dd_n1 : P.beta[j] + o->w_dd;
    if (P.x0[j - 1] < 1 || P.x1[j - 1] > P.dd_n1) return fail(HSP_EINVAL, "DD-PML layers leave the domain");
    P.nl_max = std::max(P.nl_max, P.x1[j - 1] - P.x0[j - 1] + 1);
  }
  if (P.nl_max > kMaxSlabLayers)
    return fail(HSP_EINVAL, "slab thicker than " + std::to_string(kMaxSlabLayers) + " layers: use more slabs");
  if (o->chunk > 0) {
    P.chunk = o->chunk;
  } else {
    P.chunk = (int)std::ceil(std::sqrt(2.0 * P.dd_n2));
    P.chunk = std::max(8, std::min(kMaxChunk, P.chunk));
  }
  P.chunk = std::min(P.chunk, P.dd_n2);
  P.nchunk = (P.dd_n2 + P.chunk - 1) / P.chunk;

  // ---- workspace layout
  Carver c;
  const size_t nf = (size_t)P.nf1 * P.nf2;
  const size_t nd = (size_t)P.dd_n1 * P.dd_n2;
  const int N1 = P.Nf1, N2 = P.Nf2;
  // fine level arrays (kind 5: A has N entries, B N+1; kind 9: N and N)
  P.o_fxA = c.take((N1 + 1) * sizeof(cd));
  P.o_fxB = c.take((N1 + 1) * sizeof(cd));
  P.o_fyA = c.take((N2 + 1) * sizeof(cd));
  P.o_fyB = c.take((N2 + 1) * sizeof(cd));
  P.o_k2n = c.take(nf * sizeof(double));
  if (P.fine_kind == 9) {
    P.o_fk2c = c.take((size_t)N1 * N2 * sizeof(double));
    P.o_fcoef = c.take((size_t)N1 * N2 * 3 * sizeof(double));
  }
  P.o_ixn = c.take((N1 + 1) * sizeof(cd));
  P.o_iyn = c.take((N2 + 1) * sizeof(cd));
  const int Nc1 = P.dd_n1 + 1, Nc2 = P.dd_n2 + 1;  // DD level cells
  if (P.two_grid) {
    P.o_cxA = c.take(Nc1 * sizeof(cd));
    P.o_cxB = c.take(Nc1 * sizeof(cd));
    P.o_cyA = c.take(Nc2 * sizeof(cd));
    P.o_cyB = c.take(Nc2 * sizeof(cd));
    P.o_ck2c = c.take((size_t)Nc1 * Nc2 * sizeof(double));
    P.o_ccoef = c.take((size_t)Nc1 * Nc2 * 3 * sizeof(double));
    P.o_rx = c.take((size_t)P.nc1 * 3 * sizeof(int));
    P.o_rwx = c.take((size_t)P.nc1 * 3 * sizeof(double));
    P.o_ry = c.take((size_t)P.nc2 * 3 * sizeof(int));
    P.o_rwy = c.take((size_t)P.nc2 * 3 * sizeof(double));
    P.o_px = c.take((size_t)P.nf1 * 2 * sizeof(int));
    P.o_pwx = c.take((size_t)P.nf1 * 2 * sizeof(double));
    P.o_py = c.take((size_t)P.nf2 * 2 * sizeof(int));
    P.o_pwy = c.take((size_t)P.nf2 * 2 * sizeof(double));
  }
  const int nav1 = std::max(N1, Nc1), nav2 = std::max(N2, Nc2);
  P.o_avgx0 = c.take(nav1 * sizeof(int));
  P.o_avgwx = c.take((size_t)nav1 * 3 * sizeof(double));
  P.o_avgy0 = c.take(nav2 * sizeof(int));
  P.o_avgwy = c.take((size_t)nav2 * 3 * sizeof(double));
  // slabs
  P.n_slabA = 0;
  P.n_xmap = 0;
  P.n_fac = 0;
  for (int j = 0; j < J; ++j) {
    const int nl = P.x1[j] - P.x0[j] + 1;
    P.n_slabA += (size_t)(nl + 2);
    P.n_xmap += (size_t)(nl + 1);
    P.n_fac += slab_factor_elems(nl, P.dd_n2);
  }
  P.o_red = c.take((size_t)2 * 2 * P.nchunk * P.nl_max * P.tsize);
  P.o_ctr = c.take(64 * sizeof(int));
  P.o_slabs = c.take(J * sizeof(SlabDev));
  P.o_slabA = c.take(P.n_slabA * sizeof(cd));
  P.o_slabB = c.take(P.n_slabA * sizeof(cd));
  P.o_xmap = c.take(P.n_xmap * sizeof(int));
  P.o_fac = c.take(P.n_fac * P.tsize);
  P.o_facscr = c.take((size_t)J * kMaxSlabLayers * kMaxSlabLayers * sizeof(cd));
  P.o_status = c.take(64);
  P.n_tasks = 2 * (size_t)J + 8;
  P.o_tasks = c.take(P.n_tasks * sizeof(TaskDev));
  // sweep vectors (DD level, precision of the preconditioner)
  P.o_swf = c.take(nd * P.tsize);
  P.o_swg = c.take(nd * P.tsize);
  P.o_swu = c.take(nd * P.tsize);
  P.o_swB = c.take((size_t)2 * 2 * P.dd_n2 * P.tsize);
  P.o_swscr = c.take((size_t)2 * P.dd_n2 * P.nl_max * P.tsize);
  // two-grid vectors
  P.o_tgx0 = c.take(nf * P.tsize);
  P.o_tgx1 = c.take(nf * P.tsize);
  if (P.two_grid) {
    P.o_tgres = c.take(nf * sizeof(cd));
    P.o_tgrc = c.take(nd * P.tsize);
    P.o_tgec = c.take(nd * P.tsize);
  }
  P.o_cvin = c.take(std::max(nf, nd) * sizeof(cd));
  P.o_cvout = c.take(std::max(nf, nd) * sizeof(cd));
  // FGMRES basis V, Z; during setup the same region holds the FP64 slab
  // factors and the temporaries of the transfer-matrix kernel
  size_t setup_elems = 0;
  for (int j = 0; j < J; ++j) setup_elems += slab_setup_elems(P.x1[j] - P.x0[j] + 1, P.dd_n2);
  const size_t ttmp_elems = (size_t)J * P.nchunk * kTransferTmpElems;
  const size_t vz_bytes = (size_t)(2 * P.m + 1) * nf * sizeof(cd);
  const size_t setup_bytes = (setup_elems + ttmp_elems) * sizeof(cd) + 512;
  P.o_V = c.take(std::max(vz_bytes, setup_bytes));
  P.o_Z = P.o_V + (size_t)(P.m + 1) * nf * sizeof(cd);
  P.o_setup = P.o_V;
  P.o_ttmp = P.o_V + ((setup_elems * sizeof(cd) + 255) & ~(size_t)255);
  P.o_w = c.take(nf * sizeof(cd));
  P.o_bconj = c.take(nf * sizeof(cd));
  P.o_part = c.take((size_t)kPartBlocks * (P.m + 2) * sizeof(cd));
  P.o_hbuf = c.take((size_t)(2 * (P.m + 2) + 2) * sizeof(cd));
  P.o_stats = c.take(8 * sizeof(double));
  P.total = c.off + 256;
  return HSP_OK;
}

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
  size_t used[HSP_PROF_NCLASS] = {0, 0, 0, 0, 0};
  double bytes[HSP_PROF_NCLASS] = {0, 0, 0, 0, 0};
  long long n[HSP_PROF_NCLASS] = {0, 0, 0, 0, 0};
};

}  // namespace

struct hsp_ctx {
  Plan P;
  hsp_grid grid;
  hsp_options opt;
  int J = 0;
  double omega = 0, c_pml = 0, h = 0;
  char* ws = nullptr;
  LevelDev fine{}, coarse{}, dd{};
  TransferDev tr{};
  SlabDev* slabs_dev = nullptr;
  std::vector<SlabDev> slabs_host;
  std::vector<Stage> stages;
  TaskDev* tasks_dev = nullptr;
  std::vector<TaskDev> tasks_host;
  void* factors = nullptr;
  Prof prof;
  int tuned_rb = 0;    // right-hand-side tile chosen by hsp_tune_batch (0: none)
  int tuned_nact = 0;  // batch size it was chosen for
  ~hsp_ctx() {
    for (int c = 0; c < HSP_PROF_NCLASS; ++c)
      for (auto& e : prof.ev[c]) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
  template <class T>
  cx<T>* at(size_t off) const {
    return reinterpret_cast<cx<T>*>(ws + off);
  }
  template <class X>
  X* raw(size_t off) const {
    return reinterpret_cast<X*>(ws + off);
  }
};

namespace {

// ---------------------------------------------------------------------------
// Sweep schedules (Table 3)
// ---------------------------------------------------------------------------
void build_schedule(hsp_ctx* C) {
  const Plan& P = C->P;
  const int J = C->J;
  const auto& be = P.beta;
  const auto& bt = P.bt;
  std::vector<TaskDev>& T = C->tasks_host;
  std::vector<Stage>& S = C->stages;
  T.clear();
  S.clear();
  bool written[2] = {false, false};
  auto blank = [](int j) {
    TaskDev t;
    std::memset(&t, 0, sizeof(t));
    t.slab = j - 1;
    return t;
  };
  auto fwd = [&](int j, int src, int buf) {
    TaskDev t = blank(j);
    t.a = t.at = be[j - 1];
    t.b = t.bt = be[j];
    t.t1 = (j > 1 && written[buf]) ? 1 : 0;
    t.bin_f = buf;
    t.beta_in = be[j - 1];
    t.t2 = (j < J) ? 1 : 0;
    t.bout_f = buf;
    t.beta_out = be[j];
    t.src = src;
    return t;
  };
  auto bwd = [&](int j, int src, int buf) {
    TaskDev t = blank(j);
    t.a = t.at = bt[j - 1];
    t.b = t.bt = bt[j];
    t.t3 = (j < J && written[buf]) ? 1 : 0;
    t.bin_b = buf;
    t.bt_in = bt[j];
    t.t4 = (j > 1) ? 1 : 0;
    t.bout_b = buf;
    t.bt_out = bt[j - 1];
    t.src = src;
    return t;
  };
  auto push_stage = [&](std::vector<TaskDev> ts) {
    Stage s{0, (int)T.size(), (int)ts.size(), 0, 0.0, 0.0};
    const double n2 = P.dd_n2;
    for (auto& t : ts) {
      T.push_back(t);
      const int nl = P.x1[t.slab] - P.x0[t.slab] + 1;
      s.nl = std::max(s.nl, nl);
      // factors G, E and the couplings; gathered rows; u read-modify-write;
      // transmission layers in and out (complex units)
      s.fac += n2 * (2.0 * nl * nl + 3.0 * nl);
      s.bytes += n2 * (2.0 * nl * nl + 3.0 * nl) + n2 * (t.b - t.a) + 2.0 * n2 * (t.bt - t.at) +
                 2.0 * n2 * (t.t1 + t.t2 + t.t3 + t.t4);
    }
    if (s.ntasks > 0) S.push_back(s);
  };
  auto mark = [&](const TaskDev& t) {
    if (t.t2) written[t.bout_f] = true;
    if (t.t4) written[t.bout_b] = true;
  };
  if (C->opt.sweep == HSP_SWEEP_UD) {
    for (int j = 1; j <= J; ++j) {
      TaskDev t = fwd(j, 0, 0);
      push_stage({t});
      mark(t);
    }
    S.push_back(Stage{1, 0, 0, 0, 0.0, 0.0});
    for (int j = J; j >= 1; --j) {
      TaskDev t = bwd(j, 1, 0);
      push_stage({t});
      mark(t);
    }
    return;
  }
  const int jm = J / 2 + 1;
  const int nA = std::max(jm - 1, J - jm);
  for (int s = 1; s <= nA; ++s) {
    std::vector<TaskDev> ts;
    if (s <= jm - 1) ts.push_back(fwd(s, 0, 0));
    if (J + 1 - s >= jm + 1) ts.push_back(bwd(J + 1 - s, 0, 1));
    for (auto& t : ts) mark(t);
    push_stage(ts);
  }
  {  // MidSolveIn
    TaskDev t = blank(jm);
    t.a = t.at = be[jm - 1];
    t.b = t.bt = bt[jm];
    t.t1 = (jm > 1 && written[0]) ? 1 : 0;
    t.bin_f = 0;
    t.beta_in = be[jm - 1];
    t.t3 = (jm < J && written[1]) ? 1 : 0;
    t.bin_b = 1;
    t.bt_in = bt[jm];
    push_stage({t});
  }
  S.push_back(Stage{1, 0, 0, 0, 0.0, 0.0});
  written[0] = written[1] = false;
  {  // MidSolveOut: forward output -> buffer 1, backward output -> buffer 0
    TaskDev t = blank(jm);
    t.a = t.at = bt[jm - 1];
    t.b = t.bt = be[jm];
    t.t2 = (jm < J) ? 1 : 0;
    t.bout_f = 1;
    t.beta_out = be[jm];
    t.t4 = (jm > 1) ? 1 : 0;
    t.bout_b = 0;
    t.bt_out = bt[jm - 1];
    t.src = 1;
    push_stage({t});
    mark(t);
  }
  for (int s = 1; s <= nA; ++s) {
    std::vector<TaskDev> ts;
    if (jm - s >= 1) ts.push_back(bwd(jm - s, 1, 0));
    if (jm + s <= J) ts.push_back(fwd(jm + s, 1, 1));
    for (auto& t : ts) mark(t);
    push_stage(ts);
  }
}

// ---------------------------------------------------------------------------
// Sweep, two-grid cycle and preconditioner
// ---------------------------------------------------------------------------
void prof_begin(hsp_ctx* C, int cls, hipStream_t s) {
  Prof& P = C->prof;
  if (!P.on) return;
  if (P.used[cls] == P.ev[cls].size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    P.ev[cls].push_back({a, b});
  }
  (void)hipEventRecord(P.ev[cls][P.used[cls]].first, s);
}

void prof_end(hsp_ctx* C, int cls, hipStream_t s, double bytes) {
  Prof& P = C->prof;
  if (!P.on || P.used[cls] >= P.ev[cls].size()) return;
  (void)hipEventRecord(P.ev[cls][P.used[cls]].second, s);
  ++P.used[cls];
  ++P.n[cls];
  P.bytes[cls] += bytes;
}

template <class T>
void run_sweep(hsp_ctx* C, const cx<T>* f, cx<T>* u, hipStream_t s) {
  const Plan& P = C->P;
  const size_t nd = (size_t)P.dd_n1 * P.dd_n2;
  cx<T>* g = C->at<T>(P.o_swg);
  launch_zero<T>(u, nd, s);
  for (const Stage& st : C->stages) {
    if (st.residual) {
      prof_begin(C, HSP_PROF_COARSE, s);
      launch_stencil<T, T, T, T>(C->dd, 1, u, f, g, 0.0, s);
      // u, f read, g written, medium per node
      prof_end(C, HSP_PROF_COARSE, s, (double)nd * (3.0 * sizeof(cx<T>) + 4.0 * sizeof(double)));
    } else {
      prof_begin(C, HSP_PROF_STAGE, s);
      launch_stage<T>(C->tasks_dev + st.first, st.ntasks, C->slabs_dev, C->dd, f, g, u, C->at<T>(P.o_swB),
                      C->at<T>(P.o_swscr), reinterpret_cast<const cx<T>*>(C->factors), P.nl_max, st.nl, P.chunk,
                      P.nchunk, C->at<T>(P.o_red), C->raw<int>(P.o_ctr), s);
      prof_end(C, HSP_PROF_STAGE, s, st.bytes * sizeof(cx<T>));
    }
  }
}

template <class T>
void run_precond(hsp_ctx* C, const cd* r, cd* z, hipStream_t s) {
  const Plan& P = C->P;
  const size_t nf = (size_t)P.nf1 * P.nf2;
  if (!P.two_grid) {
    if (sizeof(T) == sizeof(double)) {
      run_sweep<T>(C, reinterpret_cast<const cx<T>*>(r), reinterpret_cast<cx<T>*>(z), s);
    } else {
      cx<T>* fin = C->at<T>(P.o_swf);
      cx<T>* uout = C->at<T>(P.o_tgx0);
      launch_convert<T, double>(r, fin, nf, 0, s);
      run_sweep<T>(C, fin, uout, s);
      launch_convert<double, T>(uout, z, nf, 0, s);
    }
    return;
  }
  const double wj = C->opt.omega_jac;
  const int nu = C->opt.nu;
  cx<T>* xa = C->at<T>(P.o_tgx0);
  cx<T>* xb = C->at<T>(P.o_tgx1);
  const size_t nc = (size_t)P.nc1 * P.nc2;
  // bytes of one smoothing step: r, x read, x written, k^2 per node
  const double jb = (double)nf * (sizeof(cd) + 2.0 * sizeof(cx<T>) + sizeof(double));
  // pre-smoothing from x = 0
  prof_begin(C, HSP_PROF_SMOOTH, s);
  if (nu > 0) {
    launch_stencil<T, T, double, T>(C->fine, 2, (const cx<T>*)nullptr, r, xa, wj, s);
    for (int k = 1; k < nu; ++k) {
      launch_stencil<T, T, double, T>(C->fine, 2, xa, r, xb, wj, s);
      std::swap(xa, xb);
    }
  } else {
    launch_zero<T>(xa, nf, s);
  }
  // coarse-grid correction: r_c = P^T (r - A x), e_c = P_X r_c, x += P e_c
  cd* res = C->at<double>(P.o_tgres);
  launch_stencil<double, T, double, double>(C->fine, 1, xa, r, res, 0.0, s);
  prof_end(C, HSP_PROF_SMOOTH, s, nu * jb + (double)nf * (2.0 * sizeof(cd) + sizeof(cx<T>) + sizeof(double)));
  cx<T>* rc = C->at<T>(P.o_tgrc);
  cx<T>* ec = C->at<T>(P.o_tgec);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  launch_restrict<double, T>(C->tr, res, rc, s);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nf * sizeof(cd) + (double)nc * sizeof(cx<T>));
  run_sweep<T>(C, rc, ec, s);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  launch_prolong_add<T, T>(C->tr, ec, xa, s);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nc * sizeof(cx<T>) + 2.0 * nf * sizeof(cx<T>));
  // post-smoothing, the last step writes z in double
  if (nu == 0) {
    launch_convert<double, T>(xa, z, nf, 0, s);
    return;
  }
  prof_begin(C, HSP_PROF_SMOOTH, s);
  for (int k = 0; k < nu; ++k) {
    if (k == nu - 1) {
      launch_stencil<T, T, double, double>(C->fine, 2, xa, r, z, wj, s);
    } else {
      launch_stencil<T, T, double, T>(C->fine, 2, xa, r, xb, wj, s);
      std::swap(xa, xb);
    }
  }
  prof_end(C, HSP_PROF_SMOOTH, s, nu * jb);
}

void precond(hsp_ctx* C, const cd* r, cd* z, hipStream_t s) {
  if (C->opt.precision == HSP_MIXED)
    run_precond<float>(C, r, z, s);
  else
    run_precond<double>(C, r, z, s);
}


// ---------------------------------------------------------------------------
// Batched right-hand sides: layout of the caller's batch workspace
// ---------------------------------------------------------------------------
constexpr int kMaxTile = 8;

// (task, tile) slots of a stage, times the tile: >= 2 ceil(R/rb) rb for every rb <= 8
inline size_t batch_slots(int R) { return 2 * (size_t)(R + kMaxTile - 1); }

struct BatchLayout {
  int R = 0, m = 0, nblk = 0;
  size_t hs = 0;  // hb entries per right-hand side: [h1 (m+1) | h2 (m+1) | nrm2 | spare]
  size_t o_xa, o_xb, o_res, o_rc, o_ec, o_swf, o_swg, o_swu, o_swB, o_scr, o_red, o_ctr;
  size_t o_V, o_Z, o_w, o_bc, o_part, o_hb, o_act, o_upd, o_y;
  size_t total = 0;
};

BatchLayout batch_layout(const Plan& P, int R, int m) {
  BatchLayout B;
  B.R = R;
  B.m = m;
  Carver c;
  const size_t nf = (size_t)P.nf1 * P.nf2, nd = (size_t)P.dd_n1 * P.dd_n2, T = P.tsize;
  const size_t slots = batch_slots(R);
  B.o_xa = c.take(R * nf * T);
  B.o_xb = c.take(R * nf * T);
  B.o_res = c.take(P.two_grid ? R * nf * sizeof(cd) : 0);
  B.o_rc = c.take(P.two_grid ? R * nd * T : 0);
  B.o_ec = c.take(P.two_grid ? R * nd * T : 0);
  B.o_swf = c.take(R * nd * T);
  B.o_swg = c.take(R * nd * T);
  B.o_swu = c.take(R * nd * T);
  B.o_swB = c.take(R * 4 * (size_t)P.dd_n2 * T);
  B.o_scr = c.take(slots * P.dd_n2 * P.nl_max * T);
  B.o_red = c.take(slots * 2 * P.nchunk * P.nl_max * T);
  B.o_ctr = c.take(2 * slots * sizeof(int));
  B.nblk = batch_dot_blocks(nf, R);
  B.hs = 2 * (size_t)(m + 2) + 2;
  B.o_V = c.take((size_t)R * (m + 1) * nf * sizeof(cd));
  B.o_Z = c.take((size_t)R * m * nf * sizeof(cd));
  B.o_w = c.take(R * nf * sizeof(cd));
  B.o_bc = c.take(R * nf * sizeof(cd));
  B.o_part = c.take((size_t)2 * R * (m + 1) * B.nblk * sizeof(cd));
  B.o_hb = c.take(R * B.hs * sizeof(cd));
  B.o_act = c.take(R * sizeof(int));
  B.o_upd = c.take(R * sizeof(int));
  B.o_y = c.take((size_t)R * m * sizeof(cd));
  B.total = c.off + 256;
  return B;
}

template <class X>
X* bat(void* ws, size_t off) {
  return reinterpret_cast<X*>(reinterpret_cast<char*>(ws) + off);
}

// Default right-hand-side tile: the largest that still gives the stage
// launches about two work items per compute unit.
int default_tile(const hsp_ctx* C, int nact) {
  if (C->tuned_rb > 0 && C->tuned_nact == nact) return C->tuned_rb;
  for (int rb = kMaxTile; rb > 1; rb /= 2)
    if (2 * C->P.nchunk * ((nact + rb - 1) / rb) >= 512) return rb;
  return 1;
}

template <class T>
void run_sweep_batch(hsp_ctx* C, const BatchLayout& B, void* ws, int nact, int rb, const cx<T>* f, cx<T>* u,
                     hipStream_t s) {
  const Plan& P = C->P;
  const size_t nd = (size_t)P.dd_n1 * P.dd_n2;
  cx<T>* g = bat<cx<T>>(ws, B.o_swg);
  launch_zero<T>(u, (size_t)nact * nd, s);
  BIdx bd;
  bd.ld = nd;
  for (const Stage& st : C->stages) {
    if (st.residual) {
      prof_begin(C, HSP_PROF_COARSE, s);
      launch_stencil<T, T, T, T>(C->dd, 1, u, f, g, 0.0, s, nact, bd, bd, bd);
      prof_end(C, HSP_PROF_COARSE, s, (double)nact * nd * (3.0 * sizeof(cx<T>) + 4.0 * sizeof(double)));
    } else {
      prof_begin(C, HSP_PROF_STAGE, s);
      launch_stage_batch<T>(C->tasks_dev + st.first, st.ntasks, C->slabs_dev, C->dd, f, g, u,
                            bat<cx<T>>(ws, B.o_swB), bat<cx<T>>(ws, B.o_scr),
                            reinterpret_cast<const cx<T>*>(C->factors), P.nl_max, st.nl, P.chunk, P.nchunk, nact,
                            rb, nd, bat<cx<T>>(ws, B.o_red), bat<int>(ws, B.o_ctr), s);
      prof_end(C, HSP_PROF_STAGE, s, (st.fac + (double)nact * (st.bytes - st.fac)) * sizeof(cx<T>));
    }
  }
}

// z_j = M r_j for nact right-hand sides: r_j at r + br.off(j), z_j at
// z + bz.off(j) (complex128), internal vectors compact per slot j.
template <class T>
void run_precond_batch(hsp_ctx* C, const BatchLayout& B, void* ws, int nact, int rb, const cd* r, BIdx br, cd* z,
                       BIdx bz, hipStream_t s) {
  const Plan& P = C->P;
  const size_t nf = (size_t)P.nf1 * P.nf2, nd = (size_t)P.dd_n1 * P.dd_n2;
  BIdx bf, bdd;
  bf.ld = nf;
  bdd.ld = nd;
  if (!P.two_grid) {
    cx<T>* fin = bat<cx<T>>(ws, B.o_swf);
    cx<T>* uo = bat<cx<T>>(ws, B.o_swu);
    launch_convert<T, double>(r, fin, nf, 0, s, nact, br, bf);
    run_sweep_batch<T>(C, B, ws, nact, rb, fin, uo, s);
    launch_convert<double, T>(uo, z, nf, 0, s, nact, bf, bz);
    return;
  }
  const double wj = C->opt.omega_jac;
  const int nu = C->opt.nu;
  cx<T>* xa = bat<cx<T>>(ws, B.o_xa);
  cx<T>* xb = bat<cx<T>>(ws, B.o_xb);
  const double jb = (double)nact * nf * (sizeof(cd) + 2.0 * sizeof(cx<T>) + sizeof(double));
  prof_begin(C, HSP_PROF_SMOOTH, s);
  if (nu > 0) {
    launch_stencil<T, T, double, T>(C->fine, 2, (const cx<T>*)nullptr, r, xa, wj, s, nact, BIdx{}, br, bf);
    for (int k = 1; k < nu; ++k) {
      launch_stencil<T, T, double, T>(C->fine, 2, xa, r, xb, wj, s, nact, bf, br, bf);
      std::swap(xa, xb);
    }
  } else {
    launch_zero<T>(xa, (size_t)nact * nf, s);
  }
  cd* res = bat<cd>(ws, B.o_res);
  launch_stencil<double, T, double, double>(C->fine, 1, xa, r, res, 0.0, s, nact, bf, br, bf);
  prof_end(C, HSP_PROF_SMOOTH, s,
           nu * jb + (double)nact * nf * (2.0 * sizeof(cd) + sizeof(cx<T>) + sizeof(double)));
  cx<T>* rc = bat<cx<T>>(ws, B.o_rc);
  cx<T>* ec = bat<cx<T>>(ws, B.o_ec);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  launch_restrict<double, T>(C->tr, res, rc, s, nact, bf, bdd);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nact * ((double)nf * sizeof(cd) + (double)nd * sizeof(cx<T>)));
  run_sweep_batch<T>(C, B, ws, nact, rb, rc, ec, s);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  launch_prolong_add<T, T>(C->tr, ec, xa, s, nact, bdd, bf);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nact * ((double)nd * sizeof(cx<T>) + 2.0 * nf * sizeof(cx<T>)));
  if (nu == 0) {
    launch_convert<double, T>(xa, z, nf, 0, s, nact, bf, bz);
    return;
  }
  prof_begin(C, HSP_PROF_SMOOTH, s);
  for (int k = 0; k < nu; ++k) {
    if (k == nu - 1) {
      launch_stencil<T, T, double, double>(C->fine, 2, xa, r, z, wj, s, nact, bf, br, bz);
    } else {
      launch_stencil<T, T, double, T>(C->fine, 2, xa, r, xb, wj, s, nact, bf, br, bf);
      std::swap(xa, xb);
    }
  }
  prof_end(C, HSP_PROF_SMOOTH, s, nu * jb);
}

void precond_batch(hsp_ctx* C, const BatchLayout& B, void* ws, int nact, int rb, const cd* r, BIdx br, cd* z,
                   BIdx bz, hipStream_t s) {
  if (C->opt.precision == HSP_MIXED)
    run_precond_batch<float>(C, B, ws, nact, rb, r, br, z, bz, s);
  else
    run_precond_batch<double>(C, B, ws, nact, rb, r, br, z, bz, s);
}

hsp_status check_batch_args(hsp_ctx* C, int nrhs, int restart, void* ws, size_t bytes, int tile, BatchLayout& B) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  if (nrhs < 0) return fail(HSP_EINVAL, "nrhs must be >= 0");
  if (restart < 1) return fail(HSP_EINVAL, "restart must be >= 1");
  if (tile != 0 && tile != 1 && tile != 2 && tile != 4 && tile != 8)
    return fail(HSP_EINVAL, "tile must be 0 (automatic), 1, 2, 4 or 8");
  if (nrhs == 0) return HSP_OK;
  if (!ws) return fail(HSP_EINVAL, "null batch workspace");
  if (((uintptr_t)ws) & 255) return fail(HSP_EINVAL, "batch workspace must be 256-byte aligned");
  B = batch_layout(C->P, nrhs, restart);
  if (bytes < B.total) return fail(HSP_ENOMEM, "batch workspace too small: need " + std::to_string(B.total) + " bytes");
  return HSP_OK;
}

hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* hsp_last_error(void) { return g_err.c_str(); }

hsp_status hsp_default_options(hsp_options* o) {
  if (!o) return fail(HSP_EINVAL, "null options");
  o->fine_stencil = 5;
  o->two_grid = 0;
  o->w_dd = 4;
  o->S_dd = 0.0;
  o->nu = 3;
  o->omega_jac = 0.8;
  o->sweep = HSP_SWEEP_X;
  o->precision = HSP_FP64;
  o->restart = 40;
  o->chunk = 0;
  return HSP_OK;
}

hsp_status hsp_workspace_size(const hsp_grid* grid, int J, const hsp_options* opt, size_t* bytes) {
  if (!bytes) return fail(HSP_EINVAL, "null bytes");
  Plan P;
  hsp_status st = make_plan(grid, J, opt, P);
  if (st != HSP_OK) return st;
  *bytes = P.total;
  return HSP_OK;
}

hsp_status hsp_setup(const double* c_dev, double omega, const hsp_grid* grid, int J, const hsp_options* opt,
                     void* ws_dev, size_t ws_bytes, void* stream, hsp_handle* out) {
  if (!out) return fail(HSP_EINVAL, "null handle pointer");
  *out = nullptr;
  if (!c_dev || !ws_dev) return fail(HSP_EINVAL, "null device pointer");
  if (!(omega > 0) || !std::isfinite(omega)) return fail(HSP_EINVAL, "omega must be positive and finite");
  if (((uintptr_t)ws_dev) & 255) return fail(HSP_EINVAL, "workspace must be 256-byte aligned");
  hsp_ctx* C = new hsp_ctx();
  hsp_status st = make_plan(grid, J, opt, C->P);
  if (st != HSP_OK) {
    delete C;
    return st;
  }
  if (ws_bytes < C->P.total) {
    delete C;
    return fail(HSP_ENOMEM, "workspace too small: need " + std::to_string(C->P.total) + " bytes");
  }
  C->grid = *grid;
  C->opt = *opt;
  C->J = J;
  C->omega = omega;
  C->h = grid->h;
  C->ws = reinterpret_cast<char*>(ws_dev);
  hipStream_t s = S_(stream);
  Plan& P = C->P;
  auto cleanup = [&](hsp_status e) {
    delete C;
    return e;
  };
#define CHK(expr)                                                                                  \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  const size_t nf = (size_t)P.nf1 * P.nf2;

  // medium statistics: positivity, finiteness, mean for c_pml
  double stats[4];
  launch_stats(c_dev, nf, C->raw<double>(P.o_stats), s);
  CHK(hipGetLastError());
  CHK(hipMemcpyAsync(stats, C->raw<double>(P.o_stats), 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  if (stats[3] > 0) return cleanup(fail(HSP_EINVAL, "c has non-positive or non-finite values"));
  C->c_pml = (grid->c_pml > 0) ? grid->c_pml : stats[0] / (double)nf;
  const double S_o = (grid->S_outer > 0) ? grid->S_outer : 5.0 * grid->pml[0];
  const double S_dd = (opt->S_dd > 0) ? opt->S_dd : 5.0 * opt->w_dd;
  const double h = grid->h;

  // fine axes
  AxisH fx, fy;
  auto make_fine_axis = [&](AxisH& ax, int N, int w) {
    ax.x.resize(N + 1);
    for (int i = 0; i <= N; ++i) ax.x[i] = i * h;
    ax.h_nom = h;
    if (w > 0) {
      ax.sig.left = ax.sig.right = true;
      ax.sig.lo = w * h;
      ax.sig.hi = (N - w) * h;
      const double d = w * h;
      ax.sig.C = S_o * C->c_pml / (d * d * d);
    }
  };
  make_fine_axis(fx, P.Nf1, grid->pml[0]);
  make_fine_axis(fy, P.Nf2, grid->pml[1]);

  std::vector<hipError_t> errs;
  std::vector<std::vector<char>> keep;  // host buffers alive until the final sync
  auto up = [&](size_t off, const void* src, size_t bytes) {
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    errs.push_back(hipMemcpyAsync(C->ws + off, keep.back().data(), bytes, hipMemcpyHostToDevice, s));
  };

  // fine level
  {
    std::vector<cd> A, B;
    axis_arrays(fx, P.fine_kind, omega, nullptr, A, B);
    up(P.o_fxA, A.data(), A.size() * sizeof(cd));
    up(P.o_fxB, B.data(), B.size() * sizeof(cd));
    axis_arrays(fy, P.fine_kind, omega, nullptr, A, B);
    up(P.o_fyA, A.data(), A.size() * sizeof(cd));
    up(P.o_fyB, B.data(), B.size() * sizeof(cd));
    std::vector<cd> ix(P.Nf1 + 1), iy(P.Nf2 + 1);
    for (int i = 0; i <= P.Nf1; ++i) ix[i] = to_cd(1.0 / alpha_of(fx.sig(fx.x[i]), omega));
    for (int k = 0; k <= P.Nf2; ++k) iy[k] = to_cd(1.0 / alpha_of(fy.sig(fy.x[k]), omega));
    up(P.o_ixn, ix.data(), ix.size() * sizeof(cd));
    up(P.o_iyn, iy.data(), iy.size() * sizeof(cd));
  }
  launch_k2_nodes(c_dev, nf, omega, C->raw<double>(P.o_k2n), s);
  C->fine.kind = P.fine_kind;
  C->fine.n1 = P.nf1;
  C->fine.n2 = P.nf2;
  C->fine.h2 = h * h;
  C->fine.xA = C->at<double>(P.o_fxA);
  C->fine.xB = C->at<double>(P.o_fxB);
  C->fine.yA = C->at<double>(P.o_fyA);
  C->fine.yB = C->at<double>(P.o_fyB);
  C->fine.xmap = nullptr;
  if (P.fine_kind == 5) {
    C->fine.k2 = C->raw<double>(P.o_k2n);
    C->fine.coef = nullptr;
  } else {
    // cell k^2 = mean of the 4 corner nodes; coefficients at the fine 1/G
    std::vector<int> x0(P.Nf1), y0(P.Nf2);
    std::vector<double> wx(3 * P.Nf1, 0.0), wy(3 * P.Nf2, 0.0);
    for (int p = 0; p < P.Nf1; ++p) x0[p] = p, wx[3 * p] = wx[3 * p + 1] = 0.5;
    for (int q = 0; q < P.Nf2; ++q) y0[q] = q, wy[3 * q] = wy[3 * q + 1] = 0.5;
    up(P.o_avgx0, x0.data(), x0.size() * sizeof(int));
    up(P.o_avgwx, wx.data(), wx.size() * sizeof(double));
    up(P.o_avgy0, y0.data(), y0.size() * sizeof(int));
    up(P.o_avgwy, wy.data(), wy.size() * sizeof(double));
    launch_cell_average(C->raw<double>(P.o_k2n), P.nf1, P.nf2, C->raw<int>(P.o_avgx0), C->raw<double>(P.o_avgwx),
                        P.Nf1, C->raw<int>(P.o_avgy0), C->raw<double>(P.o_avgwy), P.Nf2, C->raw<double>(P.o_fk2c),
                        s);
    launch_cell_coefs(C->raw<double>(P.o_fk2c), (size_t)P.Nf1 * P.Nf2, h, C->raw<double>(P.o_fcoef), s);
    C->fine.k2 = C->raw<double>(P.o_fk2c);
    C->fine.coef = C->raw<double>(P.o_fcoef);
    CHK(hipStreamSynchronize(s));  // the averaging arrays are reused below
  }

  // DD level axes
  AxisH dx, dy;
  if (P.two_grid) {
    auto make_coarse = [&](const AxisH& fa, const std::vector<int>& ifp, AxisH& ca) {
      ca.x.resize(ifp.size());
      for (size_t i = 0; i < ifp.size(); ++i) ca.x[i] = fa.x[ifp[i]];
      ca.sig = fa.sig;
      ca.h_nom = 2.0 * h;
    };
    make_coarse(fx, P.ifp1, dx);
    make_coarse(fy, P.ifp2, dy);
    const int Nc1 = P.nc1 + 1, Nc2 = P.nc2 + 1;
    std::vector<cd> A, B;
    axis_arrays(dx, 9, omega, nullptr, A, B);
    up(P.o_cxA, A.data(), A.size() * sizeof(cd));
    up(P.o_cxB, B.data(), B.size() * sizeof(cd));
    axis_arrays(dy, 9, omega, nullptr, A, B);
    up(P.o_cyA, A.data(), A.size() * sizeof(cd));
    up(P.o_cyB, B.data(), B.size() * sizeof(cd));
    // coarse cell k^2: (1/2,1/2) on unrefined, (1/4,1/2,1/4) on refined cells
    std::vector<int> x0(Nc1), y0(Nc2);
    std::vector<double> wx(3 * Nc1, 0.0), wy(3 * Nc2, 0.0);
    auto fillw = [](const std::vector<int>& ifp, const std::vector<char>& ref, std::vector<int>& o,
                    std::vector<double>& w) {
      for (size_t p = 0; p < ref.size(); ++p) {
        o[p] = ifp[p];
        if (ref[p]) {
          w[3 * p] = 0.25;
          w[3 * p + 1] = 0.5;
          w[3 * p + 2] = 0.25;
        } else {
          w[3 * p] = 0.5;
          w[3 * p + 1] = 0.5;
        }
      }
    };
    fillw(P.ifp1, P.ref1, x0, wx);
    fillw(P.ifp2, P.ref2, y0, wy);
    up(P.o_avgx0, x0.data(), x0.size() * sizeof(int));
    up(P.o_avgwx, wx.data(), wx.size() * sizeof(double));
    up(P.o_avgy0, y0.data(), y0.size() * sizeof(int));
    up(P.o_avgwy, wy.data(), wy.size() * sizeof(double));
    launch_cell_average(C->raw<double>(P.o_k2n), P.nf1, P.nf2, C->raw<int>(P.o_avgx0), C->raw<double>(P.o_avgwx), Nc1,
                        C->raw<int>(P.o_avgy0), C->raw<double>(P.o_avgwy), Nc2, C->raw<double>(P.o_ck2c), s);
    launch_cell_coefs(C->raw<double>(P.o_ck2c), (size_t)Nc1 * Nc2, 2.0 * h, C->raw<double>(P.o_ccoef), s);
    C->coarse.kind = 9;
    C->coarse.n1 = P.nc1;
    C->coarse.n2 = P.nc2;
    C->coarse.h2 = 0;
    C->coarse.xA = C->at<double>(P.o_cxA);
    C->coarse.xB = C->at<double>(P.o_cxB);
    C->coarse.yA = C->at<double>(P.o_cyA);
    C->coarse.yB = C->at<double>(P.o_cyB);
    C->coarse.k2 = C->raw<double>(P.o_ck2c);
    C->coarse.coef = C->raw<double>(P.o_ccoef);
    C->coarse.xmap = nullptr;
    C->dd = C->coarse;
    // transfer maps
    auto rmaps = [](const std::vector<int>& ifp, const std::vector<char>& ref, int nc, std::vector<int>& ri,
                    std::vector<double>& rw) {
      ri.assign(3 * nc, -1);
      rw.assign(3 * nc, 0.0);
      for (int I = 1; I <= nc; ++I) {
        const int F = ifp[I];
        int q = 0;
        ri[3 * (I - 1) + q] = F - 1, rw[3 * (I - 1) + q] = 1.0, ++q;
        if (ref[I - 1]) ri[3 * (I - 1) + q] = F - 2, rw[3 * (I - 1) + q] = 0.5, ++q;
        if (ref[I]) ri[3 * (I - 1) + q] = F, rw[3 * (I - 1) + q] = 0.5, ++q;
      }
    };
    auto pmaps = [](const std::vector<int>& ifp, const std::vector<char>& ref, int nf_, std::vector<int>& pi,
                    std::vector<double>& pw) {
      pi.assign(2 * nf_, -1);
      pw.assign(2 * nf_, 0.0);
      const int Nc = (int)ifp.size() - 1;
      for (int I = 0; I <= Nc; ++I) {
        const int F = ifp[I];
        if (F >= 1 && F <= nf_ && I >= 1 && I <= Nc - 1) pi[2 * (F - 1)] = I - 1, pw[2 * (F - 1)] = 1.0;
        if (I < Nc && ref[I]) {
          const int f = F + 1;  // midpoint of the refined cell
          int q = 0;
          if (I >= 1) pi[2 * (f - 1) + q] = I - 1, pw[2 * (f - 1) + q] = 0.5, ++q;
          if (I + 1 <= Nc - 1) pi[2 * (f - 1) + q] = I, pw[2 * (f - 1) + q] = 0.5, ++q;
        }
      }
    };
    std::vector<int> ri;
    std::vector<double> rw;
    rmaps(P.ifp1, P.ref1, P.nc1, ri, rw);
    up(P.o_rx, ri.data(), ri.size() * sizeof(int));
    up(P.o_rwx, rw.data(), rw.size() * sizeof(double));
    rmaps(P.ifp2, P.ref2, P.nc2, ri, rw);
    up(P.o_ry, ri.data(), ri.size() * sizeof(int));
    up(P.o_rwy, rw.data(), rw.size() * sizeof(double));
    pmaps(P.ifp1, P.ref1, P.nf1, ri, rw);
    up(P.o_px, ri.data(), ri.size() * sizeof(int));
    up(P.o_pwx, rw.data(), rw.size() * sizeof(double));
    pmaps(P.ifp2, P.ref2, P.nf2, ri, rw);
    up(P.o_py, ri.data(), ri.size() * sizeof(int));
    up(P.o_pwy, rw.data(), rw.size() * sizeof(double));
    C->tr.nf1 = P.nf1;
    C->tr.nf2 = P.nf2;
    C->tr.nc1 = P.nc1;
    C->tr.nc2 = P.nc2;
    C->tr.rx = C->raw<int>(P.o_rx);
    C->tr.rwx = C->raw<double>(P.o_rwx);
    C->tr.ry = C->raw<int>(P.o_ry);
    C->tr.rwy = C->raw<double>(P.o_rwy);
    C->tr.px = C->raw<int>(P.o_px);
    C->tr.pwx = C->raw<double>(P.o_pwx);
    C->tr.py = C->raw<int>(P.o_py);
    C->tr.pwy = C->raw<double>(P.o_pwy);
  } else {
    dx = fx;
    dy = fy;
    C->dd = C->fine;
  }

  // slabs on the DD level
  {
    const auto& be = P.beta;
    const int kind = P.dd_kind;
    const double d = opt->w_dd * dx.h_nom;
    const double Cdd = S_dd * C->c_pml / (d * d * d);
    std::vector<cd> SA(P.n_slabA, mk<double>(0, 0)), SB(P.n_slabA, mk<double>(0, 0));
    std::vector<int> XM(P.n_xmap, 0);
    size_t oA = 0, oM = 0, oF = 0, oS = 0;
    C->slabs_host.resize(J);
    const int ncell = P.dd_n1 + 1;  // cells of the DD level along x
    for (int j = 1; j <= J; ++j) {
      const int x0 = P.x0[j - 1], x1 = P.x1[j - 1], nl = x1 - x0 + 1;
      // slab sigma: DD-PML beyond b_j and before b~_{j-1}, global sigma in between
      Sigma gs = dx.sig;
      const bool hasL = j > 1, hasR = j < J;
      const double bl = hasL ? 0.5 * (dx.x[be[j - 1] - 1] + dx.x[be[j - 1]]) : 0.0;
      const double br = hasR ? 0.5 * (dx.x[be[j]] + dx.x[be[j] + 1]) : 0.0;
      auto sig = [&](double x) {
        if (hasL && x < bl) return Cdd * (bl - x) * (bl - x);
        if (hasR && x > br) return Cdd * (x - br) * (x - br);
        return gs(x);
      };
      // local nodes: global nodes x0-1 .. x1+1
      auto gxn = [&](int lnode) { return dx.x[x0 - 1 + lnode]; };
      if (kind == 5) {
        for (int p = 0; p <= nl; ++p) SA[oA + p] = to_cd(alpha_of(sig(0.5 * (gxn(p) + gxn(p + 1))), omega));
        for (int i = 0; i <= nl + 1; ++i) SB[oA + i] = to_cd(1.0 / alpha_of(sig(gxn(i)), omega));
        const int lo = hasL ? be[j - 1] : 1, hi = hasR ? be[j] : P.dd_n1;
        for (int l = 0; l < nl; ++l) XM[oM + l] = std::min(std::max(x0 + l, lo), hi) - 1;
      } else {
        for (int p = 0; p <= nl; ++p) {
          const double hp = gxn(p + 1) - gxn(p);
          const cplx al = alpha_of(sig(0.5 * (gxn(p) + gxn(p + 1))), omega);
          SA[oA + p] = to_cd(al / hp);
          SB[oA + p] = to_cd(hp / al);
        }
        const int lo = hasL ? be[j - 1] - 1 : 0, hi = hasR ? be[j] : ncell - 1;
        for (int p = 0; p <= nl; ++p) XM[oM + p] = std::min(std::max(x0 - 1 + p, lo), hi);
      }
      SlabDev sd;
      sd.x0 = x0;
      sd.nl = nl;
      sd.op = C->dd;
      sd.op.n1 = nl;
      sd.op.xA = C->at<double>(P.o_slabA) + oA;
      sd.op.xB = C->at<double>(P.o_slabB) + oA;
      sd.op.xmap = C->raw<int>(P.o_xmap) + oM;
      sd.fac_off = oF;
      sd.scr_off = oS;
      C->slabs_host[j - 1] = sd;
      oA += nl + 2;
      oM += nl + 1;
      oF += slab_factor_elems(nl, P.dd_n2);
      oS += slab_setup_elems(nl, P.dd_n2);
    }
    up(P.o_slabA, SA.data(), SA.size() * sizeof(cd));
    up(P.o_slabB, SB.data(), SB.size() * sizeof(cd));
    up(P.o_xmap, XM.data(), XM.size() * sizeof(int));
    up(P.o_slabs, C->slabs_host.data(), J * sizeof(SlabDev));
    C->slabs_dev = C->raw<SlabDev>(P.o_slabs);
    C->factors = C->ws + P.o_fac;
  }
  build_schedule(C);
  if (C->tasks_host.size() > P.n_tasks) return cleanup(fail(HSP_EINVAL, "internal: schedule too long"));
  up(P.o_tasks, C->tasks_host.data(), C->tasks_host.size() * sizeof(TaskDev));
  C->tasks_dev = C->raw<TaskDev>(P.o_tasks);
  for (hipError_t e : errs)
    if (e != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string("upload: ") + hipGetErrorString(e)));

  // factorization of all slabs, then the chunk transfer matrices
  int* status = C->raw<int>(P.o_status);
  CHK(hipMemsetAsync(status, 0, sizeof(int), s));
  CHK(hipMemsetAsync(C->raw<int>(P.o_ctr), 0, 64 * sizeof(int), s));
  if (P.tsize == sizeof(cf))
    launch_factor<float>(C->slabs_dev, J, P.nl_max, P.dd_n2, P.chunk, P.nchunk, reinterpret_cast<cf*>(C->factors),
                         C->at<double>(P.o_setup), C->at<double>(P.o_facscr), C->at<double>(P.o_ttmp), status, s);
  else
    launch_factor<double>(C->slabs_dev, J, P.nl_max, P.dd_n2, P.chunk, P.nchunk, reinterpret_cast<cd*>(C->factors),
                          C->at<double>(P.o_setup), C->at<double>(P.o_facscr), C->at<double>(P.o_ttmp), status, s);
  CHK(hipGetLastError());
  int hstat = 0;
  CHK(hipMemcpyAsync(&hstat, status, sizeof(int), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  if (hstat != 0) return cleanup(fail(HSP_ESINGULAR, "zero or non-finite pivot in a slab factorization"));
#undef CHK
  *out = C;
  g_err = "no error";
  return HSP_OK;
}

hsp_status hsp_destroy(hsp_handle hd) {
  delete hd;
  return HSP_OK;
}

hsp_status hsp_get_info(hsp_handle C, hsp_info* info) {
  if (!C || !info) return fail(HSP_EINVAL, "null argument");
  info->n_fine[0] = C->P.nf1;
  info->n_fine[1] = C->P.nf2;
  info->n_coarse[0] = C->P.two_grid ? C->P.nc1 : 0;
  info->n_coarse[1] = C->P.two_grid ? C->P.nc2 : 0;
  info->J = C->J;
  info->max_slab_layers = C->P.nl_max;
  info->precision = C->opt.precision;
  info->two_grid = C->P.two_grid;
  return HSP_OK;
}

hsp_status hsp_get_partition(hsp_handle C, int* beta, int* x0, int* x1) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  for (int j = 0; j <= C->J; ++j)
    if (beta) beta[j] = C->P.beta[j];
  for (int j = 0; j < C->J; ++j) {
    if (x0) x0[j] = C->P.x0[j];
    if (x1) x1[j] = C->P.x1[j];
  }
  return HSP_OK;
}

hsp_status hsp_rhs(hsp_handle C, const void* f, void* b, void* stream) {
  if (!C || !f || !b) return fail(HSP_EINVAL, "null argument");
  launch_scale_rhs_arrays(C->P.nf1, C->P.nf2, C->h * C->h, C->at<double>(C->P.o_ixn), C->at<double>(C->P.o_iyn),
                          (const cd*)f, (cd*)b, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_apply_operator(hsp_handle C, const void* x, void* y, void* stream) {
  if (!C || !x || !y || x == y) return fail(HSP_EINVAL, "null or aliased argument");
  launch_stencil<double, double, double, double>(C->fine, 0, (const cd*)x, (const cd*)nullptr, (cd*)y, 0.0,
                                                 S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_apply_level_operator(hsp_handle C, int level, const void* x, void* y, void* stream) {
  if (!C || !x || !y || x == y) return fail(HSP_EINVAL, "null or aliased argument");
  if (level != 0 && !(level == 1 && C->P.two_grid)) return fail(HSP_EINVAL, "no such level");
  const LevelDev& L = level == 0 ? C->fine : C->coarse;
  hipStream_t s = S_(stream);
  if (level == 0 || C->opt.precision == HSP_FP64) {
    launch_stencil<double, double, double, double>(L, 0, (const cd*)x, (const cd*)nullptr, (cd*)y, 0.0, s);
  } else {
    const size_t n = (size_t)L.n1 * L.n2;
    cf* xin = C->at<float>(C->P.o_cvin);
    cf* yo = C->at<float>(C->P.o_cvout);
    launch_convert<float, double>((const cd*)x, xin, n, 0, s);
    launch_stencil<float, float, float, float>(L, 0, xin, (const cf*)nullptr, yo, 0.0, s);
    launch_convert<double, float>(yo, (cd*)y, n, 0, s);
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_restrict(hsp_handle C, const void* rf, void* rc, void* stream) {
  if (!C || !rf || !rc) return fail(HSP_EINVAL, "null argument");
  if (!C->P.two_grid) return fail(HSP_EINVAL, "no coarse level");
  launch_restrict<double, double>(C->tr, (const cd*)rf, (cd*)rc, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_prolong_add(hsp_handle C, const void* ec, void* xf, void* stream) {
  if (!C || !ec || !xf) return fail(HSP_EINVAL, "null argument");
  if (!C->P.two_grid) return fail(HSP_EINVAL, "no coarse level");
  launch_prolong_add<double, double>(C->tr, (const cd*)ec, (cd*)xf, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_smooth(hsp_handle C, const void* r, void* x, int steps, void* stream) {
  if (!C || !r || !x || r == x || steps < 1) return fail(HSP_EINVAL, "bad argument");
  hipStream_t s = S_(stream);
  const double wj = C->opt.omega_jac;
  cd* tmp = C->at<double>(C->P.o_cvin);
  // out-of-place steps, ending in x
  cd* bufs[2] = {(cd*)x, tmp};
  int cur = (steps % 2 == 1) ? 0 : 1;
  launch_stencil<double, double, double, double>(C->fine, 2, (const cd*)nullptr, (const cd*)r, bufs[cur], wj, s);
  for (int k = 1; k < steps; ++k) {
    launch_stencil<double, double, double, double>(C->fine, 2, bufs[cur], (const cd*)r, bufs[1 - cur], wj, s);
    cur = 1 - cur;
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_sweep(hsp_handle C, const void* f, void* u, void* stream) {
  if (!C || !f || !u || f == u) return fail(HSP_EINVAL, "null or aliased argument");
  hipStream_t s = S_(stream);
  const size_t nd = (size_t)C->P.dd_n1 * C->P.dd_n2;
  if (C->opt.precision == HSP_FP64) {
    cd* fin = C->at<double>(C->P.o_swf);
    launch_convert<double, double>((const cd*)f, fin, nd, 0, s);
    run_sweep<double>(C, fin, (cd*)u, s);
  } else {
    cf* fin = C->at<float>(C->P.o_swf);
    cf* uo = C->at<float>(C->P.o_cvout);
    launch_convert<float, double>((const cd*)f, fin, nd, 0, s);
    run_sweep<float>(C, fin, uo, s);
    launch_convert<double, float>(uo, (cd*)u, nd, 0, s);
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_slab_solve(hsp_handle C, int j, const void* b, void* x, void* stream) {
  if (!C || !b || !x || b == x) return fail(HSP_EINVAL, "null or aliased argument");
  if (j < 0 || j >= C->J) return fail(HSP_EINVAL, "slab index out of range");
  hipStream_t s = S_(stream);
  const Plan& P = C->P;
  const int nl = P.x1[j] - P.x0[j] + 1;
  const size_t n = (size_t)nl * P.dd_n2;
  // one task in slab layout, placed in the last task slot
  TaskDev t;
  std::memset(&t, 0, sizeof(t));
  t.slab = j;
  t.mode = 1;
  TaskDev* td = C->tasks_dev + (P.n_tasks - 1);
  HIPCHK(hipMemcpyAsync(td, &t, sizeof(t), hipMemcpyHostToDevice, s));
  if (C->opt.precision == HSP_FP64) {
    cd* fin = C->at<double>(P.o_swf);
    cd* uo = C->at<double>(P.o_swu);
    launch_convert<double, double>((const cd*)b, fin, n, 0, s);
    launch_stage<double>(td, 1, C->slabs_dev, C->dd, fin, fin, uo, C->at<double>(P.o_swB), C->at<double>(P.o_swscr),
                         reinterpret_cast<const cd*>(C->factors), P.nl_max, nl, P.chunk, P.nchunk,
                         C->at<double>(P.o_red), C->raw<int>(P.o_ctr), s);
    launch_convert<double, double>(uo, (cd*)x, n, 0, s);
  } else {
    cf* fin = C->at<float>(P.o_swf);
    cf* uo = C->at<float>(P.o_swu);
    launch_convert<float, double>((const cd*)b, fin, n, 0, s);
    launch_stage<float>(td, 1, C->slabs_dev, C->dd, fin, fin, uo, C->at<float>(P.o_swB), C->at<float>(P.o_swscr),
                        reinterpret_cast<const cf*>(C->factors), P.nl_max, nl, P.chunk, P.nchunk,
                        C->at<float>(P.o_red), C->raw<int>(P.o_ctr), s);
    launch_convert<double, float>(uo, (cd*)x, n, 0, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));  // the task descriptor is host stack memory
  return HSP_OK;
}

hsp_status hsp_gradient_accumulate(hsp_handle C, const void* u, const void* lam, double* g, void* stream) {
  if (!C || !u || !lam || !g) return fail(HSP_EINVAL, "null argument");
  if (C->opt.fine_stencil != 5) return fail(HSP_EINVAL, "the gradient is implemented for the 5-point fine operator");
  if (!(C->grid.c_pml > 0)) return fail(HSP_EINVAL, "the gradient needs an explicit c_pml (not mean(c))");
  launch_grad_m(C->P.nf1, C->P.nf2, C->h * C->h * C->omega * C->omega, C->at<double>(C->P.o_ixn),
                C->at<double>(C->P.o_iyn), (const cd*)u, (const cd*)lam, g, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_profile_enable(hsp_handle C, int on) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  C->prof.on = on != 0;
  return HSP_OK;
}

hsp_status hsp_profile_read(hsp_handle C, int cls, double* total_ms, long long* launches, double* alg_bytes) {
  if (!C || cls < 0 || cls >= HSP_PROF_NCLASS) return fail(HSP_EINVAL, "bad handle or class");
  Prof& P = C->prof;
  double ms = 0;
  if (P.used[cls] > 0) {
    HIPCHK(hipEventSynchronize(P.ev[cls][P.used[cls] - 1].second));
    for (size_t i = 0; i < P.used[cls]; ++i) {
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, P.ev[cls][i].first, P.ev[cls][i].second));
      ms += e;
    }
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = P.n[cls];
  if (alg_bytes) *alg_bytes = P.bytes[cls];
  P.used[cls] = 0;
  P.n[cls] = 0;
  P.bytes[cls] = 0;
  return HSP_OK;
}

hsp_status hsp_apply_precond(hsp_handle C, const void* r, void* z, void* stream) {
  if (!C || !r || !z || r == z) return fail(HSP_EINVAL, "null or aliased argument");
  precond(C, (const cd*)r, (cd*)z, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_solve(hsp_handle C, const void* b_in, void* u_out, double tol, int maxit, int conj_transpose,
                     int* iters, double* relres, void* stream) {
  if (!C || !b_in || !u_out || b_in == u_out) return fail(HSP_EINVAL, "null or aliased argument");
  if (!(tol > 0) || maxit < 1) return fail(HSP_EINVAL, "tol must be > 0 and maxit >= 1");
  hipStream_t s = S_(stream);
  const Plan& P = C->P;
  const size_t n = (size_t)P.nf1 * P.nf2;
  const int m = P.m;
  cd* V = C->at<double>(P.o_V);
  cd* Z = C->at<double>(P.o_Z);
  cd* w = C->at<double>(P.o_w);
  cd* part = C->at<double>(P.o_part);
  cd* hb = C->at<double>(P.o_hbuf);  // [h1 (m+1) | h2 (m+1) | nrm2 | spare]
  cd* x = (cd*)u_out;
  const cd* b = (const cd*)b_in;
  if (conj_transpose) {
    cd* bc = C->at<double>(P.o_bconj);
    launch_convert<double, double>(b, bc, n, 1, s);
    b = bc;
  }
  const LevelDev& A = C->fine;
  // conj(vecs_j) . vv for j < cnt into out[j] (w read once per tile of basis vectors)
  auto dotn = [&](const cd* vecs, int cnt, const cd* vv, cd* out) {
    launch_bmultidot(vecs, n, BIdx{}, cnt, vv, BIdx{}, n, part, kPartBlocks, out, 1, 1, s);
  };
  // ||b||
  dotn(b, 1, b, hb + 2 * (m + 1));
  cd hn;
  HIPCHK(hipMemcpyAsync(&hn, hb + 2 * (m + 1), sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(hn.re);
  launch_zero<double>(x, n, s);
  if (bnorm == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0;
    return HSP_OK;
  }
  std::vector<cplx> H((size_t)(m + 1) * m), g(m + 1), sn(m);
  std::vector<double> cs(m);
  std::vector<cd> hh(2 * (m + 1) + 1);
  int it = 0;
  bool done = false;
  while (it < maxit && !done) {
    // r = b - A x into V_0
    launch_stencil<double, double, double, double>(A, 1, x, b, V, 0.0, s);
    dotn(V, 1, V, hb + 2 * (m + 1));
    HIPCHK(hipMemcpyAsync(&hn, hb + 2 * (m + 1), sizeof(cd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double beta = std::sqrt(hn.re);
    if (beta <= tol * bnorm) break;
    launch_normalize(V, hb + 2 * (m + 1), V, n, s);
    std::fill(H.begin(), H.end(), cplx(0));
    std::fill(g.begin(), g.end(), cplx(0));
    g[0] = beta;
    int k_used = 0;
    for (int k = 0; k < m && it < maxit; ++k) {
      cd* vk = V + (size_t)k * n;
      cd* zk = Z + (size_t)k * n;
      precond(C, vk, zk, s);
      prof_begin(C, HSP_PROF_KRYLOV, s);
      launch_stencil<double, double, double, double>(A, 0, zk, (const cd*)nullptr, w, 0.0, s);
      // classical Gram-Schmidt, twice
      dotn(V, k + 1, w, hb);
      launch_multiaxpy(V, n, k + 1, hb, w, n, 1, s);
      dotn(V, k + 1, w, hb + (m + 1));
      launch_multiaxpy(V, n, k + 1, hb + (m + 1), w, n, 1, s);
      dotn(w, 1, w, hb + 2 * (m + 1));
      launch_normalize(w, hb + 2 * (m + 1), V + (size_t)(k + 1) * n, n, s);
      // matvec (z, k^2 read, w written) + two Gram-Schmidt passes over k+1
      // basis vectors + norm + normalisation, complex128 vectors
      prof_end(C, HSP_PROF_KRYLOV, s, (double)n * (2.0 * sizeof(cd) + sizeof(double)) +
                                          (double)n * sizeof(cd) * (4.0 * k + 13.0));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hh.data(), hb, hh.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i <= k; ++i)
        H[(size_t)i * m + k] = cplx(hh[i].re + hh[m + 1 + i].re, hh[i].im + hh[m + 1 + i].im);
      H[(size_t)(k + 1) * m + k] = std::sqrt(std::max(hh[2 * (m + 1)].re, 0.0));
      // apply previous rotations, then a new one
      for (int i = 0; i < k; ++i) {
        const cplx a = H[(size_t)i * m + k], bb = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * bb;
        H[(size_t)(i + 1) * m + k] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      const cplx a = H[(size_t)k * m + k], bb = H[(size_t)(k + 1) * m + k];
      if (std::abs(bb) == 0) {
        cs[k] = 1;
        sn[k] = 0;
      } else if (std::abs(a) == 0) {
        cs[k] = 0;
        sn[k] = 1;
      } else {
        const double t = std::sqrt(std::norm(a) + std::norm(bb));
        cs[k] = std::abs(a) / t;
        sn[k] = (a / std::abs(a)) * std::conj(bb) / t;
      }
      H[(size_t)k * m + k] = cs[k] * a + sn[k] * bb;
      H[(size_t)(k + 1) * m + k] = 0;
      g[k + 1] = -std::conj(sn[k]) * g[k];
      g[k] = cs[k] * g[k];
      ++it;
      k_used = k + 1;
      if (std::abs(g[k + 1]) <= tol * bnorm) {
        done = true;
        break;
      }
    }
    // y = H^{-1} g, x += Z y
    std::vector<cplx> y(k_used);
    for (int i = k_used - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int j2 = i + 1; j2 < k_used; ++j2) acc -= H[(size_t)i * m + j2] * y[j2];
      y[i] = acc / H[(size_t)i * m + i];
    }
    std::vector<cd> yd(k_used);
    for (int i = 0; i < k_used; ++i) yd[i] = to_cd(y[i]);
    HIPCHK(hipMemcpyAsync(hb, yd.data(), k_used * sizeof(cd), hipMemcpyHostToDevice, s));
    launch_multiaxpy(Z, n, k_used, hb, x, n, 0, s);
    HIPCHK(hipStreamSynchronize(s));
  }
  // true residual
  launch_stencil<double, double, double, double>(A, 1, x, b, w, 0.0, s);
  dotn(w, 1, w, hb + 2 * (m + 1));
  HIPCHK(hipMemcpyAsync(&hn, hb + 2 * (m + 1), sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double rr = std::sqrt(std::max(hn.re, 0.0)) / bnorm;
  if (conj_transpose) launch_convert<double, double>(x, x, n, 1, s);
  HIPCHK(hipGetLastError());
  if (iters) *iters = it;
  if (relres) *relres = rr;
  if (!done && rr > tol) return fail(HSP_ENOCONV, "maxit reached before the tolerance");
  return HSP_OK;
}

}  // extern "C"

// ===========================================================================
// Batched right-hand sides (many sources or receivers of one medium and
// frequency share the setup; Sec. 4 notes that the slab factors serve every
// right-hand side)
// ===========================================================================
namespace {

// Hessenberg matrix of one right-hand side's flexible Arnoldi process.  With
// the delayed Gram-Schmidt the newest column is provisional (its
// reorthogonalisation terms arrive with the next step); the least-squares
// problem min ||beta e_1 - H y|| is solved from scratch by Givens rotations
// whenever it is needed (k <= restart, negligible host work).
struct Arnoldi {
  int m = 0;
  double beta = 0;
  std::vector<cplx> H;  // (m+1) x m, H[i m + j]
  void reset(int m_, double b) {
    m = m_;
    beta = b;
    H.assign((size_t)(m + 1) * m, cplx(0));
  }
  cplx& at(int i, int j) { return H[(size_t)i * m + j]; }
  // residual estimate over columns 0..k-1; y (optional) receives the
  // minimiser
  double lsq(int k, cd* y) const {
    std::vector<cplx> R((size_t)(k + 1) * k), g(k + 1, cplx(0)), sn(k);
    std::vector<double> cs(k);
    for (int i = 0; i <= k; ++i)
      for (int j = 0; j < k; ++j) R[(size_t)i * k + j] = H[(size_t)i * m + j];
    g[0] = beta;
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i < j; ++i) {
        const cplx a = R[(size_t)i * k + j], bb = R[(size_t)(i + 1) * k + j];
        R[(size_t)i * k + j] = cs[i] * a + sn[i] * bb;
        R[(size_t)(i + 1) * k + j] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      const cplx a = R[(size_t)j * k + j], bb = R[(size_t)(j + 1) * k + j];
      if (std::abs(bb) == 0) {
        cs[j] = 1;
        sn[j] = 0;
      } else if (std::abs(a) == 0) {
        cs[j] = 0;
        sn[j] = 1;
      } else {
        const double t = std::sqrt(std::norm(a) + std::norm(bb));
        cs[j] = std::abs(a) / t;
        sn[j] = (a / std::abs(a)) * std::conj(bb) / t;
      }
      R[(size_t)j * k + j] = cs[j] * a + sn[j] * bb;
      R[(size_t)(j + 1) * k + j] = 0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
    }
    if (y) {
      std::vector<cplx> yy(k);
      for (int i = k - 1; i >= 0; --i) {
        cplx acc = g[i];
        for (int j = i + 1; j < k; ++j) acc -= R[(size_t)i * k + j] * yy[j];
        yy[i] = acc / R[(size_t)i * k + i];
      }
      for (int i = 0; i < k; ++i) y[i] = to_cd(yy[i]);
    }
    return std::abs(g[k]);
  }
};

}  // namespace

extern "C" {

hsp_status hsp_batch_workspace_size(hsp_handle C, int nrhs, int restart, size_t* bytes) {
  if (!C || !bytes) return fail(HSP_EINVAL, "null argument");
  if (nrhs < 1 || restart < 1) return fail(HSP_EINVAL, "nrhs and restart must be >= 1");
  *bytes = batch_layout(C->P, nrhs, restart).total;
  return HSP_OK;
}

hsp_status hsp_apply_precond_batch(hsp_handle C, int nrhs, const void* r, void* z, int tile, void* ws,
                                   size_t ws_bytes, void* stream) {
  BatchLayout B;
  hsp_status st = check_batch_args(C, nrhs, 1, ws, ws_bytes, tile, B);
  if (st != HSP_OK || nrhs == 0) return st;
  if (!r || !z || r == z) return fail(HSP_EINVAL, "null or aliased argument");
  hipStream_t s = S_(stream);
  const size_t nf = (size_t)C->P.nf1 * C->P.nf2;
  HIPCHK(hipMemsetAsync(bat<int>(ws, B.o_ctr), 0, 2 * batch_slots(nrhs) * sizeof(int), s));
  BIdx bv;
  bv.ld = nf;
  precond_batch(C, B, ws, nrhs, tile ? tile : default_tile(C, nrhs), (const cd*)r, bv, (cd*)z, bv, s);
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_tune_batch(hsp_handle C, int nrhs, int restart, void* ws, size_t ws_bytes, int* tile_out,
                          double* ms_out, void* stream) {
  BatchLayout B;
  hsp_status st = check_batch_args(C, nrhs, restart, ws, ws_bytes, 0, B);
  if (st != HSP_OK) return st;
  if (nrhs == 0) return fail(HSP_EINVAL, "nrhs must be >= 1");
  hipStream_t s = S_(stream);
  const size_t nf = (size_t)C->P.nf1 * C->P.nf2;
  cd* r = bat<cd>(ws, B.o_V);
  cd* z = bat<cd>(ws, B.o_Z);
  HIPCHK(hipMemsetAsync(bat<int>(ws, B.o_ctr), 0, 2 * batch_slots(nrhs) * sizeof(int), s));
  launch_fill(r, (size_t)nrhs * nf, mk<double>(1.0, 0.0), s);
  BIdx bv;
  bv.ld = nf;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HSP_EDEVICE, "hipEventCreate failed");
  }
  const bool prof = C->prof.on;
  C->prof.on = false;
  int best = 1;
  double best_ms = 1e300;
  hipError_t err = hipSuccess;
  for (int rb = 1; rb <= kMaxTile && err == hipSuccess; rb *= 2) {
    precond_batch(C, B, ws, nrhs, rb, r, bv, z, bv, s);  // warm-up
    err = hipEventRecord(e0, s);
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) precond_batch(C, B, ws, nrhs, rb, r, bv, z, bv, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && 0.5 * ms < best_ms) {
      best_ms = 0.5 * ms;
      best = rb;
    }
  }
  C->prof.on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(HSP_EDEVICE, std::string("tuning: ") + hipGetErrorString(err));
  HIPCHK(hipGetLastError());
  C->tuned_rb = best;
  C->tuned_nact = nrhs;
  if (tile_out) *tile_out = best;
  if (ms_out) *ms_out = best_ms;
  return HSP_OK;
}

hsp_status hsp_solve_batch(hsp_handle C, int nrhs, const void* b_in, void* u_out, double tol, int maxit, int restart,
                           int conj_transpose, int tile, void* ws, size_t ws_bytes, int* iters, double* relres,
                           void* stream) {
  BatchLayout B;
  hsp_status st = check_batch_args(C, nrhs, restart, ws, ws_bytes, tile, B);
  if (st != HSP_OK || nrhs == 0) return st;
  if (!b_in || !u_out || b_in == u_out) return fail(HSP_EINVAL, "null or aliased argument");
  if (!(tol > 0) || maxit < 1) return fail(HSP_EINVAL, "tol must be > 0 and maxit >= 1");
  hipStream_t s = S_(stream);
  const int R = nrhs, m = restart;
  const size_t nf = (size_t)C->P.nf1 * C->P.nf2;
  const size_t hs = B.hs;
  cd* V = bat<cd>(ws, B.o_V);
  cd* Z = bat<cd>(ws, B.o_Z);
  cd* w = bat<cd>(ws, B.o_w);
  cd* part = bat<cd>(ws, B.o_part);
  cd* hb = bat<cd>(ws, B.o_hb);
  cd* ydev = bat<cd>(ws, B.o_y);
  int* act_d = bat<int>(ws, B.o_act);
  int* upd_d = bat<int>(ws, B.o_upd);
  cd* x = (cd*)u_out;
  const cd* b = (const cd*)b_in;
  const LevelDev& A = C->fine;
  HIPCHK(hipMemsetAsync(bat<int>(ws, B.o_ctr), 0, 2 * batch_slots(R) * sizeof(int), s));
  BIdx bid;  // identity map over all right-hand sides
  bid.ld = nf;
  if (conj_transpose) {
    cd* bc = bat<cd>(ws, B.o_bc);
    launch_convert<double, double>(b, bc, (size_t)R * nf, 1, s);
    b = bc;
  }
  std::vector<cd> hh((size_t)R * hs);
  auto read_hb = [&](int cnt) -> hsp_status {
    HIPCHK(hipMemcpyAsync(hh.data(), hb, (size_t)cnt * hs * sizeof(cd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HSP_OK;
  };
  // ||b_z||
  launch_bmultidot(b, 0, bid, 1, b, bid, nf, part, B.nblk, hb + 2 * (m + 1), hs, R, s);
  st = read_hb(R);
  if (st != HSP_OK) return st;
  std::vector<double> bnorm(R);
  for (int z = 0; z < R; ++z) bnorm[z] = std::sqrt(std::max(hh[(size_t)z * hs + 2 * (m + 1)].re, 0.0));
  launch_zero<double>(x, (size_t)R * nf, s);
  std::vector<int> its(R, 0), done(R, 0), act, upd;
  for (int z = 0; z < R; ++z) {
    if (bnorm[z] == 0)
      done[z] = 1;
    else
      act.push_back(z);
  }
  std::vector<Arnoldi> ar(R);
  std::vector<cd> yh((size_t)R * m);
  auto upload = [&](int* dst, const std::vector<int>& v) -> hsp_status {
    if (!v.empty()) HIPCHK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s));
    return HSP_OK;
  };
  // x_z += Z_z y_z for the right-hand sides in `upd` (k basis vectors each)
  auto update = [&](const std::vector<int>& list, int k) -> hsp_status {
    if (list.empty() || k == 0) return HSP_OK;
    // the host staging arrays yh / upd may still feed an earlier copy
    HIPCHK(hipStreamSynchronize(s));
    upd = list;
    for (size_t i = 0; i < upd.size(); ++i) ar[upd[i]].lsq(k, yh.data() + i * m);
    HIPCHK(hipMemcpyAsync(ydev, yh.data(), upd.size() * m * sizeof(cd), hipMemcpyHostToDevice, s));
    hsp_status e = upload(upd_d, upd);
    if (e != HSP_OK) return e;
    BIdx bz, bx;
    bz.ld = (size_t)m * nf;
    bz.map = upd_d;
    bx.ld = nf;
    bx.map = upd_d;
    launch_bmultiaxpy(Z, nf, bz, k, ydev, m, x, bx, nf, 0, (int)upd.size(), s);
    return HSP_OK;
  };
  const int rb_fixed = tile;
  const int koff = 2 * (m + 1);  // hb offset of nu, h_kk, ||u_{k+1}||^2
  int it = 0;
  while (it < maxit && !act.empty()) {
    int nact = (int)act.size();
    st = upload(act_d, act);
    if (st != HSP_OK) return st;
    BIdx bx, bV;
    bx.ld = nf;
    bx.map = act_d;
    bV.ld = (size_t)(m + 1) * nf;
    bV.map = act_d;
    // r = b - A x into V_z0, its norm, normalisation
    launch_stencil<double, double, double, double>(A, 1, x, b, V, 0.0, s, nact, bx, bx, bV);
    launch_bmultidot(V, 0, bV, 1, V, bV, nf, part, B.nblk, hb + 2 * (m + 1), hs, nact, s);
    launch_bnormalize(V, bV, hb + 2 * (m + 1), hs, V, bV, nf, nact, s);
    st = read_hb(nact);
    if (st != HSP_OK) return st;
    {
      std::vector<int> keep;
      for (int zi = 0; zi < nact; ++zi) {
        const int z = act[zi];
        const double beta = std::sqrt(std::max(hh[(size_t)zi * hs + 2 * (m + 1)].re, 0.0));
        if (beta <= tol * bnorm[z]) {
          done[z] = 1;
          continue;
        }
        ar[z].reset(m, beta);
        keep.push_back(z);
      }
      act.swap(keep);
    }
    nact = (int)act.size();
    if (nact == 0) break;
    st = upload(act_d, act);
    if (st != HSP_OK) return st;
    int k = 0;
    for (; k < m && it < maxit && nact > 0; ++k) {
      const int rb = rb_fixed ? rb_fixed : default_tile(C, nact);
      BIdx bVk, bZk, bw;
      bVk.ld = (size_t)(m + 1) * nf;
      bVk.map = act_d;
      bZk.ld = (size_t)m * nf;
      bZk.map = act_d;
      bw.ld = nf;
      precond_batch(C, B, ws, nact, rb, V + (size_t)k * nf, bVk, Z + (size_t)k * nf, bZk, s);
      prof_begin(C, HSP_PROF_KRYLOV, s);
      launch_stencil<double, double, double, double>(A, 0, Z + (size_t)k * nf, (const cd*)nullptr, w, 0.0, s, nact,
                                                     bZk, BIdx{}, bw);
      // delayed classical Gram-Schmidt: one projection pass (basis against
      // u_k and w) and one update pass (v_k final, u_{k+1} and its norm)
      BIdx bVb;
      bVb.ld = (size_t)(m + 1) * nf;
      bVb.map = act_d;
      launch_bdcgs_project(V, nf, bVb, k, w, bw, nf, part, B.nblk, hb, hs, koff, nact, s);
      launch_bdcgs_update(V, nf, bVb, k, hb, hs, koff, w, bw, nf, part, B.nblk, hb + koff + 2, nact, s);
      // matvec (z, k^2 read, w written); projection reads k+1 basis vectors
      // and w; update reads k basis vectors, u_k and w and writes v_k, u_{k+1}
      prof_end(C, HSP_PROF_KRYLOV, s,
               (double)nact * ((double)nf * (2.0 * sizeof(cd) + sizeof(double)) +
                               (double)nf * sizeof(cd) * (2.0 * k + 6.0)));
      HIPCHK(hipGetLastError());
      st = read_hb(nact);
      if (st != HSP_OK) return st;
      ++it;
      std::vector<int> keep, conv;
      for (int zi = 0; zi < nact; ++zi) {
        const int z = act[zi];
        const cd* d = hh.data() + (size_t)zi * hs;
        Arnoldi& a = ar[z];
        if (k > 0) {  // finalise column k-1 with the reorthogonalisation terms
          for (int j = 0; j < k; ++j) a.at(j, k - 1) += cplx(d[j].re, d[j].im);
          a.at(k, k - 1) = d[koff].re;
        }
        for (int j = 0; j < k; ++j) a.at(j, k) = cplx(d[k + 1 + j].re, d[k + 1 + j].im);
        a.at(k, k) = cplx(d[koff + 1].re, d[koff + 1].im);
        a.at(k + 1, k) = std::sqrt(std::max(d[koff + 2].re, 0.0));
        const double est = a.lsq(k + 1, nullptr);
        its[z] = it;
        if (est <= tol * bnorm[z]) {
          conv.push_back(z);
          done[z] = 1;
        } else {
          keep.push_back(z);
        }
      }
      st = update(conv, k + 1);
      if (st != HSP_OK) return st;
      if (keep.size() != act.size()) {
        act.swap(keep);
        nact = (int)act.size();
        st = upload(act_d, act);
        if (st != HSP_OK) return st;
      }
    }
    // end of a restart cycle (or maxit): fold the active corrections into x
    st = update(act, k);
    if (st != HSP_OK) return st;
    HIPCHK(hipStreamSynchronize(s));
  }
  // true residuals of every right-hand side
  launch_stencil<double, double, double, double>(A, 1, x, b, w, 0.0, s, R, bid, bid, bid);
  launch_bmultidot(w, 0, bid, 1, w, bid, nf, part, B.nblk, hb + 2 * (m + 1), hs, R, s);
  st = read_hb(R);
  if (st != HSP_OK) return st;
  if (conj_transpose) launch_convert<double, double>(x, x, (size_t)R * nf, 1, s);
  HIPCHK(hipGetLastError());
  bool all = true;
  for (int z = 0; z < R; ++z) {
    const double rr = bnorm[z] > 0 ? std::sqrt(std::max(hh[(size_t)z * hs + 2 * (m + 1)].re, 0.0)) / bnorm[z] : 0.0;
    if (iters) iters[z] = its[z];
    if (relres) relres[z] = rr;
    if (!done[z] && rr > tol) all = false;
  }
  if (!all) return fail(HSP_ENOCONV, "maxit reached before the tolerance for some right-hand sides");
  return HSP_OK;
}

}  // extern "C"
