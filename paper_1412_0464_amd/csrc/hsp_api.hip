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
#include <type_traits>
#include <vector>

#include "ctx.h"

using namespace hsp;

namespace {

thread_local std::string g_err = "no error";

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
  if (o->sweep != HSP_SWEEP_X && o->sweep != HSP_SWEEP_UD && o->sweep != HSP_SWEEP_NX)
    return fail(HSP_EINVAL, "bad sweep");
  if (o->precision != HSP_FP64 && o->precision != HSP_MIXED) return fail(HSP_EINVAL, "bad precision");
  if (!std::isfinite(o->omega_jac)) return fail(HSP_EINVAL, "bad omega_jac");
  if (g->sponge != 0 && g->sponge != 1) return fail(HSP_EINVAL, "sponge must be 0 or 1");
  if (g->sponge && o->fine_stencil != 5) return fail(HSP_EINVAL, "sponge layers need fine_stencil 5");
  if (o->chunk < 0 || o->chunk > kMaxChunk) return fail(HSP_EINVAL, "chunk must be in 0..64");
  if (o->krylov_fp32 != 0 && o->krylov_fp32 != 1) return fail(HSP_EINVAL, "krylov_fp32 must be 0 or 1");
  if (o->krylov_fp32 && o->precision != HSP_MIXED)
    return fail(HSP_EINVAL, "krylov_fp32 requires precision HSP_MIXED");
  if (o->slab_factor != HSP_SLAB_AUTO && o->slab_factor != HSP_SLAB_BLOCK)
    return fail(HSP_EINVAL, "2-D slabs are block tridiagonal: slab_factor must be HSP_SLAB_AUTO or HSP_SLAB_BLOCK");
  return HSP_OK;
}

}  // namespace

namespace hsp {

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

hsp_status nx_cells(int J, int N, std::vector<int>& jc, std::vector<int>& jm) {
  if (N < 1 || N > 16) return fail(HSP_EINVAL, "ncell must be in 1..16");
  if (2 * N - 1 > J) return fail(HSP_EINVAL, "the NX-sweep needs J >= 2 ncell - 1 slabs");
  jc.assign(N + 1, 0);
  jm.assign(N + 1, 0);
  jc[N] = J + 1;
  for (int m = 1; m < N; ++m) jc[m] = (m * (J + 1) + N / 2) / N;
  for (int m = 1; m <= N; ++m) {
    if (jc[m] - jc[m - 1] < 2) return fail(HSP_EINVAL, "a group of the NX-sweep holds no slab");
    jm[m] = (jc[m - 1] + jc[m] + 1) / 2;
  }
  return HSP_OK;
}

hsp_status sweep_shape(int J, const hsp_options* o, int* nbuf, int* maxtask) {
  *nbuf = 2;
  *maxtask = 2;
  if (o->sweep != HSP_SWEEP_NX) return HSP_OK;
  std::vector<int> jc, jm;
  hsp_status st = nx_cells(J, o->ncell, jc, jm);
  if (st != HSP_OK) return st;
  *nbuf = std::max(2, 2 * o->ncell);
  *maxtask = std::max(2, 2 * o->ncell);
  return HSP_OK;
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

}  // namespace hsp

namespace hsp {

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
  P.sponge = g->sponge;
  if (P.two_grid) {
    // cells that are not coarsened: the PML cells, none with sponge layers
    const int cw[2] = {P.sponge ? 0 : g->pml[0], P.sponge ? 0 : g->pml[1]};
    for (int a = 0; a < 2; ++a) {
      const int N = a == 0 ? P.Nf1 : P.Nf2;
      if ((N - 2 * cw[a]) % 2 != 0 || N - 2 * cw[a] < 2)
        return fail(HSP_EINVAL, P.sponge ? "two-grid with sponge layers needs an even cell count per axis"
                                         : "two-grid needs an even, positive interior cell count per axis");
    }
    coarse_map(P.Nf1, cw[0], P.ifp1, P.ref1);
    coarse_map(P.Nf2, cw[1], P.ifp2, P.ref2);
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
  w_dd_outer = P.sponge ? 0 : g->pml[0];  // sponge layers are ordinary layers of the partition
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
    // about sqrt(n2): balances the chunk-local chains (m steps) against the
    // chains over the chunk ends (P - 1 steps)
    P.chunk = (int)std::ceil(std::sqrt((double)P.dd_n2));
    P.chunk = std::max(8, std::min(kMaxChunk, P.chunk));
  }
  P.chunk = std::min(P.chunk, P.dd_n2);
  P.nchunk = (P.dd_n2 + P.chunk - 1) / P.chunk;
  st = sweep_shape(J, o, &P.nbuf, &P.maxtask);
  if (st != HSP_OK) return st;

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
  if (P.sponge) {
    P.o_k2i = c.take(nf * sizeof(double));
    P.o_bx = c.take(P.nf1 * sizeof(double));
    P.o_by = c.take(P.nf2 * sizeof(double));
  }
  const int Nc1 = P.dd_n1 + 1, Nc2 = P.dd_n2 + 1;  // DD level cells
  if (P.two_grid) {
    P.o_cxA = c.take(Nc1 * sizeof(cd));
    P.o_cxB = c.take(Nc1 * sizeof(cd));
    P.o_cyA = c.take(Nc2 * sizeof(cd));
    P.o_cyB = c.take(Nc2 * sizeof(cd));
    P.o_ck2c = c.take((size_t)Nc1 * Nc2 * sizeof(double));
    if (P.sponge) P.o_ck2ci = c.take((size_t)Nc1 * Nc2 * sizeof(double));
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
  P.o_red = c.take((size_t)P.maxtask * 2 * P.nchunk * P.nl_max * P.tsize);
  P.o_ctr = c.take(64 * sizeof(int));
  P.o_slabs = c.take(J * sizeof(SlabDev));
  P.o_slabA = c.take(P.n_slabA * sizeof(cd));
  P.o_slabB = c.take(P.n_slabA * sizeof(cd));
  P.o_xmap = c.take(P.n_xmap * sizeof(int));
  P.o_fac = c.take(P.n_fac * P.tsize);
  P.o_facscr = c.take((size_t)J * kMaxSlabLayers * kMaxSlabLayers * sizeof(cd));
  P.o_status = c.take(64);
  P.o_growth = c.take((size_t)J * sizeof(double));
  P.n_tasks = 2 * (size_t)J + 8;
  P.o_tasks = c.take(P.n_tasks * sizeof(TaskDev));
  P.o_tcoef = c.take(P.n_tasks * trans_coef_elems(P.dd_n2) * sizeof(cd));
  // sweep vectors (DD level, precision of the preconditioner)
  P.o_swf = c.take(nd * P.tsize);
  P.o_swg = c.take(nd * P.tsize);
  P.o_swu = c.take(nd * P.tsize);
  P.o_swB = c.take((size_t)P.nbuf * 2 * P.dd_n2 * P.tsize);
  P.o_swscr = c.take((size_t)P.maxtask * P.dd_n2 * P.nl_max * P.tsize);
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

}  // namespace hsp


namespace hsp {

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
  std::vector<char> written(std::max(2, P.nbuf), 0);
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
  // MidSolveIn / MidSolveOut of Table 2 on slab j (buffers: forward and
  // backward data in, or forward and backward data out)
  auto midin = [&](int j, int src, int bf, int bb) {
    TaskDev t = blank(j);
    t.a = t.at = be[j - 1];
    t.b = t.bt = bt[j];
    t.t1 = (j > 1 && written[bf]) ? 1 : 0;
    t.bin_f = bf;
    t.beta_in = be[j - 1];
    t.t3 = (j < J && written[bb]) ? 1 : 0;
    t.bin_b = bb;
    t.bt_in = bt[j];
    t.src = src;
    return t;
  };
  auto midout = [&](int j, int src, int bf, int bb) {
    TaskDev t = blank(j);
    t.a = t.at = bt[j - 1];
    t.b = t.bt = be[j];
    t.t2 = (j < J) ? 1 : 0;
    t.bout_f = bf;
    t.beta_out = be[j];
    t.t4 = (j > 1) ? 1 : 0;
    t.bout_b = bb;
    t.bt_out = bt[j - 1];
    t.src = src;
    return t;
  };
  auto run_stage = [&](std::vector<TaskDev> ts) {
    for (auto& t : ts) mark(t);
    push_stage(ts);
  };
  if (C->opt.sweep == HSP_SWEEP_NX) {
    // SweepingPrecNX: the X-sweeps of the N groups share every stage; the
    // boundary slabs between the groups are solved first (on f) and last
    // (on g).  Forward data of group m in buffer 2(m-1), backward data in
    // 2(m-1)+1.
    std::vector<int> jc, jm;
    (void)nx_cells(J, C->opt.ncell, jc, jm);  // validated by the plan
    const int N = C->opt.ncell;
    auto BF = [](int m) { return 2 * (m - 1); };
    auto BB = [](int m) { return 2 * (m - 1) + 1; };
    {
      std::vector<TaskDev> ts;
      for (int m = 1; m < N; ++m) ts.push_back(midout(jc[m], 0, BF(m + 1), BB(m)));
      run_stage(ts);
    }
    for (int st = 1;; ++st) {
      std::vector<TaskDev> ts;
      for (int m = 1; m <= N; ++m) {
        if (jc[m - 1] + st <= jm[m] - 1) ts.push_back(fwd(jc[m - 1] + st, 0, BF(m)));
        if (jc[m] - st >= jm[m] + 1) ts.push_back(bwd(jc[m] - st, 0, BB(m)));
      }
      if (ts.empty()) break;
      run_stage(ts);
    }
    {
      std::vector<TaskDev> ts;
      for (int m = 1; m <= N; ++m) ts.push_back(midin(jm[m], 0, BF(m), BB(m)));
      push_stage(ts);
    }
    S.push_back(Stage{1, 0, 0, 0, 0.0, 0.0});
    std::fill(written.begin(), written.end(), 0);
    {
      std::vector<TaskDev> ts;
      for (int m = 1; m <= N; ++m) ts.push_back(midout(jm[m], 1, BB(m), BF(m)));
      run_stage(ts);
    }
    for (int st = 1;; ++st) {
      std::vector<TaskDev> ts;
      for (int m = 1; m <= N; ++m) {
        if (jm[m] - st >= jc[m - 1] + 1) ts.push_back(bwd(jm[m] - st, 1, BF(m)));
        if (jm[m] + st <= jc[m] - 1) ts.push_back(fwd(jm[m] + st, 1, BB(m)));
      }
      if (ts.empty()) break;
      run_stage(ts);
    }
    {
      std::vector<TaskDev> ts;
      for (int m = 1; m < N; ++m) ts.push_back(midin(jc[m], 1, BB(m), BF(m + 1)));
      push_stage(ts);
    }
    return;
  }
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
  std::fill(written.begin(), written.end(), 0);
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

}  // namespace hsp

namespace {

// ---------------------------------------------------------------------------
// Sweep, two-grid cycle and preconditioner
// ---------------------------------------------------------------------------
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
  if (std::is_same<T, float>::value && smooth_fused_ok(C->fine, nu)) {
    // each smoothing phase as one kernel (LDS tiles with a halo of nu nodes)
    cd* res = C->at<double>(P.o_tgres);
    cx<T>* rc = C->at<T>(P.o_tgrc);
    cx<T>* ec = C->at<T>(P.o_tgec);
    prof_begin(C, HSP_PROF_SMOOTH, s);
    launch_smooth_pre(C->fine, nu, wj, r, BIdx{}, reinterpret_cast<cf*>(xa), BIdx{}, res, BIdx{}, 1, s);
    // r, k^2 read; x_nu (complex64) and the residual (complex128) written
    prof_end(C, HSP_PROF_SMOOTH, s, (double)nf * (2.0 * sizeof(cd) + sizeof(double) + sizeof(cf)));
    prof_begin(C, HSP_PROF_TRANSFER, s);
    launch_restrict<double, T>(C->tr, res, rc, s);
    prof_end(C, HSP_PROF_TRANSFER, s, (double)nf * sizeof(cd) + (double)nc * sizeof(cx<T>));
    run_sweep<T>(C, rc, ec, s);
    prof_begin(C, HSP_PROF_SMOOTH, s);
    launch_smooth_post(C->fine, C->tr, nu, wj, r, BIdx{}, reinterpret_cast<const cf*>(xa), BIdx{},
                       reinterpret_cast<const cf*>(ec), BIdx{}, z, BIdx{}, 1, s);
    // x, r, k^2 read, the coarse correction read, z written
    prof_end(C, HSP_PROF_SMOOTH, s,
             (double)nf * (2.0 * sizeof(cd) + sizeof(double) + sizeof(cx<T>)) + (double)nc * sizeof(cx<T>));
    return;
  }
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
  if (C->d3) {
    d3_precond(C, r, z, s);
    return;
  }
  if (C->opt.precision == HSP_MIXED)
    run_precond<float>(C, r, z, s);
  else
    run_precond<double>(C, r, z, s);
}




}  // namespace

namespace hsp {

hsp_status fail(hsp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

DebugKnobs& debug_knobs() {
  static DebugKnobs k;
  return k;
}

double growth_limit(size_t tsize) {
  if (debug_knobs().growth_limit > 0) return debug_knobs().growth_limit;
  const double eps = tsize == sizeof(cf) ? 1.1920929e-7 : 2.220446049250313e-16;
  return 0.01 / eps;
}

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

}  // namespace hsp

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
  o->krylov_fp32 = 0;
  o->ncell = 2;
  o->slab_factor = HSP_SLAB_AUTO;
  return HSP_OK;
}

hsp_status hsp_workspace_size(const hsp_grid* grid, int J, const hsp_options* opt, size_t* bytes) {
  if (!bytes) return fail(HSP_EINVAL, "null bytes");
  if (grid && grid->dim == 3) return d3_workspace_size(grid, J, opt, bytes);
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
  if (grid && grid->dim == 3) {
    hsp_status st3 = d3_setup(c_dev, omega, grid, J, opt, ws_dev, ws_bytes, S_(stream), out);
    if (st3 == HSP_OK) g_err = "no error";
    return st3;
  }
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
    if (w > 0 && !P.sponge) {
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
  if (P.sponge) {
    // beta per unknown node and axis: beta_max (dist / d)^2 inside the layers
    auto beta_axis = [&](int N, int w, std::vector<double>& b) {
      b.assign(N - 1, 0.0);
      if (w <= 0) return;
      const double d = w * h;
      const double bmax = grid->S_outer > 0 ? grid->S_outer : 3.0 * std::log(100.0) / ((omega / C->c_pml) * d);
      for (int i = 1; i < N; ++i) {
        const double x = i * h;
        const double dist = std::max(std::max(d - x, x - (N - w) * h), 0.0);
        b[i - 1] = bmax * (dist / d) * (dist / d);
      }
    };
    std::vector<double> bx, by;
    beta_axis(P.Nf1, grid->pml[0], bx);
    beta_axis(P.Nf2, grid->pml[1], by);
    up(P.o_bx, bx.data(), bx.size() * sizeof(double));
    up(P.o_by, by.data(), by.size() * sizeof(double));
  }
  C->fine.kind = P.fine_kind;
  C->fine.n1 = P.nf1;
  C->fine.n2 = P.nf2;
  C->fine.h2 = h * h;
  C->fine.xA = C->at<double>(P.o_fxA);
  C->fine.xB = C->at<double>(P.o_fxB);
  C->fine.yA = C->at<double>(P.o_fyA);
  C->fine.yB = C->at<double>(P.o_fyB);
  C->fine.xmap = nullptr;
  C->fine.k2i = nullptr;
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
    if (P.sponge) {
      // the coefficients come from the real k^2; the operator takes the
      // damped k^2 (1 + i beta)^2, averaged to the cells part by part
      CHK(hipStreamSynchronize(s));  // beta arrays uploaded
      launch_sponge_k2(P.nf1, P.nf2, C->raw<double>(P.o_bx), C->raw<double>(P.o_by), C->raw<double>(P.o_k2n),
                       C->raw<double>(P.o_k2i), s);
      launch_cell_average(C->raw<double>(P.o_k2n), P.nf1, P.nf2, C->raw<int>(P.o_avgx0), C->raw<double>(P.o_avgwx),
                          Nc1, C->raw<int>(P.o_avgy0), C->raw<double>(P.o_avgwy), Nc2, C->raw<double>(P.o_ck2c), s);
      launch_cell_average(C->raw<double>(P.o_k2i), P.nf1, P.nf2, C->raw<int>(P.o_avgx0), C->raw<double>(P.o_avgwx),
                          Nc1, C->raw<int>(P.o_avgy0), C->raw<double>(P.o_avgwy), Nc2, C->raw<double>(P.o_ck2ci), s);
      C->fine.k2i = C->raw<double>(P.o_k2i);
    }
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
    C->coarse.k2i = P.sponge ? C->raw<double>(P.o_ck2ci) : nullptr;
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
    if (P.sponge) {
      CHK(hipStreamSynchronize(s));  // beta arrays uploaded
      launch_sponge_k2(P.nf1, P.nf2, C->raw<double>(P.o_bx), C->raw<double>(P.o_by), C->raw<double>(P.o_k2n),
                       C->raw<double>(P.o_k2i), s);
      C->fine.k2i = C->raw<double>(P.o_k2i);
    }
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
  C->tcoef = C->raw<cd>(P.o_tcoef);
  launch_trans_coef(C->tasks_dev, (int)C->tasks_host.size(), C->slabs_dev, C->dd, C->raw<cd>(P.o_tcoef), s);
  for (hipError_t e : errs)
    if (e != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string("upload: ") + hipGetErrorString(e)));

  // factorization of all slabs, then the chunk transfer matrices
  int* status = C->raw<int>(P.o_status);
  CHK(hipMemsetAsync(status, 0, sizeof(int), s));
  CHK(hipMemsetAsync(C->raw<int>(P.o_ctr), 0, 64 * sizeof(int), s));
  double* growth = C->raw<double>(P.o_growth);
  const int dbg = debug_knobs().singular_slab;
  if (P.tsize == sizeof(cf))
    launch_factor<float>(C->slabs_dev, J, P.nl_max, P.dd_n2, P.chunk, P.nchunk, reinterpret_cast<cf*>(C->factors),
                         C->at<double>(P.o_setup), C->at<double>(P.o_facscr), C->at<double>(P.o_ttmp), status,
                         growth, dbg, s);
  else
    launch_factor<double>(C->slabs_dev, J, P.nl_max, P.dd_n2, P.chunk, P.nchunk, reinterpret_cast<cd*>(C->factors),
                          C->at<double>(P.o_setup), C->at<double>(P.o_facscr), C->at<double>(P.o_ttmp), status,
                          growth, dbg, s);
  CHK(hipGetLastError());
  int hstat = 0;
  std::vector<double> hgrowth(J);
  CHK(hipMemcpyAsync(&hstat, status, sizeof(int), hipMemcpyDeviceToHost, s));
  CHK(hipMemcpyAsync(hgrowth.data(), growth, J * sizeof(double), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  if (hstat != 0) return cleanup(fail(HSP_ESINGULAR, "zero or non-finite pivot in a slab factorization"));
  C->growth = *std::max_element(hgrowth.begin(), hgrowth.end());
  if (!(C->growth <= growth_limit(P.tsize)))
    return cleanup(fail(HSP_ESINGULAR, "growth factor " + std::to_string(C->growth) +
                                           " of the slab Schur complements exceeds the limit " +
                                           std::to_string(growth_limit(P.tsize))));
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
  if (C->d3) {
    d3_info(C, info);
    return HSP_OK;
  }
  info->dim = 2;
  info->n_fine_z = 0;
  info->n_coarse_z = 0;
  info->n_fine[0] = C->P.nf1;
  info->n_fine[1] = C->P.nf2;
  info->n_coarse[0] = C->P.two_grid ? C->P.nc1 : 0;
  info->n_coarse[1] = C->P.two_grid ? C->P.nc2 : 0;
  info->J = C->J;
  info->max_slab_layers = C->P.nl_max;
  info->precision = C->opt.precision;
  info->two_grid = C->P.two_grid;
  info->pivot_growth = C->growth;
  info->slab_factor = HSP_SLAB_BLOCK;
  return HSP_OK;
}

hsp_status hsp_debug_set(int knob, double value) {
  switch (knob) {
    case HSP_DEBUG_SINGULAR_SLAB:
      debug_knobs().singular_slab = (int)value;
      return HSP_OK;
    case HSP_DEBUG_GROWTH_LIMIT:
      debug_knobs().growth_limit = value;
      return HSP_OK;
    default:
      return fail(HSP_EINVAL, "unknown debug knob");
  }
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
  if (C->d3) return d3_rhs(C, (const cd*)f, (cd*)b, S_(stream));
  launch_scale_rhs_arrays(C->P.nf1, C->P.nf2, C->h * C->h, C->at<double>(C->P.o_ixn), C->at<double>(C->P.o_iyn),
                          (const cd*)f, (cd*)b, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_apply_operator(hsp_handle C, const void* x, void* y, void* stream) {
  if (!C || !x || !y || x == y) return fail(HSP_EINVAL, "null or aliased argument");
  if (C->d3) {
    d3_fine_apply(C, 0, (const cd*)x, nullptr, (cd*)y, S_(stream));
    HIPCHK(hipGetLastError());
    return HSP_OK;
  }
  launch_stencil<double, double, double, double>(C->fine, 0, (const cd*)x, (const cd*)nullptr, (cd*)y, 0.0,
                                                 S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_apply_level_operator(hsp_handle C, int level, const void* x, void* y, void* stream) {
  if (!C || !x || !y || x == y) return fail(HSP_EINVAL, "null or aliased argument");
  if (C->d3) return d3_apply_level_operator(C, level, (const cd*)x, (cd*)y, S_(stream));
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
  if (C->d3) return d3_restrict(C, (const cd*)rf, (cd*)rc, S_(stream));
  if (!C->P.two_grid) return fail(HSP_EINVAL, "no coarse level");
  launch_restrict<double, double>(C->tr, (const cd*)rf, (cd*)rc, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_prolong_add(hsp_handle C, const void* ec, void* xf, void* stream) {
  if (!C || !ec || !xf) return fail(HSP_EINVAL, "null argument");
  if (C->d3) return d3_prolong_add(C, (const cd*)ec, (cd*)xf, S_(stream));
  if (!C->P.two_grid) return fail(HSP_EINVAL, "no coarse level");
  launch_prolong_add<double, double>(C->tr, (const cd*)ec, (cd*)xf, S_(stream));
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status hsp_smooth(hsp_handle C, const void* r, void* x, int steps, void* stream) {
  if (!C || !r || !x || r == x || steps < 1) return fail(HSP_EINVAL, "bad argument");
  if (C->d3) return d3_smooth(C, (const cd*)r, (cd*)x, steps, S_(stream));
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
  if (C->d3) return d3_sweep(C, (const cd*)f, (cd*)u, S_(stream));
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
  if (C->d3) return d3_slab_solve(C, j, (const cd*)b, (cd*)x, S_(stream));
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
  if (C->d3) return fail(HSP_EINVAL, "the gradient is implemented for 2-D problems");
  if (C->P.sponge) return fail(HSP_EINVAL, "the gradient is implemented for PML layers, not sponge layers");
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
  if (C->d3) return d3_check(C);
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
  // fine operator: y = A x (mode 0) or y = b - A x (mode 1)
  auto fine_op = [&](int mode, const cd* xx, const cd* bb, cd* yy) {
    if (C->d3)
      d3_fine_apply(C, mode, xx, bb, yy, s);
    else
      launch_stencil<double, double, double, double>(A, mode, xx, bb, yy, 0.0, s);
  };
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
    fine_op(1, x, b, V);
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
      fine_op(0, zk, nullptr, w);
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
  fine_op(1, x, b, w);
  dotn(w, 1, w, hb + 2 * (m + 1));
  HIPCHK(hipMemcpyAsync(&hn, hb + 2 * (m + 1), sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double rr = std::sqrt(std::max(hn.re, 0.0)) / bnorm;
  if (conj_transpose) launch_convert<double, double>(x, x, n, 1, s);
  HIPCHK(hipGetLastError());
  if (C->d3) {
    const hsp_status st3 = d3_check(C);
    if (st3 != HSP_OK) return st3;
  }
  if (iters) *iters = it;
  if (relres) *relres = rr;
  if (!done && rr > tol) return fail(HSP_ENOCONV, "maxit reached before the tolerance");
  return HSP_OK;
}

}  // extern "C"

