// Many right-hand sides of one or several problems (media / frequencies)
// solved together: the multi-RHS pipelining of Sec. 5, where the slab
// factors of a problem serve all of its sources, extended to several
// problems whose sweep stages share launches.
//
// A group is a list of members (a set-up handle and its number of
// right-hand sides).  Every member gets a slice of the caller's group
// workspace (per right-hand-side vectors, FGMRES bases, slab scratch).  The
// stage lists of the members are aligned on the residual of the sweep (the
// coarse residual between MidSolveIn and MidSolveOut, Table 3), and every
// step of the aligned schedule is one launch pair over the work items of
// all members that have a slab stage at that step.  FGMRES runs one process
// per right-hand side, all advanced in lock step with one host
// synchronisation per iteration; converged right-hand sides leave the
// launches.  Optionally the preconditioner application is captured once per
// active set in a HIP graph and replayed, the current basis vector being
// selected through a device-side offset.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ctx.h"

using namespace hsp;

namespace {

constexpr int kMaxTile = 8;

// (task, tile) slots of a stage, times the tile: >= maxtask ceil(R/rb) rb for
// every rb <= 8 (maxtask: the most slab solves in one stage of the sweep)
inline size_t batch_slots(int R, int maxtask) { return (size_t)maxtask * (size_t)(R + kMaxTile - 1); }

// Layout of one member's slice of a group workspace.
struct BatchLayout {
  int R = 0, m = 0, nblk = 0;
  size_t hs = 0;  // hb entries per right-hand side
  size_t o_xa, o_xb, o_res, o_rc, o_ec, o_swf, o_swg, o_swu, o_swB, o_scr, o_red, o_ctr;
  size_t o_V, o_Z, o_w, o_bc, o_part, o_hb, o_act, o_upd, o_y, o_dyn;
  size_t total = 0;
};

BatchLayout batch_layout(const Plan& P, int R, int m, bool v32) {
  BatchLayout B;
  B.R = R;
  B.m = m;
  Carver c;
  const size_t nf = (size_t)P.nf1 * P.nf2, nd = (size_t)P.dd_n1 * P.dd_n2, T = P.tsize;
  const size_t slots = batch_slots(R, P.maxtask);
  B.o_xa = c.take(R * nf * T);
  B.o_xb = c.take(R * nf * T);
  B.o_res = c.take(P.two_grid ? R * nf * sizeof(cd) : 0);
  B.o_rc = c.take(P.two_grid ? R * nd * T : 0);
  B.o_ec = c.take(P.two_grid ? R * nd * T : 0);
  B.o_swf = c.take(R * nd * T);
  B.o_swg = c.take(R * nd * T);
  B.o_swu = c.take(R * nd * T);
  B.o_swB = c.take(R * (size_t)P.nbuf * 2 * (size_t)P.dd_n2 * T);
  B.o_scr = c.take(slots * P.dd_n2 * P.nl_max * T);
  B.o_red = c.take(slots * 2 * P.nchunk * P.nl_max * T);
  B.o_ctr = c.take(2 * slots * sizeof(int));
  B.nblk = batch_dot_blocks(nf, R);
  B.hs = 2 * (size_t)(m + 2) + 2;
  // Krylov basis V in complex128 (complex64 with krylov_fp32) and the
  // preconditioned vectors Z in the precision of the preconditioner (exact
  // for its output); everything else of FGMRES in complex128
  B.o_V = c.take((size_t)R * (m + 1) * nf * (v32 ? sizeof(cf) : sizeof(cd)));
  B.o_Z = c.take((size_t)R * m * nf * T);
  B.o_w = c.take(R * nf * sizeof(cd));
  B.o_bc = c.take(R * nf * sizeof(cd));
  B.o_part = c.take((size_t)2 * R * (m + 1) * B.nblk * sizeof(cd));
  B.o_hb = c.take(R * B.hs * sizeof(cd));
  B.o_act = c.take(R * sizeof(int));
  B.o_upd = c.take(R * sizeof(int));
  B.o_y = c.take((size_t)R * m * sizeof(cd));
  B.o_dyn = c.take(4 * sizeof(long long));
  B.total = c.off + 256;
  return B;
}

int residual_index(const hsp_ctx* C) {
  for (size_t i = 0; i < C->stages.size(); ++i)
    if (C->stages[i].residual) return (int)i;
  return 0;
}

struct Member {
  hsp_ctx* C = nullptr;
  int R = 0;
  BatchLayout B;
  size_t ws_off = 0;  // byte offset of the member's slice
  char* ws = nullptr;
  int off = 0;        // step of the member's first stage
  template <class X>
  X* at(size_t o) const {
    return reinterpret_cast<X*>(ws + o);
  }
};

// Input / output vectors of one member's preconditioner application:
// right-hand side j (slot j) at r + br.off(j), result at z + bz.off(j).
struct PrecIO {
  const void* r = nullptr;
  int r32 = 0;  // r is complex64 (else complex128)
  BIdx br;
  void* z = nullptr;
  int z32 = 0;  // z is complex64 (else complex128)
  BIdx bz;
};

struct Group {
  std::vector<Member> mem;
  int m = 0;
  int nsteps = 0;
  bool mixed = false;
  bool v32 = false;  // complex64 Arnoldi basis (mixed precision with krylov_fp32)
  size_t o_segs = 0, total = 0;
  char* ws = nullptr;
  BSeg* segs_dev = nullptr;
  struct Step {
    int first = 0, nseg = 0, nitems = 0, nl = 0, m = 0;
  };
  std::vector<Step> steps;
  std::vector<BSeg> segs_host;
  std::vector<int> seg_key;  // (rb, nact...) the table was built for
  // graph of one preconditioner application
  hipGraphExec_t exec = nullptr;
  std::vector<int> graph_key;
  hipStream_t cap = nullptr;
  ~Group() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// Sizes and offsets of a group workspace (members, then the segment table).
hsp_status group_plan(int nprob, const hsp_handle* hds, const int* nrhs, int restart, Group& G) {
  if (nprob < 1 || !hds || !nrhs) return fail(HSP_EINVAL, "a group needs nprob >= 1 handles and right-hand-side counts");
  if (restart < 1) return fail(HSP_EINVAL, "restart must be >= 1");
  G.mem.clear();
  G.m = restart;
  Carver c;
  int rmax = 0;
  for (int p = 0; p < nprob; ++p) {
    if (!hds[p]) return fail(HSP_EINVAL, "null handle in group");
    if (hds[p]->d3) return fail(HSP_EINVAL, "batched and grouped solves are implemented for 2-D problems");
    if (nrhs[p] < 0) return fail(HSP_EINVAL, "nrhs must be >= 0");
    const bool mixed = hds[p]->opt.precision == HSP_MIXED;
    const bool v32 = mixed && hds[p]->opt.krylov_fp32 != 0;
    if (p == 0) {
      G.mixed = mixed;
      G.v32 = v32;
    }
    if (mixed != G.mixed || v32 != G.v32)
      return fail(HSP_EINVAL, "the problems of a group must share the precision and the Krylov storage");
    for (int q = 0; q < p; ++q)
      if (hds[q] == hds[p]) return fail(HSP_EINVAL, "a handle appears twice in a group");
    Member mb;
    mb.C = hds[p];
    mb.R = nrhs[p];
    if (mb.R > 0) {
      mb.B = batch_layout(mb.C->P, mb.R, restart, G.v32);
      mb.ws_off = c.take(mb.B.total);
    }
    rmax = std::max(rmax, residual_index(mb.C));
    G.mem.push_back(mb);
  }
  G.nsteps = 0;
  for (auto& mb : G.mem) {
    const int o = rmax - residual_index(mb.C);
    G.nsteps = std::max(G.nsteps, o + (int)mb.C->stages.size());
  }
  G.o_segs = c.take((size_t)G.nsteps * nprob * sizeof(BSeg));
  G.total = c.off + 256;
  return HSP_OK;
}

// Places the members in the workspace and sets their stage offsets.
void group_bind(Group& G, void* ws) {
  G.ws = reinterpret_cast<char*>(ws);
  int rmax = 0;
  for (auto& mb : G.mem) rmax = std::max(rmax, residual_index(mb.C));
  for (auto& mb : G.mem) {
    if (mb.R > 0) mb.ws = G.ws + mb.ws_off;
    mb.off = rmax - residual_index(mb.C);
  }
  G.segs_dev = reinterpret_cast<BSeg*>(G.ws + G.o_segs);
}

// Segment table of every step for the active counts nact (one launch
// triple per step covers the slab stages of all members at that step).
hsp_status build_segments(Group& G, const std::vector<int>& nact, int rb, hipStream_t s) {
  std::vector<int> key(1, rb);
  key.insert(key.end(), nact.begin(), nact.end());
  if (key == G.seg_key) return HSP_OK;
  HIPCHK(hipStreamSynchronize(s));  // the host table may still feed a copy
  G.seg_key = key;
  G.steps.assign(G.nsteps, Group::Step{});
  G.segs_host.clear();
  for (int st = 0; st < G.nsteps; ++st) {
    Group::Step& S = G.steps[st];
    S.first = (int)G.segs_host.size();
    for (size_t p = 0; p < G.mem.size(); ++p) {
      const Member& mb = G.mem[p];
      const int idx = st - mb.off;
      if (nact[p] == 0 || idx < 0 || idx >= (int)mb.C->stages.size()) continue;
      const Stage& sg = mb.C->stages[idx];
      if (sg.residual) continue;
      const Plan& P = mb.C->P;
      const BatchLayout& B = mb.B;
      BSeg q;
      std::memset(&q, 0, sizeof(q));
      q.tasks = mb.C->tasks_dev + sg.first;
      q.slabs = mb.C->slabs_dev;
      q.G = mb.C->dd;
      q.f = mb.ws + (P.two_grid ? B.o_rc : B.o_swf);
      q.g = mb.ws + B.o_swg;
      q.u = mb.ws + (P.two_grid ? B.o_ec : B.o_swu);
      q.bufs = mb.ws + B.o_swB;
      q.scratch = mb.ws + B.o_scr;
      q.factors = mb.C->factors;
      q.red = mb.ws + B.o_red;
      q.counters = mb.at<int>(B.o_ctr);
      q.tcoef = mb.C->tcoef + (size_t)sg.first * trans_coef_elems(P.dd_n2);
      q.ld = (size_t)P.dd_n1 * P.dd_n2;
      q.ntasks = sg.ntasks;
      q.ntiles = (nact[p] + rb - 1) / rb;
      q.nact = nact[p];
      q.nl_max = P.nl_max;
      q.m = P.chunk;
      q.P = P.nchunk;
      q.item0 = S.nitems;
      q.nbuf = P.nbuf;
      S.nitems += q.ntasks * q.P * q.ntiles;
      S.nl = std::max(S.nl, sg.nl);
      S.m = std::max(S.m, P.chunk);
      G.segs_host.push_back(q);
      ++S.nseg;
    }
  }
  if (!G.segs_host.empty())
    HIPCHK(hipMemcpyAsync(G.segs_dev, G.segs_host.data(), G.segs_host.size() * sizeof(BSeg), hipMemcpyHostToDevice,
                          s));
  return HSP_OK;
}

template <class X>
X* mptr(const Member& mb, size_t o) {
  return reinterpret_cast<X*>(mb.ws + o);
}

// One preconditioner application of every member with active right-hand
// sides (the two-grid cycle of Sec. 4 or the plain sweep), all slab stages
// of a step in one launch pair.  build_segments must have run for nact.
template <class T>
void run_precond_group(Group& G, const std::vector<int>& nact, const std::vector<PrecIO>& io, hipStream_t s) {
  const size_t nm = G.mem.size();
  // fine level down to the sweep input
  for (size_t p = 0; p < nm; ++p) {
    if (nact[p] == 0) continue;
    const Member& mb = G.mem[p];
    hsp_ctx* C = mb.C;
    const Plan& P = C->P;
    const BatchLayout& B = mb.B;
    const int na = nact[p];
    const size_t nf = (size_t)P.nf1 * P.nf2, nd = (size_t)P.dd_n1 * P.dd_n2;
    BIdx bf, bdd;
    bf.ld = nf;
    bdd.ld = nd;
    if (!P.two_grid) {
      if (io[p].r32)
        launch_convert<T, float>(static_cast<const cf*>(io[p].r), mptr<cx<T>>(mb, B.o_swf), nf, 0, s, na, io[p].br,
                                 bf);
      else
        launch_convert<T, double>(static_cast<const cd*>(io[p].r), mptr<cx<T>>(mb, B.o_swf), nf, 0, s, na,
                                  io[p].br, bf);
      launch_zero<T>(mptr<cx<T>>(mb, B.o_swu), (size_t)na * nd, s);
      continue;
    }
    const double wj = C->opt.omega_jac;
    const int nu = C->opt.nu;
    cx<T>* xa = mptr<cx<T>>(mb, B.o_xa);
    cx<T>* xb = mptr<cx<T>>(mb, B.o_xb);
    if (std::is_same<T, float>::value && smooth_fused_ok(C->fine, nu)) {
      cd* res = mptr<cd>(mb, B.o_res);
      prof_begin(C, HSP_PROF_SMOOTH, s);
      if (io[p].r32)
        launch_smooth_pre<float>(C->fine, nu, wj, static_cast<const cf*>(io[p].r), io[p].br,
                                 reinterpret_cast<cf*>(xa), bf, res, bf, na, s);
      else
        launch_smooth_pre<double>(C->fine, nu, wj, static_cast<const cd*>(io[p].r), io[p].br,
                                  reinterpret_cast<cf*>(xa), bf, res, bf, na, s);
      // r read, k^2 read, the last iterate (complex64) and the residual
      // (complex128) written
      const double rb = io[p].r32 ? sizeof(cf) : sizeof(cd);
      prof_end(C, HSP_PROF_SMOOTH, s, (double)na * nf * (rb + sizeof(double) + sizeof(cf) + sizeof(cd)));
      prof_begin(C, HSP_PROF_TRANSFER, s);
      launch_restrict<double, T>(C->tr, res, mptr<cx<T>>(mb, B.o_rc), s, na, bf, bdd);
      prof_end(C, HSP_PROF_TRANSFER, s, (double)na * ((double)nf * sizeof(cd) + (double)nd * sizeof(cx<T>)));
      launch_zero<T>(mptr<cx<T>>(mb, B.o_ec), (size_t)na * nd, s);
      continue;
    }
    const double jb = (double)na * nf * (sizeof(cd) + 2.0 * sizeof(cx<T>) + sizeof(double));
    prof_begin(C, HSP_PROF_SMOOTH, s);
    // the same steps for a complex128 or a complex64 right-hand side
    auto presmooth = [&](auto tag) {
      using TR = decltype(tag);
      const cx<TR>* r = static_cast<const cx<TR>*>(io[p].r);
      if (nu > 0) {
        launch_stencil<T, T, TR, T>(C->fine, 2, (const cx<T>*)nullptr, r, xa, wj, s, na, BIdx{}, io[p].br, bf);
        for (int k = 1; k < nu; ++k) {
          launch_stencil<T, T, TR, T>(C->fine, 2, xa, r, xb, wj, s, na, bf, io[p].br, bf);
          std::swap(xa, xb);
        }
      } else {
        launch_zero<T>(xa, (size_t)na * nf, s);
      }
      launch_stencil<double, T, TR, double>(C->fine, 1, xa, r, mptr<cd>(mb, B.o_res), 0.0, s, na, bf, io[p].br, bf);
    };
    if (io[p].r32)
      presmooth(0.0f);
    else
      presmooth(0.0);
    cd* res = mptr<cd>(mb, B.o_res);
    prof_end(C, HSP_PROF_SMOOTH, s, nu * jb + (double)na * nf * (2.0 * sizeof(cd) + sizeof(cx<T>) + sizeof(double)));
    prof_begin(C, HSP_PROF_TRANSFER, s);
    launch_restrict<double, T>(C->tr, res, mptr<cx<T>>(mb, B.o_rc), s, na, bf, bdd);
    prof_end(C, HSP_PROF_TRANSFER, s, (double)na * ((double)nf * sizeof(cd) + (double)nd * sizeof(cx<T>)));
    launch_zero<T>(mptr<cx<T>>(mb, B.o_ec), (size_t)na * nd, s);
  }
  // the sweeps, step by step
  hsp_ctx* C0 = G.mem[0].C;
  for (int st = 0; st < G.nsteps; ++st) {
    for (size_t p = 0; p < nm; ++p) {
      const Member& mb = G.mem[p];
      const int idx = st - mb.off;
      if (nact[p] == 0 || idx < 0 || idx >= (int)mb.C->stages.size() || !mb.C->stages[idx].residual) continue;
      hsp_ctx* C = mb.C;
      const Plan& P = C->P;
      const BatchLayout& B = mb.B;
      const size_t nd = (size_t)P.dd_n1 * P.dd_n2;
      BIdx bd;
      bd.ld = nd;
      cx<T>* f = mptr<cx<T>>(mb, P.two_grid ? B.o_rc : B.o_swf);
      cx<T>* u = mptr<cx<T>>(mb, P.two_grid ? B.o_ec : B.o_swu);
      prof_begin(C, HSP_PROF_COARSE, s);
      launch_stencil<T, T, T, T>(C->dd, 1, u, f, mptr<cx<T>>(mb, B.o_swg), 0.0, s, nact[p], bd, bd, bd);
      prof_end(C, HSP_PROF_COARSE, s, (double)nact[p] * nd * (3.0 * sizeof(cx<T>) + 4.0 * sizeof(double)));
    }
    const Group::Step& S = G.steps[st];
    if (S.nseg == 0) continue;
    double bytes = 0;
    for (size_t p = 0; p < nm; ++p) {
      const Member& mb = G.mem[p];
      const int idx = st - mb.off;
      if (nact[p] == 0 || idx < 0 || idx >= (int)mb.C->stages.size()) continue;
      const Stage& sg = mb.C->stages[idx];
      if (!sg.residual) bytes += sg.fac + (double)nact[p] * (sg.bytes - sg.fac);
    }
    prof_begin(C0, HSP_PROF_STAGE, s);
    launch_stage_group<T>(G.segs_dev + S.first, S.nseg, S.nitems, S.nl, S.m, G.seg_key[0], s);
    prof_end(C0, HSP_PROF_STAGE, s, bytes * sizeof(cx<T>));
  }
  // back to the fine level
  for (size_t p = 0; p < nm; ++p) {
    if (nact[p] == 0) continue;
    const Member& mb = G.mem[p];
    hsp_ctx* C = mb.C;
    const Plan& P = C->P;
    const BatchLayout& B = mb.B;
    const int na = nact[p];
    const size_t nf = (size_t)P.nf1 * P.nf2, nd = (size_t)P.dd_n1 * P.dd_n2;
    BIdx bf, bdd;
    bf.ld = nf;
    bdd.ld = nd;
    if (!P.two_grid) {
      if (io[p].z32)
        launch_convert<float, T>(mptr<cx<T>>(mb, B.o_swu), static_cast<cf*>(io[p].z), nf, 0, s, na, bf, io[p].bz);
      else
        launch_convert<double, T>(mptr<cx<T>>(mb, B.o_swu), static_cast<cd*>(io[p].z), nf, 0, s, na, bf,
                                  io[p].bz);
      continue;
    }
    const double wj = C->opt.omega_jac;
    const int nu = C->opt.nu;
    cx<T>* xa = mptr<cx<T>>(mb, B.o_xa);
    cx<T>* xb = mptr<cx<T>>(mb, B.o_xb);
    if (std::is_same<T, float>::value && smooth_fused_ok(C->fine, nu)) {
      prof_begin(C, HSP_PROF_SMOOTH, s);
      const cf* xin = reinterpret_cast<const cf*>(xa);
      const cf* ec = reinterpret_cast<const cf*>(mptr<cx<T>>(mb, B.o_ec));
      auto post = [&](auto rtag, auto ztag) {
        using TR = decltype(rtag);
        using TZ = decltype(ztag);
        launch_smooth_post<TR, TZ>(C->fine, C->tr, nu, wj, static_cast<const cx<TR>*>(io[p].r), io[p].br, xin, bf,
                                   ec, bdd, static_cast<cx<TZ>*>(io[p].z), io[p].bz, na, s);
      };
      if (io[p].r32 && io[p].z32)
        post(0.0f, 0.0f);
      else if (io[p].r32)
        post(0.0f, 0.0);
      else if (io[p].z32)
        post(0.0, 0.0f);
      else
        post(0.0, 0.0);
      // r, the pre-smoothed iterate, k^2 and the coarse correction read, z written
      const double rb = io[p].r32 ? sizeof(cf) : sizeof(cd), zb = io[p].z32 ? sizeof(cf) : sizeof(cd);
      prof_end(C, HSP_PROF_SMOOTH, s,
               (double)na * ((double)nf * (rb + sizeof(cf) + sizeof(double) + zb) + (double)nd * sizeof(cx<T>)));
      continue;
    }
    if (nu > 0 && nu % 2 == 0) std::swap(xa, xb);  // where the pre-smoothing ended
    prof_begin(C, HSP_PROF_TRANSFER, s);
    launch_prolong_add<T, T>(C->tr, mptr<cx<T>>(mb, B.o_ec), xa, s, na, bdd, bf);
    prof_end(C, HSP_PROF_TRANSFER, s, (double)na * ((double)nd * sizeof(cx<T>) + 2.0 * nf * sizeof(cx<T>)));
    if (nu == 0) {
      if (io[p].z32)
        launch_convert<float, T>(xa, static_cast<cf*>(io[p].z), nf, 0, s, na, bf, io[p].bz);
      else
        launch_convert<double, T>(xa, static_cast<cd*>(io[p].z), nf, 0, s, na, bf, io[p].bz);
      continue;
    }
    const double jb = (double)na * nf * (sizeof(cd) + 2.0 * sizeof(cx<T>) + sizeof(double));
    prof_begin(C, HSP_PROF_SMOOTH, s);
    auto postsmooth = [&](auto rtag, auto ztag) {
      using TR = decltype(rtag);
      using TZ = decltype(ztag);
      const cx<TR>* r = static_cast<const cx<TR>*>(io[p].r);
      for (int k = 0; k < nu; ++k) {
        if (k == nu - 1) {
          launch_stencil<T, T, TR, TZ>(C->fine, 2, xa, r, static_cast<cx<TZ>*>(io[p].z), wj, s, na, bf, io[p].br,
                                       io[p].bz);
        } else {
          launch_stencil<T, T, TR, T>(C->fine, 2, xa, r, xb, wj, s, na, bf, io[p].br, bf);
          std::swap(xa, xb);
        }
      }
    };
    if (io[p].r32 && io[p].z32)
      postsmooth(0.0f, 0.0f);
    else if (io[p].r32)
      postsmooth(0.0f, 0.0);
    else if (io[p].z32)
      postsmooth(0.0, 0.0f);
    else
      postsmooth(0.0, 0.0);
    prof_end(C, HSP_PROF_SMOOTH, s, nu * jb);
  }
}

void precond_group(Group& G, const std::vector<int>& nact, const std::vector<PrecIO>& io, hipStream_t s) {
  if (G.mixed)
    run_precond_group<float>(G, nact, io, s);
  else
    run_precond_group<double>(G, nact, io, s);
}

// The preconditioner application through a captured graph: captured (on a
// private stream) whenever the active counts or the tile change, then
// replayed on the caller's stream.
hsp_status precond_group_graph(Group& G, const std::vector<int>& nact, const std::vector<PrecIO>& io,
                               hipStream_t s) {
  std::vector<int> key = G.seg_key;
  if (G.exec == nullptr || key != G.graph_key) {
    if (G.exec) {
      HIPCHK(hipGraphExecDestroy(G.exec));
      G.exec = nullptr;
    }
    if (!G.cap) HIPCHK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    std::vector<bool> prof(G.mem.size());
    for (size_t p = 0; p < G.mem.size(); ++p) {
      prof[p] = G.mem[p].C->prof.on;
      G.mem[p].C->prof.on = false;  // no event records inside the graph
    }
    HIPCHK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    precond_group(G, nact, io, G.cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(G.cap, &graph);
    for (size_t p = 0; p < G.mem.size(); ++p) G.mem[p].C->prof.on = prof[p];
    if (e != hipSuccess) return fail(HSP_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      G.exec = nullptr;
      return fail(HSP_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(e2));
    }
    G.graph_key = key;
  }
  HIPCHK(hipGraphLaunch(G.exec, s));
  return HSP_OK;
}

// Default right-hand-side tile: the tile tuned for a single-member batch of
// this size, else the largest tile that still gives the stage launches about
// two work items per compute unit.
int default_tile(const Group& G, const std::vector<int>& nact) {
  if (G.mem.size() == 1 && G.mem[0].C->tuned_rb > 0 && G.mem[0].C->tuned_nact == nact[0])
    return G.mem[0].C->tuned_rb;
  for (int rb = kMaxTile; rb > 1; rb /= 2) {
    long items = 0;
    for (size_t p = 0; p < G.mem.size(); ++p)
      items += 2L * G.mem[p].C->P.nchunk * ((nact[p] + rb - 1) / rb);
    if (items >= 512) return rb;
  }
  return 1;
}

hsp_status check_tile(int tile) {
  if (tile != 0 && tile != 1 && tile != 2 && tile != 4 && tile != 8)
    return fail(HSP_EINVAL, "tile must be 0 (automatic), 1, 2, 4 or 8");
  return HSP_OK;
}

hsp_status check_ws(const Group& G, void* ws, size_t bytes) {
  if (!ws) return fail(HSP_EINVAL, "null group workspace");
  if (((uintptr_t)ws) & 255) return fail(HSP_EINVAL, "group workspace must be 256-byte aligned");
  if (bytes < G.total) return fail(HSP_ENOMEM, "group workspace too small: need " + std::to_string(G.total) + " bytes");
  return HSP_OK;
}

// The arrival counters of the stage launches start at zero.  by_kernel: clear
// them with a fill kernel instead of hipMemsetAsync.
hsp_status zero_counters(const Group& G, hipStream_t s, bool by_kernel = false) {
  for (const Member& mb : G.mem) {
    if (mb.R <= 0) continue;
    const size_t n = 2 * batch_slots(mb.R, mb.C->P.maxtask);  // even: cleared as n/2 complex64 zeros
    if (by_kernel)
      launch_zero<float>(mptr<cf>(mb, mb.B.o_ctr), n / 2, s);
    else
      HIPCHK(hipMemsetAsync(mptr<int>(mb, mb.B.o_ctr), 0, n * sizeof(int), s));
  }
  return HSP_OK;
}

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
  // residual estimate over columns 0..k-1; y (optional) receives the minimiser
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

// Per-member state of the grouped FGMRES.
struct MemberSolve {
  const cd* b = nullptr;  // right-hand sides (conjugated copy for A^H)
  cd* x = nullptr;
  std::vector<double> bnorm;
  std::vector<int> its, done, act, upd;
  std::vector<Arnoldi> ar;
  std::vector<cd> hh, yh;
  long long dyn = 0;  // host staging of the device offset k nf
};

hsp_status group_solve(Group& G, const void* const* b_in, void* const* u_out, double tol, int maxit, int conj,
                       int tile, int flags, int* iters, double* relres, hipStream_t s) {
  const int m = G.m;
  const size_t nm = G.mem.size();
  const bool graph = (flags & HSP_GROUP_GRAPH) != 0;
  std::vector<MemberSolve> ms(nm);
  hsp_status st = zero_counters(G, s);
  if (st != HSP_OK) return st;
  // ||b||
  for (size_t p = 0; p < nm; ++p) {
    const Member& mb = G.mem[p];
    MemberSolve& S = ms[p];
    if (mb.R == 0) continue;
    const Plan& P = mb.C->P;
    const BatchLayout& B = mb.B;
    const size_t nf = (size_t)P.nf1 * P.nf2;
    S.b = (const cd*)b_in[p];
    S.x = (cd*)u_out[p];
    if (!S.b || !S.x || (const void*)S.b == (const void*)S.x) return fail(HSP_EINVAL, "null or aliased vectors");
    if (conj) {
      cd* bc = mptr<cd>(mb, B.o_bc);
      launch_convert<double, double>(S.b, bc, (size_t)mb.R * nf, 1, s);
      S.b = bc;
    }
    BIdx bid;
    bid.ld = nf;
    cd* hb = mptr<cd>(mb, B.o_hb);
    launch_bmultidot(S.b, 0, bid, 1, S.b, bid, nf, mptr<cd>(mb, B.o_part), B.nblk, hb + 2 * (m + 1), B.hs, mb.R, s);
    S.hh.resize((size_t)mb.R * B.hs);
    S.yh.resize((size_t)mb.R * m);
    HIPCHK(hipMemcpyAsync(S.hh.data(), hb, (size_t)mb.R * B.hs * sizeof(cd), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (size_t p = 0; p < nm; ++p) {
    const Member& mb = G.mem[p];
    MemberSolve& S = ms[p];
    S.bnorm.assign(mb.R, 0.0);
    S.its.assign(mb.R, 0);
    S.done.assign(mb.R, 0);
    S.ar.resize(mb.R);
    for (int z = 0; z < mb.R; ++z) {
      S.bnorm[z] = std::sqrt(std::max(S.hh[(size_t)z * mb.B.hs + 2 * (m + 1)].re, 0.0));
      if (S.bnorm[z] == 0)
        S.done[z] = 1;
      else
        S.act.push_back(z);
    }
    if (mb.R > 0) launch_zero<double>(S.x, (size_t)mb.R * ((size_t)mb.C->P.nf1 * mb.C->P.nf2), s);
  }
  auto any_active = [&]() {
    for (auto& S : ms)
      if (!S.act.empty()) return true;
    return false;
  };
  // x += Z y for the right-hand sides in `list` of member p (k columns)
  auto update = [&](size_t p, const std::vector<int>& list, int k) -> hsp_status {
    if (list.empty() || k == 0) return HSP_OK;
    const Member& mb = G.mem[p];
    MemberSolve& S = ms[p];
    const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
    HIPCHK(hipStreamSynchronize(s));  // the staging arrays may still feed a copy
    S.upd = list;
    for (size_t i = 0; i < S.upd.size(); ++i) S.ar[S.upd[i]].lsq(k, S.yh.data() + i * m);
    cd* ydev = mptr<cd>(mb, mb.B.o_y);
    int* upd_d = mptr<int>(mb, mb.B.o_upd);
    HIPCHK(hipMemcpyAsync(ydev, S.yh.data(), S.upd.size() * m * sizeof(cd), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(upd_d, S.upd.data(), S.upd.size() * sizeof(int), hipMemcpyHostToDevice, s));
    BIdx bz, bx;
    bz.ld = (size_t)m * nf;
    bz.map = upd_d;
    bx.ld = nf;
    bx.map = upd_d;
    if (G.mixed)
      launch_bmultiaxpy<float>(mptr<cf>(mb, mb.B.o_Z), nf, bz, k, ydev, m, S.x, bx, nf, 0, (int)S.upd.size(), s);
    else
      launch_bmultiaxpy<double>(mptr<cd>(mb, mb.B.o_Z), nf, bz, k, ydev, m, S.x, bx, nf, 0, (int)S.upd.size(), s);
    return HSP_OK;
  };
  auto upload_act = [&](size_t p) -> hsp_status {
    MemberSolve& S = ms[p];
    if (!S.act.empty())
      HIPCHK(hipMemcpyAsync(mptr<int>(G.mem[p], G.mem[p].B.o_act), S.act.data(), S.act.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    return HSP_OK;
  };
  const int koff = 2 * (m + 1);  // hb offset of nu, h_kk, ||u_{k+1}||^2
  int it = 0;
  // relative true residual of right-hand side z of member p (after the
  // residual pass below)
  auto true_relres = [&](size_t p, int z) {
    const MemberSolve& S = ms[p];
    return S.bnorm[z] > 0 ? std::sqrt(std::max(S.hh[(size_t)z * G.mem[p].B.hs + 2 * (m + 1)].re, 0.0)) / S.bnorm[z]
                          : 0.0;
  };
  for (;;) {
    while (it < maxit && any_active()) {
      // residuals, their norms and the first basis vectors
      for (size_t p = 0; p < nm; ++p) {
        MemberSolve& S = ms[p];
        if (S.act.empty()) continue;
        const Member& mb = G.mem[p];
        const BatchLayout& B = mb.B;
        const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
        st = upload_act(p);
        if (st != HSP_OK) return st;
        const int na = (int)S.act.size();
        int* act_d = mptr<int>(mb, B.o_act);
        cd* w = mptr<cd>(mb, B.o_w);
        cd* hb = mptr<cd>(mb, B.o_hb);
        BIdx bx, bV, bw;
        bx.ld = nf;
        bx.map = act_d;
        bV.ld = (size_t)(m + 1) * nf;
        bV.map = act_d;
        bw.ld = nf;
        // r = b - A x in complex128, its norm, v_0 = r / ||r|| in the basis precision
        launch_stencil<double, double, double, double>(mb.C->fine, 1, S.x, S.b, w, 0.0, s, na, bx, bx, bw);
        launch_bmultidot(w, 0, bw, 1, w, bw, nf, mptr<cd>(mb, B.o_part), B.nblk, hb + 2 * (m + 1), B.hs, na, s);
        if (G.v32)
          launch_bnormalize<float>(w, bw, hb + 2 * (m + 1), B.hs, mptr<cf>(mb, B.o_V), bV, nf, na, s);
        else
          launch_bnormalize<double>(w, bw, hb + 2 * (m + 1), B.hs, mptr<cd>(mb, B.o_V), bV, nf, na, s);
        HIPCHK(hipMemcpyAsync(S.hh.data(), hb, (size_t)na * B.hs * sizeof(cd), hipMemcpyDeviceToHost, s));
      }
      HIPCHK(hipStreamSynchronize(s));
      for (size_t p = 0; p < nm; ++p) {
        MemberSolve& S = ms[p];
        std::vector<int> keep;
        for (size_t zi = 0; zi < S.act.size(); ++zi) {
          const int z = S.act[zi];
          const double beta = std::sqrt(std::max(S.hh[zi * G.mem[p].B.hs + 2 * (m + 1)].re, 0.0));
          if (beta <= tol * S.bnorm[z]) {
            S.done[z] = 1;
            continue;
          }
          S.ar[z].reset(m, beta);
          keep.push_back(z);
        }
        S.act.swap(keep);
        st = upload_act(p);
        if (st != HSP_OK) return st;
      }
      if (!any_active()) break;
      int k = 0;
      for (; k < m && it < maxit && any_active(); ++k) {
        std::vector<int> nact(nm);
        for (size_t p = 0; p < nm; ++p) nact[p] = (int)ms[p].act.size();
        const int rb = tile ? tile : default_tile(G, nact);
        st = build_segments(G, nact, rb, s);
        if (st != HSP_OK) return st;
        // z_k = M v_k (slot k of every active right-hand side)
        std::vector<PrecIO> io(nm);
        for (size_t p = 0; p < nm; ++p) {
          if (nact[p] == 0) continue;
          const Member& mb = G.mem[p];
          const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
          int* act_d = mptr<int>(mb, mb.B.o_act);
          io[p].br.ld = (size_t)(m + 1) * nf;
          io[p].br.map = act_d;
          io[p].bz.ld = (size_t)m * nf;
          io[p].bz.map = act_d;
          // slot k of the basis (complex64 with krylov_fp32) and of Z
          // (complex64 for the mixed-precision solver)
          const size_t vk = graph ? 0 : (size_t)k * nf;
          io[p].r32 = G.v32 ? 1 : 0;
          io[p].r = G.v32 ? (const void*)(mptr<cf>(mb, mb.B.o_V) + vk) : (const void*)(mptr<cd>(mb, mb.B.o_V) + vk);
          io[p].z32 = G.mixed ? 1 : 0;
          io[p].z = G.mixed ? (void*)(mptr<cf>(mb, mb.B.o_Z) + vk) : (void*)(mptr<cd>(mb, mb.B.o_Z) + vk);
          if (graph) {
            long long* dyn = mptr<long long>(mb, mb.B.o_dyn);
            ms[p].dyn = (long long)k * (long long)nf;
            HIPCHK(hipMemcpyAsync(dyn, &ms[p].dyn, sizeof(long long), hipMemcpyHostToDevice, s));
            io[p].br.dyn = dyn;
            io[p].bz.dyn = dyn;
          }
        }
        if (graph) {
          st = precond_group_graph(G, nact, io, s);
          if (st != HSP_OK) return st;
        } else {
          precond_group(G, nact, io, s);
        }
        // w = A z_k, delayed classical Gram-Schmidt: one projection pass
        // (basis against u_k and w) and one update pass (v_k final, u_{k+1}
        // and its norm)
        for (size_t p = 0; p < nm; ++p) {
          if (nact[p] == 0) continue;
          const Member& mb = G.mem[p];
          const BatchLayout& B = mb.B;
          const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
          int* act_d = mptr<int>(mb, B.o_act);
          cd* w = mptr<cd>(mb, B.o_w);
          cd* hb = mptr<cd>(mb, B.o_hb);
          cd* part = mptr<cd>(mb, B.o_part);
          BIdx bZk, bw, bVb;
          bZk.ld = (size_t)m * nf;
          bZk.map = act_d;
          bw.ld = nf;
          bVb.ld = (size_t)(m + 1) * nf;
          bVb.map = act_d;
          // algorithmic bytes (basis vectors in the basis precision): matvec
          // z read and w written per source, k^2 read once (the batched
          // stencil forms each node's coefficients once for a group of
          // sources); projection k+1 basis vectors (u_k in slot
          // k) and w read; update k basis vectors, u_k and w read, v_k and
          // u_{k+1} written
          const double vb = G.v32 ? sizeof(cf) : sizeof(cd), zb = G.mixed ? sizeof(cf) : sizeof(cd);
          const double na = nact[p];
          prof_begin(mb.C, HSP_PROF_KRYLOV, s);
          if (G.mixed)
            launch_stencil<double, float, double, double>(mb.C->fine, 0, mptr<cf>(mb, B.o_Z) + (size_t)k * nf,
                                                          (const cd*)nullptr, w, 0.0, s, nact[p], bZk, BIdx{}, bw);
          else
            launch_stencil<double, double, double, double>(mb.C->fine, 0, mptr<cd>(mb, B.o_Z) + (size_t)k * nf,
                                                           (const cd*)nullptr, w, 0.0, s, nact[p], bZk, BIdx{}, bw);
          prof_end(mb.C, HSP_PROF_KRYLOV, s, na * nf * (zb + sizeof(cd)) + (double)nf * sizeof(double));
          // blocks per right-hand side for the active count; the partial
          // buffer holds 2 (m+1) B.nblk entries for each of R right-hand
          // sides, and both passes use at most B.nblk R / nact per active one
          const int pcap = (int)std::max<long>(1, (long)B.nblk * mb.R / nact[p]);
          const int nbp = std::min(batch_dot_blocks(nf, nact[p]), pcap);
          const int nbu = std::min(batch_upd_blocks(nf, nact[p]), pcap);
          prof_begin(mb.C, HSP_PROF_PROJECT, s);
          if (G.v32)
            launch_bdcgs_project<float>(mptr<cf>(mb, B.o_V), nf, bVb, k, w, bw, nf, part, nbp, hb, B.hs, koff,
                                        nact[p], s);
          else
            launch_bdcgs_project<double>(mptr<cd>(mb, B.o_V), nf, bVb, k, w, bw, nf, part, nbp, hb, B.hs, koff,
                                         nact[p], s);
          prof_end(mb.C, HSP_PROF_PROJECT, s, na * nf * (vb * (k + 1.0) + sizeof(cd)));
          prof_begin(mb.C, HSP_PROF_UPDATE, s);
          if (G.v32)
            launch_bdcgs_update<float>(mptr<cf>(mb, B.o_V), nf, bVb, k, hb, B.hs, koff, w, bw, nf, part, nbu,
                                       hb + koff + 2, nact[p], s);
          else
            launch_bdcgs_update<double>(mptr<cd>(mb, B.o_V), nf, bVb, k, hb, B.hs, koff, w, bw, nf, part, nbu,
                                        hb + koff + 2, nact[p], s);
          prof_end(mb.C, HSP_PROF_UPDATE, s, na * nf * (vb * (k + 3.0) + sizeof(cd)));
          HIPCHK(hipMemcpyAsync(ms[p].hh.data(), hb, (size_t)nact[p] * B.hs * sizeof(cd), hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        ++it;
        for (size_t p = 0; p < nm; ++p) {
          MemberSolve& S = ms[p];
          if (S.act.empty()) continue;
          const size_t hs = G.mem[p].B.hs;
          std::vector<int> keep, conv;
          for (size_t zi = 0; zi < S.act.size(); ++zi) {
            const int z = S.act[zi];
            const cd* d = S.hh.data() + zi * hs;
            Arnoldi& a = S.ar[z];
            if (k > 0) {  // finalise column k-1 with the reorthogonalisation terms
              for (int j = 0; j < k; ++j) a.at(j, k - 1) += cplx(d[j].re, d[j].im);
              a.at(k, k - 1) = d[koff].re;
            }
            for (int j = 0; j < k; ++j) a.at(j, k) = cplx(d[k + 1 + j].re, d[k + 1 + j].im);
            a.at(k, k) = cplx(d[koff + 1].re, d[koff + 1].im);
            a.at(k + 1, k) = std::sqrt(std::max(d[koff + 2].re, 0.0));
            const double est = a.lsq(k + 1, nullptr);
            S.its[z] = it;
            if (est <= tol * S.bnorm[z]) {
              conv.push_back(z);
              S.done[z] = 1;
            } else {
              keep.push_back(z);
            }
          }
          st = update(p, conv, k + 1);
          if (st != HSP_OK) return st;
          if (keep.size() != S.act.size()) {
            S.act.swap(keep);
            st = upload_act(p);
            if (st != HSP_OK) return st;
          }
        }
      }
      // end of a restart cycle (or maxit): fold the active corrections into x
      for (size_t p = 0; p < nm; ++p) {
        st = update(p, ms[p].act, k);
        if (st != HSP_OK) return st;
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    // true residuals of every right-hand side
    for (size_t p = 0; p < nm; ++p) {
      const Member& mb = G.mem[p];
      if (mb.R == 0) continue;
      const BatchLayout& B = mb.B;
      const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
      BIdx bid;
      bid.ld = nf;
      cd* w = mptr<cd>(mb, B.o_w);
      cd* hb = mptr<cd>(mb, B.o_hb);
      launch_stencil<double, double, double, double>(mb.C->fine, 1, ms[p].x, ms[p].b, w, 0.0, s, mb.R, bid, bid,
                                                     bid);
      launch_bmultidot(w, 0, bid, 1, w, bid, nf, mptr<cd>(mb, B.o_part), B.nblk, hb + 2 * (m + 1), B.hs, mb.R, s);
      HIPCHK(hipMemcpyAsync(ms[p].hh.data(), hb, (size_t)mb.R * B.hs * sizeof(cd), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    // A right-hand side whose true residual misses the tolerance although
    // the least-squares estimate met it (with a complex64 basis the
    // estimate is only as good as the stored basis) gets another restart
    // cycle from its complex128 residual.
    bool again = false;
    for (size_t p = 0; p < nm && it < maxit; ++p) {
      MemberSolve& S = ms[p];
      for (int z = 0; z < G.mem[p].R; ++z)
        if (S.done[z] && S.bnorm[z] > 0 && true_relres(p, z) > tol) {
          S.done[z] = 0;
          S.act.push_back(z);
          again = true;
        }
    }
    if (!again) break;
  }
  if (conj)
    for (size_t p = 0; p < nm; ++p)
      if (G.mem[p].R > 0)
        launch_convert<double, double>(ms[p].x, ms[p].x,
                                       (size_t)G.mem[p].R * ((size_t)G.mem[p].C->P.nf1 * G.mem[p].C->P.nf2), 1, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  bool all = true;
  size_t o = 0;
  for (size_t p = 0; p < nm; ++p) {
    const Member& mb = G.mem[p];
    const MemberSolve& S = ms[p];
    for (int z = 0; z < mb.R; ++z, ++o) {
      const double rr = true_relres(p, z);
      if (iters) iters[o] = S.its[z];
      if (relres) relres[o] = rr;
      if (S.bnorm[z] > 0 && rr > tol) all = false;
    }
  }
  if (!all) return fail(HSP_ENOCONV, "maxit reached before the tolerance for some right-hand sides");
  return HSP_OK;
}

// r32, z32: the right-hand sides / the results are complex64 (the Krylov
// vectors of the mixed-precision solver), else complex128.
hsp_status group_precond(Group& G, const void* const* r, void* const* z, int tile, int flags, hipStream_t s,
                         int r32 = 0, int z32 = 0, bool zero_by_kernel = false) {
  const size_t nm = G.mem.size();
  std::vector<int> nact(nm);
  std::vector<PrecIO> io(nm);
  for (size_t p = 0; p < nm; ++p) {
    const Member& mb = G.mem[p];
    nact[p] = mb.R;
    if (mb.R == 0) continue;
    if (!r[p] || !z[p] || r[p] == z[p]) return fail(HSP_EINVAL, "null or aliased vectors");
    const size_t nf = (size_t)mb.C->P.nf1 * mb.C->P.nf2;
    io[p].r = r[p];
    io[p].r32 = r32;
    io[p].z = z[p];
    io[p].z32 = z32;
    io[p].br.ld = nf;
    io[p].bz.ld = nf;
  }
  hsp_status st = zero_counters(G, s, zero_by_kernel);
  if (st != HSP_OK) return st;
  st = build_segments(G, nact, tile ? tile : default_tile(G, nact), s);
  if (st != HSP_OK) return st;
  if (flags & HSP_GROUP_GRAPH) {
    st = precond_group_graph(G, nact, io, s);
    if (st != HSP_OK) return st;
  } else {
    precond_group(G, nact, io, s);
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

// ---- fixed device scratch of hsp_apply_precond_batch_noalloc --------------
// One copy of this array lives on every GPU the library runs on, from the
// first use until the process ends.  Host code never passes the symbol
// itself to a kernel: it is a host-side stand-in, and the device address of
// each GPU's copy comes from hipGetSymbolAddress with that GPU current.
constexpr size_t kNoallocScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch (looked up once per device).
hsp_status noalloc_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HSP_EDEVICE, "device index out of range for the fixed scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HSP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HSP_OK;
}

}  // namespace

extern "C" {

hsp_status hsp_group_workspace_size(int nprob, const hsp_handle* hds, const int* nrhs, int restart, size_t* bytes) {
  if (!bytes) return fail(HSP_EINVAL, "null bytes");
  Group G;
  hsp_status st = group_plan(nprob, hds, nrhs, restart, G);
  if (st != HSP_OK) return st;
  *bytes = G.total;
  return HSP_OK;
}

hsp_status hsp_apply_precond_group(int nprob, const hsp_handle* hds, const int* nrhs, const void* const* r_dev,
                                   void* const* z_dev, int tile, int flags, void* ws, size_t ws_bytes,
                                   void* stream) {
  Group G;
  hsp_status st = group_plan(nprob, hds, nrhs, 1, G);
  if (st != HSP_OK) return st;
  if ((st = check_tile(tile)) != HSP_OK) return st;
  if (!r_dev || !z_dev) return fail(HSP_EINVAL, "null vector arrays");
  if ((st = check_ws(G, ws, ws_bytes)) != HSP_OK) return st;
  group_bind(G, ws);
  return group_precond(G, r_dev, z_dev, tile, flags, S_(stream));
}

hsp_status hsp_solve_group(int nprob, const hsp_handle* hds, const int* nrhs, const void* const* b_dev,
                           void* const* u_dev, double tol, int maxit, int restart, int conj_transpose, int tile,
                           int flags, void* ws, size_t ws_bytes, int* iters, double* relres, void* stream) {
  Group G;
  hsp_status st = group_plan(nprob, hds, nrhs, restart, G);
  if (st != HSP_OK) return st;
  if ((st = check_tile(tile)) != HSP_OK) return st;
  if (!(tol > 0) || maxit < 1) return fail(HSP_EINVAL, "tol must be > 0 and maxit >= 1");
  if (!b_dev || !u_dev) return fail(HSP_EINVAL, "null vector arrays");
  if ((st = check_ws(G, ws, ws_bytes)) != HSP_OK) return st;
  group_bind(G, ws);
  return group_solve(G, b_dev, u_dev, tol, maxit, conj_transpose, tile, flags, iters, relres, S_(stream));
}

// ---- one problem, many right-hand sides (a group of one) -----------------

hsp_status hsp_batch_workspace_size(hsp_handle C, int nrhs, int restart, size_t* bytes) {
  if (!C || !bytes) return fail(HSP_EINVAL, "null argument");
  if (nrhs < 1 || restart < 1) return fail(HSP_EINVAL, "nrhs and restart must be >= 1");
  return hsp_group_workspace_size(1, &C, &nrhs, restart, bytes);
}

hsp_status hsp_apply_precond_batch(hsp_handle C, int nrhs, const void* r, void* z, int tile, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  if (nrhs < 0) return fail(HSP_EINVAL, "nrhs must be >= 0");
  hsp_status st = check_tile(tile);
  if (st != HSP_OK || nrhs == 0) return st;
  return hsp_apply_precond_group(1, &C, &nrhs, &r, &z, tile, 0, ws, ws_bytes, stream);
}

hsp_status hsp_apply_precond_batch_noalloc(hsp_handle C, int nrhs, const void* r, void* z, int tile,
                                           size_t* scratch_bytes, void* stream) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  if (nrhs < 0) return fail(HSP_EINVAL, "nrhs must be >= 0");
  hsp_status st = check_tile(tile);
  if (st != HSP_OK) return st;
  if (scratch_bytes) *scratch_bytes = kNoallocScratchBytes;
  if (nrhs == 0) return HSP_OK;
  if (!r || !z || r == z) return fail(HSP_EINVAL, "null or aliased vectors");
  Group G;
  if ((st = group_plan(1, &C, &nrhs, 1, G)) != HSP_OK) return st;
  if (G.total > kNoallocScratchBytes)
    return fail(HSP_ENOMEM, "batch needs " + std::to_string(G.total) + " bytes of scratch, more than the fixed " +
                                std::to_string(kNoallocScratchBytes) + " bytes: use fewer right-hand sides");
  void* ws = nullptr;
  if ((st = noalloc_scratch(&ws)) != HSP_OK) return st;
  group_bind(G, ws);
  const void* rr[1] = {r};
  void* zz[1] = {z};
  return group_precond(G, rr, zz, tile, 0, S_(stream), 0, 0, /*zero_by_kernel=*/true);
}

hsp_status hsp_tune_batch(hsp_handle C, int nrhs, int restart, void* ws, size_t ws_bytes, int* tile_out,
                          double* ms_out, void* stream) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  if (nrhs < 1) return fail(HSP_EINVAL, "nrhs must be >= 1");
  Group G;
  hsp_status st = group_plan(1, &C, &nrhs, restart, G);
  if (st != HSP_OK) return st;
  if ((st = check_ws(G, ws, ws_bytes)) != HSP_OK) return st;
  group_bind(G, ws);
  hipStream_t s = S_(stream);
  const Member& mb = G.mem[0];
  const size_t nf = (size_t)C->P.nf1 * C->P.nf2;
  // constant right-hand sides in the type the solver hands to the
  // preconditioner (its Krylov basis)
  cd* w = mptr<cd>(mb, mb.B.o_w);
  void* z = mb.ws + mb.B.o_Z;
  launch_fill(w, (size_t)nrhs * nf, mk<double>(1.0, 0.0), s);
  const void* r = w;
  if (G.v32) {
    cf* r32 = mptr<cf>(mb, mb.B.o_V);
    launch_convert<float, double>(w, r32, (size_t)nrhs * nf, 0, s);
    r = r32;
  }
  const void* rr[1] = {r};
  void* zz[1] = {z};
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
  for (int rb = 1; rb <= kMaxTile && err == hipSuccess && st == HSP_OK; rb *= 2) {
    st = group_precond(G, rr, zz, rb, 0, s, G.v32 ? 1 : 0, G.mixed ? 1 : 0);  // warm-up
    if (st != HSP_OK) break;
    err = hipEventRecord(e0, s);
    for (int rep = 0; rep < 2 && err == hipSuccess && st == HSP_OK; ++rep)
      st = group_precond(G, rr, zz, rb, 0, s, G.v32 ? 1 : 0, G.mixed ? 1 : 0);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && st == HSP_OK && 0.5 * ms < best_ms) {
      best_ms = 0.5 * ms;
      best = rb;
    }
  }
  C->prof.on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HSP_OK) return st;
  if (err != hipSuccess) return fail(HSP_EDEVICE, std::string("tuning: ") + hipGetErrorString(err));
  C->tuned_rb = best;
  C->tuned_nact = nrhs;
  if (tile_out) *tile_out = best;
  if (ms_out) *ms_out = best_ms;
  return HSP_OK;
}

hsp_status hsp_solve_batch(hsp_handle C, int nrhs, const void* b_in, void* u_out, double tol, int maxit, int restart,
                           int conj_transpose, int tile, void* ws, size_t ws_bytes, int* iters, double* relres,
                           void* stream) {
  if (!C) return fail(HSP_EINVAL, "null handle");
  if (nrhs < 0) return fail(HSP_EINVAL, "nrhs must be >= 0");
  if (restart < 1) return fail(HSP_EINVAL, "restart must be >= 1");
  hsp_status st = check_tile(tile);
  if (st != HSP_OK || nrhs == 0) return st;
  return hsp_solve_group(1, &C, &nrhs, &b_in, &u_out, tol, maxit, restart, conj_transpose, tile, 0, ws, ws_bytes,
                         iters, relres, stream);
}

}  // extern "C"
