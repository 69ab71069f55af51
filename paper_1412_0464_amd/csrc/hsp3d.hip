// Host side of the three-dimensional path: workspace planning, setup (PML
// profiles, PML-aware coarse mesh, coarse optimized 27-point FE medium,
// slab partition along x, slab operators with DD-PML and k continuation,
// dense-block factorization of every slab), the sweep of Table 3, the
// two-grid cycle of Sec. 4 and the component entry points.  The FGMRES of
// hsp_solve is shared with the 2-D path.
//
// Precision: slab factors, sweeps and smoothing in complex64 (the blocks are
// factored on the FP32 matrix cores), the fine residual, restriction input,
// FGMRES and solution in complex128 (HSP_MIXED; HSP_FP64 is refused in 3-D).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "d3.h"

namespace hsp {

struct D3Ctx {
  int m[3] = {0, 0, 0}, N[3] = {0, 0, 0};  // fine unknowns / cells per axis
  int two_grid = 0, fine_kind = 7;
  int mc[3] = {0, 0, 0};                   // coarse unknowns
  int dm[3] = {0, 0, 0};                   // DD-level unknowns
  std::vector<int> ifp[3];
  std::vector<char> ref[3];
  d3::Level3 fine{}, coarse{}, dd{};
  d3::Transfer3 tr{};
  std::vector<d3::Slab3> slabs_host;
  d3::Slab3* slabs_dev = nullptr;
  std::vector<int> nls;
  int n_max = 0, nl_max = 0;
  cf* factors = nullptr;
  std::vector<double> stage_bytes;  // algorithmic bytes per stage
  hipError_t launch_err = hipSuccess;  // first failed launch of a stage (reported by the next call)
  // workspace offsets
  size_t o_fA[3], o_fB[3], o_ib[3], o_k2n, o_fk2c, o_fcoef;
  size_t o_cA[3], o_cB[3], o_ck2c, o_ccoef;
  size_t o_avx[3], o_avw[3];
  size_t o_r[3], o_rw[3], o_p[3], o_pw[3];
  size_t o_slabA, o_slabB, o_xmap, o_slabs, o_fac, o_setup, o_status, o_growth, o_tasks;
  size_t o_swf, o_swg, o_swu, o_bufs, o_fs, o_ys;
  size_t o_tgx0, o_tgx1, o_tgres, o_tgrc, o_tgec, o_cvin, o_cvout;
  size_t n_slabA = 0, n_xmap = 0, n_fac = 0, n_tasks = 0;
  // nested-dissection factorization (slab_factor HSP_SLAB_ND)
  int slab_factor = HSP_SLAB_BLOCK;
  d3::NDPlan ndp;
  std::vector<d3::NDSizes> ndz;        // per slab
  std::vector<d3::NDLevelHost> ndlv;   // per level
  d3::NDSolve nds{};
  size_t nd_njobs = 0, nd_nitems = 0, nd_u_stride = 0, nd_nmaps = 0;
  size_t nd_buf[2] = {0, 0};           // complex64 elements of the two level buffers
  size_t nd_piv = 0, nd_brow = 0, nd_spr = 0;  // Gauss-Jordan scratch of the largest level
  size_t o_ndgeom = 0, o_ndpts = 0, o_ndlmap = 0, o_ndchmap = 0, o_ndcmap = 0, o_ndfr = 0, o_nditems = 0,
         o_ndtab = 0, o_ndU = 0, o_ndmaps = 0;
  size_t nf() const { return (size_t)m[0] * m[1] * m[2]; }
  size_t nd() const { return (size_t)dm[0] * dm[1] * dm[2]; }
};

void destroy_d3(D3Ctx* d) { delete d; }

namespace {

constexpr int kMaxBlock3 = 1536;  // unknowns per y-plane of a slab (panel rows: 1024 in registers, 512 in LDS)
// zeroed tail of the factor array: the substitutions read whole 128-entry
// groups per lane, past the end of the last row
constexpr size_t kFacTail = 128 * 24;

inline size_t blk_elems(int n) { return (size_t)2 * n * n + (size_t)n * (n + (n & 1)); }

hsp_status validate3(const hsp_grid* g, int J, const hsp_options* o) {
  if (!g || !o) return fail(HSP_EINVAL, "null grid or options");
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1) return fail(HSP_EINVAL, "n must be >= 1");
    if (g->pml[a] < 0) return fail(HSP_EINVAL, "pml must be >= 0");
  }
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(HSP_EINVAL, "h must be positive and finite");
  if (J < 1) return fail(HSP_EINVAL, "J must be >= 1");
  if (o->w_dd < 1) return fail(HSP_EINVAL, "w_dd must be >= 1");
  if (o->nu < 0) return fail(HSP_EINVAL, "nu must be >= 0");
  if (o->restart < 1) return fail(HSP_EINVAL, "restart must be >= 1");
  if (o->fine_stencil != 7 && o->fine_stencil != 27)
    return fail(HSP_EINVAL, "fine_stencil must be 7 or 27 in three dimensions");
  if (o->sweep != HSP_SWEEP_X && o->sweep != HSP_SWEEP_UD && o->sweep != HSP_SWEEP_NX)
    return fail(HSP_EINVAL, "bad sweep");
  if (o->precision != HSP_MIXED)
    return fail(HSP_EINVAL, "the 3-D path factors its slabs in complex64: precision must be HSP_MIXED");
  if (o->krylov_fp32 != 0) return fail(HSP_EINVAL, "krylov_fp32 applies to the 2-D batched solvers only");
  if (!std::isfinite(o->omega_jac)) return fail(HSP_EINVAL, "bad omega_jac");
  if (g->sponge != 0) return fail(HSP_EINVAL, "sponge layers are implemented for 2-D problems");
  if (o->slab_factor != HSP_SLAB_AUTO && o->slab_factor != HSP_SLAB_BLOCK && o->slab_factor != HSP_SLAB_ND)
    return fail(HSP_EINVAL, "bad slab_factor");
  return HSP_OK;
}

// Bytes of the setup scratch of the nested-dissection factorization.
size_t nd_coef_elems(const D3Ctx& D, int J) {
  size_t n = 0;
  for (int j = 0; j < J; ++j) n += (size_t)D.nls[j] * D.dm[2] * D.dm[1] * 27;
  return n;
}
size_t nd_setup_bytes(const D3Ctx& D, int J) {
  return (D.nd_buf[0] + D.nd_buf[1] + D.nd_brow + D.nd_spr + nd_coef_elems(D, J)) * sizeof(cf) +
         2 * D.nd_piv * sizeof(int) + D.nd_njobs * (sizeof(d3::NDJob) + sizeof(d3::GJob)) +
         (size_t)J * (2 * sizeof(double) + sizeof(size_t)) + 10 * 256;
}

// The dissection, the per-slab sizes, the level table and the scratch sizes.
hsp_status plan_nd(D3Ctx& D, int J) {
  std::string why;
  if (!d3::nd_plan(D.dm[1], D.dm[2], D.ndp, &why)) return fail(HSP_EINVAL, "internal: " + why);
  const d3::NDPlan& np = D.ndp;
  D.ndz.resize(J);
  D.n_fac = 0;
  D.nd_u_stride = 0;
  D.nd_nitems = 0;
  for (int j = 0; j < J; ++j) {
    D.ndz[j] = d3::nd_sizes(np, D.nls[j]);
    const d3::NDSizes& z = D.ndz[j];
    if (z.s_max > d3::kGJMaxPivots || z.nf_max > d3::kNDMaxFront)
      return fail(HSP_EINVAL, "nested-dissection fronts of " + std::to_string(z.nf_max) + " unknowns (" +
                                  std::to_string(z.s_max) + " pivots) exceed " + std::to_string(d3::kNDMaxFront) +
                                  " (" + std::to_string(d3::kGJMaxPivots) + "): use more slabs or HSP_SLAB_BLOCK");
    D.n_fac += z.factor;
    D.nd_u_stride = std::max(D.nd_u_stride, z.update);
  }
  D.nd_u_stride = (D.nd_u_stride + 63) / 64 * 64;
  D.ndlv.assign(np.depth, d3::NDLevelHost());
  D.nd_njobs = 0;
  D.nd_buf[0] = D.nd_buf[1] = 0;
  D.nd_piv = D.nd_brow = D.nd_spr = 0;
  D.nd_nmaps = 0;
  for (int L = 0; L < np.depth; ++L) {
    d3::NDLevelHost& l = D.ndlv[L];
    l.first_job = (int)D.nd_njobs;
    l.njobs = J * (int)np.levels[L].size();
    D.nd_njobs += l.njobs;
    for (int j = 0; j < J; ++j)
      for (int f : np.levels[L]) {
        const d3::NDGeom& g = np.fronts[f];
        l.s_max = std::max(l.s_max, g.ns * D.nls[j]);
        l.b_max = std::max(l.b_max, g.nb * D.nls[j]);
        l.nf_max = std::max(l.nf_max, (g.ns + g.nb) * D.nls[j]);
      }
    d3::nd_row_shape(l.s_max, &l.fwd_g, &l.fwd_np);
    d3::nd_row_shape(l.b_max, &l.bwd_g, &l.bwd_np);
    size_t buf = 0, piv = 0, brow = 0;
    for (int j = 0; j < J; ++j) {
      int fi = 0, bi = 0;
      for (int f : np.levels[L]) {
        const d3::NDGeom& g = np.fronts[f];
        const int s = g.ns * D.nls[j], b = g.nb * D.nls[j], nf = s + b;
        buf += (size_t)nf * nf;
        piv += s;
        brow += (size_t)32 * nf;
        fi += (nf + l.fwd_rows() - 1) / l.fwd_rows();
        if (b > 0) bi += (s + l.bwd_rows() - 1) / l.bwd_rows();
        D.nd_nmaps += (size_t)s + b + 2 * (size_t)nf;
      }
      l.fwd_items = std::max(l.fwd_items, fi);
      l.bwd_items = std::max(l.bwd_items, bi);
      D.nd_nitems += fi + bi;
    }
    D.nd_buf[L & 1] = std::max(D.nd_buf[L & 1], buf);
    D.nd_piv = std::max(D.nd_piv, piv);
    D.nd_brow = std::max(D.nd_brow, brow);
    D.nd_spr = std::max(D.nd_spr, (size_t)l.njobs * 32 * 32);
  }
  return HSP_OK;
}

// Sizes and the workspace layout (fills the FGMRES part of C->P as well).
hsp_status plan3(const hsp_grid* g, int J, const hsp_options* o, D3Ctx& D, Plan& P, size_t* total) {
  hsp_status st = validate3(g, J, o);
  if (st != HSP_OK) return st;
  for (int a = 0; a < 3; ++a) {
    D.N[a] = g->n[a] + 1 + 2 * g->pml[a];
    D.m[a] = D.N[a] - 1;
  }
  D.two_grid = o->two_grid ? 1 : 0;
  D.fine_kind = o->fine_stencil;
  if (D.two_grid) {
    for (int a = 0; a < 3; ++a) {
      if ((D.N[a] - 2 * g->pml[a]) % 2 != 0 || D.N[a] - 2 * g->pml[a] < 2)
        return fail(HSP_EINVAL, "two-grid needs an even, positive interior cell count per axis");
      coarse_map(D.N[a], g->pml[a], D.ifp[a], D.ref[a]);
      D.mc[a] = (int)D.ifp[a].size() - 2;
      D.dm[a] = D.mc[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) D.dm[a] = D.m[a];
  }
  const int w_outer = g->pml[0];
  if (D.dm[0] - 2 * w_outer < J) return fail(HSP_EINVAL, "too many slabs for the interior layers");
  P.beta = partition(D.dm[0], w_outer, J);
  P.bt = P.beta;
  for (int j = 1; j < J; ++j) P.bt[j] = P.beta[j] - 1;
  P.x0.resize(J);
  P.x1.resize(J);
  D.nls.resize(J);
  D.nl_max = 0;
  D.n_max = 0;
  for (int j = 1; j <= J; ++j) {
    if (P.beta[j] - P.beta[j - 1] < 3) return fail(HSP_EINVAL, "a core is thinner than 3 layers");
    P.x0[j - 1] = (j == 1) ? 1 : P.beta[j - 1] - o->w_dd;
    P.x1[j - 1] = (j == J) ? D.dm[0] : P.beta[j] + o->w_dd;
    if (P.x0[j - 1] < 1 || P.x1[j - 1] > D.dm[0]) return fail(HSP_EINVAL, "DD-PML layers leave the domain");
    const int nl = P.x1[j - 1] - P.x0[j - 1] + 1;
    D.nls[j - 1] = nl;
    D.nl_max = std::max(D.nl_max, nl);
    D.n_max = std::max(D.n_max, nl * D.dm[2]);
  }
  D.slab_factor = (o->slab_factor == HSP_SLAB_BLOCK) ? HSP_SLAB_BLOCK : HSP_SLAB_ND;
  if (D.slab_factor == HSP_SLAB_BLOCK && D.n_max > kMaxBlock3)
    return fail(HSP_EINVAL, "slab planes of " + std::to_string(D.n_max) + " unknowns exceed " +
                                std::to_string(kMaxBlock3) + ": use more slabs or a smaller z extent");
  if (D.slab_factor == HSP_SLAB_ND) {
    st = plan_nd(D, J);
    if (st != HSP_OK) return st;
  }
  st = sweep_shape(J, o, &P.nbuf, &P.maxtask);
  if (st != HSP_OK) return st;
  P.nl_max = D.nl_max;
  P.two_grid = D.two_grid;
  P.tsize = sizeof(cf);
  P.m = o->restart;
  P.nf1 = D.m[0];
  P.nf2 = D.m[1] * D.m[2];
  P.dd_n1 = D.dm[0];
  P.dd_n2 = D.dm[1] * D.dm[2];

  Carver c;
  const size_t nf = D.nf(), nd = D.nd();
  for (int a = 0; a < 3; ++a) {
    D.o_fA[a] = c.take((D.N[a] + 1) * sizeof(cd));
    D.o_fB[a] = c.take((D.N[a] + 1) * sizeof(cd));
    D.o_ib[a] = c.take((D.N[a] + 1) * sizeof(cd));
  }
  D.o_k2n = c.take(nf * sizeof(double));
  const size_t nfc = (size_t)D.N[0] * D.N[1] * D.N[2];
  if (D.fine_kind == 27) {
    D.o_fk2c = c.take(nfc * sizeof(double));
    D.o_fcoef = c.take(nfc * 5 * sizeof(double));
  }
  int nav[3];
  for (int a = 0; a < 3; ++a) nav[a] = std::max(D.N[a], D.mc[a] + 1);
  for (int a = 0; a < 3; ++a) {
    D.o_avx[a] = c.take(nav[a] * sizeof(int));
    D.o_avw[a] = c.take((size_t)nav[a] * 3 * sizeof(double));
  }
  if (D.two_grid) {
    const size_t ncc = (size_t)(D.mc[0] + 1) * (D.mc[1] + 1) * (D.mc[2] + 1);
    for (int a = 0; a < 3; ++a) {
      D.o_cA[a] = c.take((D.mc[a] + 1) * sizeof(cd));
      D.o_cB[a] = c.take((D.mc[a] + 1) * sizeof(cd));
      D.o_r[a] = c.take((size_t)D.mc[a] * 3 * sizeof(int));
      D.o_rw[a] = c.take((size_t)D.mc[a] * 3 * sizeof(double));
      D.o_p[a] = c.take((size_t)D.m[a] * 2 * sizeof(int));
      D.o_pw[a] = c.take((size_t)D.m[a] * 2 * sizeof(double));
    }
    D.o_ck2c = c.take(ncc * sizeof(double));
    D.o_ccoef = c.take(ncc * 5 * sizeof(double));
  }
  D.n_slabA = D.n_xmap = 0;
  if (D.slab_factor == HSP_SLAB_BLOCK) D.n_fac = 0;
  for (int j = 0; j < J; ++j) {
    D.n_slabA += D.nls[j] + 2;
    D.n_xmap += D.nls[j] + 1;
    if (D.slab_factor == HSP_SLAB_BLOCK) D.n_fac += blk_elems(D.nls[j] * D.dm[2]) * D.dm[1];
  }
  D.o_slabA = c.take(D.n_slabA * sizeof(cd));
  D.o_slabB = c.take(D.n_slabA * sizeof(cd));
  D.o_xmap = c.take(D.n_xmap * sizeof(int));
  D.o_slabs = c.take(J * sizeof(d3::Slab3));
  D.o_fac = c.take((D.n_fac + kFacTail) * sizeof(cf));
  D.o_setup = c.take(D.slab_factor == HSP_SLAB_ND ? nd_setup_bytes(D, J) : d3::setup3_scratch_bytes(J, D.n_max));
  if (D.slab_factor == HSP_SLAB_ND) {
    const d3::NDPlan& np = D.ndp;
    D.o_ndgeom = c.take(np.fronts.size() * sizeof(d3::NDGeom));
    D.o_ndpts = c.take(np.pts.size() * sizeof(int));
    D.o_ndlmap = c.take(np.lmap.size() * sizeof(int));
    D.o_ndchmap = c.take(std::max<size_t>(np.chmap.size(), 1) * sizeof(int));
    D.o_ndcmap = c.take(std::max<size_t>(np.cmap.size(), 1) * sizeof(int));
    D.o_ndfr = c.take((size_t)J * np.fronts.size() * sizeof(d3::NDFront));
    D.o_nditems = c.take(std::max<size_t>(D.nd_nitems, 1) * sizeof(int2));
    D.o_ndtab = c.take((size_t)J * np.depth * 4 * sizeof(int));
    D.o_ndU = c.take((size_t)P.maxtask * D.nd_u_stride * sizeof(cf));
    D.o_ndmaps = c.take(D.nd_nmaps * sizeof(int));
  }
  D.o_status = c.take(64);
  D.o_growth = c.take((size_t)J * sizeof(double));
  D.n_tasks = 2 * (size_t)J + 8;
  D.o_tasks = c.take(D.n_tasks * sizeof(TaskDev));
  const size_t pl = (size_t)D.dm[1] * D.dm[2];
  const size_t slot = (size_t)D.dm[1] * (D.n_max + (D.n_max & 1));
  D.o_swf = c.take(nd * sizeof(cf));
  D.o_swg = c.take(nd * sizeof(cf));
  D.o_swu = c.take(nd * sizeof(cf));
  D.o_bufs = c.take((size_t)P.nbuf * 2 * pl * sizeof(cf));
  D.o_fs = c.take((size_t)P.maxtask * slot * sizeof(cf));
  D.o_ys = c.take((size_t)P.maxtask * slot * sizeof(cf));
  D.o_tgx0 = c.take(nf * sizeof(cf));
  D.o_tgx1 = c.take(nf * sizeof(cf));
  if (D.two_grid) {
    D.o_tgres = c.take(nf * sizeof(cd));
    D.o_tgrc = c.take(nd * sizeof(cf));
    D.o_tgec = c.take(nd * sizeof(cf));
  }
  D.o_cvin = c.take(std::max(nf, nd) * sizeof(cd));
  D.o_cvout = c.take(std::max(nf, nd) * sizeof(cd));
  // FGMRES of hsp_solve
  P.o_V = c.take((size_t)(2 * P.m + 1) * nf * sizeof(cd));
  P.o_Z = P.o_V + (size_t)(P.m + 1) * nf * sizeof(cd);
  P.o_w = c.take(nf * sizeof(cd));
  P.o_bconj = c.take(nf * sizeof(cd));
  P.o_part = c.take((size_t)kPartBlocks * (P.m + 2) * sizeof(cd));
  P.o_hbuf = c.take((size_t)(2 * (P.m + 2) + 2) * sizeof(cd));
  P.o_stats = c.take(8 * sizeof(double));
  P.total = c.off + 256;
  *total = P.total;
  return HSP_OK;
}

// Per-axis arrays of a level (see Level3): kind 7 at half nodes and nodes,
// kind 27 per cell.
void axis_arrays3(const AxisH& ax, int kind, double omega, std::vector<cd>& A, std::vector<cd>& B) {
  const int N = (int)ax.x.size() - 1;
  if (kind == 7) {
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

// Restriction maps: coarse unknown I gathers fine unknowns with weights
// 1 (its own node) and 1/2 (the midpoints of its refined cells).
void restrict_maps(const std::vector<int>& ifp, const std::vector<char>& ref, int nc, std::vector<int>& ri,
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
}

// Prolongation maps: tent interpolation, no coarsening in the PML cells.
void prolong_maps(const std::vector<int>& ifp, const std::vector<char>& ref, int nf_, std::vector<int>& pi,
                  std::vector<double>& pw) {
  pi.assign(2 * nf_, -1);
  pw.assign(2 * nf_, 0.0);
  const int Nc = (int)ifp.size() - 1;
  for (int I = 0; I <= Nc; ++I) {
    const int F = ifp[I];
    if (F >= 1 && F <= nf_ && I >= 1 && I <= Nc - 1) pi[2 * (F - 1)] = I - 1, pw[2 * (F - 1)] = 1.0;
    if (I < Nc && ref[I]) {
      const int f = F + 1;
      int q = 0;
      if (I >= 1) pi[2 * (f - 1) + q] = I - 1, pw[2 * (f - 1) + q] = 0.5, ++q;
      if (I + 1 <= Nc - 1) pi[2 * (f - 1) + q] = I, pw[2 * (f - 1) + q] = 0.5, ++q;
    }
  }
}

void run_sweep3(hsp_ctx* C, const cf* f, cf* u, hipStream_t s) {
  D3Ctx& D = *C->d3;
  const size_t nd = D.nd();
  cf* g = C->at<float>(D.o_swg);
  launch_zero<float>(u, nd, s);
  for (size_t k = 0; k < C->stages.size(); ++k) {
    const Stage& st = C->stages[k];
    if (st.residual) {
      prof_begin(C, HSP_PROF_COARSE, s);
      d3::launch_stencil3<float, float, float, float>(D.dd, 1, u, f, g, 0.0, s);
      prof_end(C, HSP_PROF_COARSE, s, (double)nd * 3.0 * sizeof(cf));
      continue;
    }
    d3::Stage3 S;
    S.tasks = C->tasks_dev + st.first;
    S.slabs = D.slabs_dev;
    S.G = D.dd;
    S.ntasks = st.ntasks;
    S.n_max = D.n_max;
    S.nl_max = D.nl_max;
    S.f = f;
    S.g = g;
    S.u = u;
    S.bufs = C->at<float>(D.o_bufs);
    S.fs = C->at<float>(D.o_fs);
    S.ys = C->at<float>(D.o_ys);
    S.factors = D.factors;
    S.nd = D.slab_factor == HSP_SLAB_ND ? &D.nds : nullptr;
    S.nd_lv = &D.ndlv;
    prof_begin(C, HSP_PROF_STAGE, s);
    const hipError_t e = d3::launch_stage3(S, s);
    if (e != hipSuccess && D.launch_err == hipSuccess) D.launch_err = e;
    prof_end(C, HSP_PROF_STAGE, s, D.stage_bytes[k]);
  }
}

}  // namespace

hsp_status d3_workspace_size(const hsp_grid* g, int J, const hsp_options* o, size_t* bytes) {
  D3Ctx D;
  Plan P;
  return plan3(g, J, o, D, P, bytes);
}

hsp_status d3_setup(const double* c_dev, double omega, const hsp_grid* grid, int J, const hsp_options* opt,
                    void* ws_dev, size_t ws_bytes, hipStream_t s, hsp_ctx** out) {
  hsp_ctx* C = new hsp_ctx();
  C->d3 = new D3Ctx();
  D3Ctx& D = *C->d3;
  Plan& P = C->P;
  size_t total = 0;
  hsp_status st = plan3(grid, J, opt, D, P, &total);
  auto cleanup = [&](hsp_status e) {
    delete C;
    return e;
  };
  if (st != HSP_OK) return cleanup(st);
  if (ws_bytes < total) return cleanup(fail(HSP_ENOMEM, "workspace too small: need " + std::to_string(total) + " bytes"));
  C->grid = *grid;
  C->opt = *opt;
  C->J = J;
  C->omega = omega;
  C->h = grid->h;
  C->ws = reinterpret_cast<char*>(ws_dev);
#define CHK(expr)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  const size_t nf = D.nf();
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

  std::vector<hipError_t> errs;
  std::vector<std::vector<char>> keep;  // host buffers alive until the final sync
  auto up = [&](size_t off, const void* src, size_t bytes) {
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    errs.push_back(hipMemcpyAsync(C->ws + off, keep.back().data(), bytes, hipMemcpyHostToDevice, s));
  };

  // fine axes and level
  AxisH fa[3];
  for (int a = 0; a < 3; ++a) {
    AxisH& ax = fa[a];
    const int N = D.N[a], w = grid->pml[a];
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
    std::vector<cd> A, B;
    axis_arrays3(ax, D.fine_kind, omega, A, B);
    up(D.o_fA[a], A.data(), A.size() * sizeof(cd));
    up(D.o_fB[a], B.data(), B.size() * sizeof(cd));
    std::vector<cd> ib(N + 1);
    for (int i = 0; i <= N; ++i) ib[i] = to_cd(1.0 / alpha_of(ax.sig(ax.x[i]), omega));
    up(D.o_ib[a], ib.data(), ib.size() * sizeof(cd));
  }
  launch_k2_nodes(c_dev, nf, omega, C->raw<double>(D.o_k2n), s);
  D.fine.kind = D.fine_kind;
  for (int a = 0; a < 3; ++a) {
    D.fine.A[a] = C->at<double>(D.o_fA[a]);
    D.fine.B[a] = C->at<double>(D.o_fB[a]);
  }
  D.fine.m1 = D.m[0];
  D.fine.m2 = D.m[1];
  D.fine.m3 = D.m[2];
  D.fine.hs = h;
  D.fine.xmap = nullptr;
  auto upload_avg = [&](int a, const std::vector<int>& x0, const std::vector<double>& w) {
    up(D.o_avx[a], x0.data(), x0.size() * sizeof(int));
    up(D.o_avw[a], w.data(), w.size() * sizeof(double));
  };
  auto avg_ptrs = [&](const int* (&x0)[3], const double* (&w)[3]) {
    for (int a = 0; a < 3; ++a) {
      x0[a] = C->raw<int>(D.o_avx[a]);
      w[a] = C->raw<double>(D.o_avw[a]);
    }
  };
  if (D.fine_kind == 7) {
    D.fine.k2 = C->raw<double>(D.o_k2n);
    D.fine.coef = nullptr;
  } else {
    // cell k^2 = mean of the 8 corner nodes; Table (b) at the fine 1/G
    for (int a = 0; a < 3; ++a) {
      std::vector<int> x0(D.N[a]);
      std::vector<double> w(3 * D.N[a], 0.0);
      for (int p = 0; p < D.N[a]; ++p) x0[p] = p, w[3 * p] = w[3 * p + 1] = 0.5;
      upload_avg(a, x0, w);
    }
    const int* x0p[3];
    const double* wp[3];
    avg_ptrs(x0p, wp);
    d3::launch_cell_average3(C->raw<double>(D.o_k2n), D.m, x0p, wp, D.N, C->raw<double>(D.o_fk2c), s);
    d3::launch_cell_coefs3(C->raw<double>(D.o_fk2c), (size_t)D.N[0] * D.N[1] * D.N[2], h,
                           C->raw<double>(D.o_fcoef), s);
    D.fine.k2 = C->raw<double>(D.o_fk2c);
    D.fine.coef = C->raw<double>(D.o_fcoef);
    CHK(hipStreamSynchronize(s));  // the averaging arrays are reused below
  }

  // DD level
  AxisH da[3];
  if (D.two_grid) {
    int ncell[3];
    for (int a = 0; a < 3; ++a) {
      da[a].x.resize(D.ifp[a].size());
      for (size_t i = 0; i < D.ifp[a].size(); ++i) da[a].x[i] = fa[a].x[D.ifp[a][i]];
      da[a].sig = fa[a].sig;
      da[a].h_nom = 2.0 * h;
      std::vector<cd> A, B;
      axis_arrays3(da[a], 27, omega, A, B);
      up(D.o_cA[a], A.data(), A.size() * sizeof(cd));
      up(D.o_cB[a], B.data(), B.size() * sizeof(cd));
      // coarse cell k^2: (1/2, 1/2) on unrefined, (1/4, 1/2, 1/4) on refined cells
      ncell[a] = D.mc[a] + 1;
      std::vector<int> x0(ncell[a]);
      std::vector<double> w(3 * ncell[a], 0.0);
      for (int p = 0; p < ncell[a]; ++p) {
        x0[p] = D.ifp[a][p];
        if (D.ref[a][p]) {
          w[3 * p] = 0.25;
          w[3 * p + 1] = 0.5;
          w[3 * p + 2] = 0.25;
        } else {
          w[3 * p] = w[3 * p + 1] = 0.5;
        }
      }
      upload_avg(a, x0, w);
      std::vector<int> ri;
      std::vector<double> rw;
      restrict_maps(D.ifp[a], D.ref[a], D.mc[a], ri, rw);
      up(D.o_r[a], ri.data(), ri.size() * sizeof(int));
      up(D.o_rw[a], rw.data(), rw.size() * sizeof(double));
      prolong_maps(D.ifp[a], D.ref[a], D.m[a], ri, rw);
      up(D.o_p[a], ri.data(), ri.size() * sizeof(int));
      up(D.o_pw[a], rw.data(), rw.size() * sizeof(double));
    }
    const int* x0p[3];
    const double* wp[3];
    avg_ptrs(x0p, wp);
    d3::launch_cell_average3(C->raw<double>(D.o_k2n), D.m, x0p, wp, ncell, C->raw<double>(D.o_ck2c), s);
    d3::launch_cell_coefs3(C->raw<double>(D.o_ck2c), (size_t)ncell[0] * ncell[1] * ncell[2], 2.0 * h,
                           C->raw<double>(D.o_ccoef), s);
    D.coarse.kind = 27;
    for (int a = 0; a < 3; ++a) {
      D.coarse.A[a] = C->at<double>(D.o_cA[a]);
      D.coarse.B[a] = C->at<double>(D.o_cB[a]);
      D.tr.nf[a] = D.m[a];
      D.tr.nc[a] = D.mc[a];
      D.tr.r[a] = C->raw<int>(D.o_r[a]);
      D.tr.rw[a] = C->raw<double>(D.o_rw[a]);
      D.tr.p[a] = C->raw<int>(D.o_p[a]);
      D.tr.pw[a] = C->raw<double>(D.o_pw[a]);
    }
    D.coarse.m1 = D.mc[0];
    D.coarse.m2 = D.mc[1];
    D.coarse.m3 = D.mc[2];
    D.coarse.hs = 0;
    D.coarse.k2 = C->raw<double>(D.o_ck2c);
    D.coarse.coef = C->raw<double>(D.o_ccoef);
    D.coarse.xmap = nullptr;
    D.dd = D.coarse;
  } else {
    for (int a = 0; a < 3; ++a) da[a] = fa[a];
    D.dd = D.fine;
  }

  // slabs along x on the DD level
  {
    const auto& be = P.beta;
    const int kind = D.dd.kind;
    const double d = opt->w_dd * da[0].h_nom;
    const double Cdd = S_dd * C->c_pml / (d * d * d);
    std::vector<cd> SA(D.n_slabA, mk<double>(0, 0)), SB(D.n_slabA, mk<double>(0, 0));
    std::vector<int> XM(D.n_xmap, 0);
    size_t oA = 0, oM = 0, oF = 0;
    D.slabs_host.resize(J);
    const int ncell = D.dm[0] + 1;
    const AxisH& dx = da[0];
    for (int j = 1; j <= J; ++j) {
      const int x0 = P.x0[j - 1], x1 = P.x1[j - 1], nl = x1 - x0 + 1;
      const Sigma gs = dx.sig;
      const bool hasL = j > 1, hasR = j < J;
      const double bl = hasL ? 0.5 * (dx.x[be[j - 1] - 1] + dx.x[be[j - 1]]) : 0.0;
      const double br = hasR ? 0.5 * (dx.x[be[j]] + dx.x[be[j] + 1]) : 0.0;
      auto sig = [&](double x) {
        if (hasL && x < bl) return Cdd * (bl - x) * (bl - x);
        if (hasR && x > br) return Cdd * (x - br) * (x - br);
        return gs(x);
      };
      auto gxn = [&](int lnode) { return dx.x[x0 - 1 + lnode]; };
      if (kind == 7) {
        for (int p = 0; p <= nl; ++p) SA[oA + p] = to_cd(alpha_of(sig(0.5 * (gxn(p) + gxn(p + 1))), omega));
        for (int i = 0; i <= nl + 1; ++i) SB[oA + i] = to_cd(1.0 / alpha_of(sig(gxn(i)), omega));
        const int lo = hasL ? be[j - 1] : 1, hi = hasR ? be[j] : D.dm[0];
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
      d3::Slab3 sd;
      sd.x0 = x0;
      sd.nl = nl;
      sd.n = nl * D.dm[2];
      sd.op = D.dd;
      sd.op.m1 = nl;
      sd.op.A[0] = C->at<double>(D.o_slabA) + oA;
      sd.op.B[0] = C->at<double>(D.o_slabB) + oA;
      sd.op.xmap = C->raw<int>(D.o_xmap) + oM;
      sd.fac_off = oF;
      D.slabs_host[j - 1] = sd;
      oA += nl + 2;
      oM += nl + 1;
      oF += blk_elems(sd.n) * D.dm[1];
    }
    up(D.o_slabA, SA.data(), SA.size() * sizeof(cd));
    up(D.o_slabB, SB.data(), SB.size() * sizeof(cd));
    up(D.o_xmap, XM.data(), XM.size() * sizeof(int));
    up(D.o_slabs, D.slabs_host.data(), J * sizeof(d3::Slab3));
    D.slabs_dev = C->raw<d3::Slab3>(D.o_slabs);
    D.factors = C->at<float>(D.o_fac);
  }
  build_schedule(C);
  if (C->tasks_host.size() + 1 > D.n_tasks) return cleanup(fail(HSP_EINVAL, "internal: schedule too long"));
  up(D.o_tasks, C->tasks_host.data(), C->tasks_host.size() * sizeof(TaskDev));
  C->tasks_dev = C->raw<TaskDev>(D.o_tasks);
  // algorithmic bytes per stage: the factor blocks W_t and E_t once, the
  // gathered right-hand side, the u read-modify-write and the transmission
  // layers (complex64)
  D.stage_bytes.assign(C->stages.size(), 0.0);
  for (size_t k = 0; k < C->stages.size(); ++k) {
    const Stage& sg = C->stages[k];
    double b = 0;
    for (int q = 0; q < sg.ntasks; ++q) {
      const TaskDev& t = C->tasks_host[sg.first + q];
      const double n = (double)D.nls[t.slab] * D.dm[2], pl = (double)D.dm[1] * D.dm[2];
      if (D.slab_factor == HSP_SLAB_ND)
        b += (double)D.ndz[t.slab].factor * sizeof(cf);
      else
        b += D.dm[1] * 3.0 * n * n * sizeof(cf);
      b += pl * ((t.b - t.a) + 2.0 * (t.bt - t.at) + 2.0 * (t.t1 + t.t2 + t.t3 + t.t4)) * sizeof(cf);
    }
    D.stage_bytes[k] = b;
  }
  for (hipError_t e : errs)
    if (e != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string("upload: ") + hipGetErrorString(e)));

  // factorization of every slab
  std::vector<double> hg(J);
  int hstat = 0;
  if (D.slab_factor == HSP_SLAB_ND) {
    const d3::NDPlan& np = D.ndp;
    const int nfr = (int)np.fronts.size();
    up(D.o_ndgeom, np.fronts.data(), nfr * sizeof(d3::NDGeom));
    up(D.o_ndpts, np.pts.data(), np.pts.size() * sizeof(int));
    up(D.o_ndlmap, np.lmap.data(), np.lmap.size() * sizeof(int));
    if (!np.chmap.empty()) up(D.o_ndchmap, np.chmap.data(), np.chmap.size() * sizeof(int));
    if (!np.cmap.empty()) up(D.o_ndcmap, np.cmap.data(), np.cmap.size() * sizeof(int));
    // setup scratch: two level buffers, Gauss-Jordan scratch, job tables, growth
    Carver sc;
    char* base = C->ws + D.o_setup;
    cf* buf[2];
    buf[0] = reinterpret_cast<cf*>(base + sc.take(D.nd_buf[0] * sizeof(cf)));
    buf[1] = reinterpret_cast<cf*>(base + sc.take(D.nd_buf[1] * sizeof(cf)));
    cf* brow = reinterpret_cast<cf*>(base + sc.take(D.nd_brow * sizeof(cf)));
    cf* spr = reinterpret_cast<cf*>(base + sc.take(D.nd_spr * sizeof(cf)));
    int* piv = reinterpret_cast<int*>(base + sc.take(D.nd_piv * sizeof(int)));
    int* col = reinterpret_cast<int*>(base + sc.take(D.nd_piv * sizeof(int)));
    d3::NDJob* jobs_dev = reinterpret_cast<d3::NDJob*>(base + sc.take(D.nd_njobs * sizeof(d3::NDJob)));
    d3::GJob* gjobs_dev = reinterpret_cast<d3::GJob*>(base + sc.take(D.nd_njobs * sizeof(d3::GJob)));
    double* gmax = reinterpret_cast<double*>(base + sc.take((size_t)J * 2 * sizeof(double)));
    cf* coefs = reinterpret_cast<cf*>(base + sc.take(nd_coef_elems(D, J) * sizeof(cf)));
    size_t* coef_off = reinterpret_cast<size_t*>(base + sc.take((size_t)J * sizeof(size_t)));
    if (sc.off > nd_setup_bytes(D, J)) return cleanup(fail(HSP_EINVAL, "internal: nested-dissection scratch"));
    // per slab and front: factor and update offsets, front matrices
    std::vector<d3::NDFront> fr((size_t)J * nfr);
    size_t ofac = 0;
    for (int j = 0; j < J; ++j) {
      size_t ou = 0;
      for (int f = 0; f < nfr; ++f) {
        const d3::NDGeom& g = np.fronts[f];
        const size_t sv = (size_t)g.ns * D.nls[j], bv = (size_t)g.nb * D.nls[j];
        d3::NDFront& e = fr[(size_t)j * nfr + f];
        e.gn = ofac;
        ofac += (sv + bv) * (sv + (sv & 1));
        e.e = ofac;
        ofac += sv * (bv + (bv & 1));
        e.u = ou;
        ou += bv;
        e.F = nullptr;
      }
    }
    // gather maps: slab-layout positions of the separator and ring unknowns,
    // the children's update-vector entries of every front unknown
    std::vector<int> maps;
    maps.reserve(D.nd_nmaps);
    {
      const int ldv = D.n_max + (D.n_max & 1), m3 = D.dm[2];
      for (int j = 0; j < J; ++j) {
        const int nl = D.nls[j];
        for (int f = 0; f < nfr; ++f) {
          const d3::NDGeom& g = np.fronts[f];
          const int sv = g.ns * nl, bv = g.nb * nl, nf = sv + bv;
          fr[(size_t)j * nfr + f].m = maps.size();
          auto var = [&](int v, int& xl, int& Pt) {
            if (v < sv) {
              xl = v / g.ns;
              Pt = v % g.ns;
            } else {
              xl = (v - sv) / g.nb;
              Pt = g.ns + (v - sv) % g.nb;
            }
          };
          for (int v = 0; v < nf; ++v) {
            int xl, Pt;
            var(v, xl, Pt);
            const int p2 = np.pts[g.pt_off + Pt];
            maps.push_back((p2 / m3) * ldv + xl * m3 + p2 % m3);
          }
          for (int c = 0; c < 2; ++c)
            for (int v = 0; v < nf; ++v) {
              int idx = -1;
              const int ch = g.child[c];
              if (ch >= 0) {
                int xl, Pt;
                var(v, xl, Pt);
                const int qc = np.chmap[g.chmap_off[c] + Pt];
                if (qc >= 0) idx = (int)(fr[(size_t)j * nfr + ch].u + (size_t)xl * np.fronts[ch].nb + qc);
              }
              maps.push_back(idx);
            }
        }
      }
    }
    if (maps.size() != D.nd_nmaps) return cleanup(fail(HSP_EINVAL, "internal: nested-dissection maps"));
    up(D.o_ndmaps, maps.data(), maps.size() * sizeof(int));
    if (ofac != D.n_fac) return cleanup(fail(HSP_EINVAL, "internal: nested-dissection factor size"));
    // jobs level by level (slab-major within a level); front matrices in the
    // buffer of the level's parity, Gauss-Jordan scratch reused per level
    std::vector<d3::NDJob> jobs(D.nd_njobs);
    std::vector<d3::GJob> gjobs(D.nd_njobs);
    for (int L = 0; L < np.depth; ++L) {
      size_t ob = 0, op = 0, obr = 0;
      int q = D.ndlv[L].first_job;
      for (int j = 0; j < J; ++j)
        for (int f : np.levels[L]) {
          const d3::NDGeom& g = np.fronts[f];
          const int sv = g.ns * D.nls[j], nf = sv + g.nb * D.nls[j];
          d3::NDFront& e = fr[(size_t)j * nfr + f];
          e.F = buf[L & 1] + ob;
          jobs[q] = {j, f};
          d3::GJob& gj = gjobs[q];
          gj.F = e.F;
          gj.nf = nf;
          gj.s = sv;
          gj.ld = nf;
          gj.piv = piv + op;
          gj.col = col + op;
          gj.brow = brow + obr;
          gj.spr = spr + (size_t)(q - D.ndlv[L].first_job) * 32 * 32;
          ob += (size_t)nf * nf;
          op += sv;
          obr += (size_t)32 * nf;
          ++q;
        }
    }
    up(D.o_ndfr, fr.data(), fr.size() * sizeof(d3::NDFront));
    CHK(hipMemcpyAsync(jobs_dev, jobs.data(), jobs.size() * sizeof(d3::NDJob), hipMemcpyHostToDevice, s));
    std::vector<size_t> coff(J);
    size_t o_coef = 0;
    for (int j = 0; j < J; ++j) {
      coff[j] = o_coef;
      o_coef += (size_t)D.nls[j] * D.dm[2] * D.dm[1] * 27;
    }
    CHK(hipMemcpyAsync(coef_off, coff.data(), J * sizeof(size_t), hipMemcpyHostToDevice, s));
    CHK(hipMemcpyAsync(gjobs_dev, gjobs.data(), gjobs.size() * sizeof(d3::GJob), hipMemcpyHostToDevice, s));
    // substitution items: (front, first row) per slab and level, forward and backward
    std::vector<int2> items;
    items.reserve(D.nd_nitems);
    std::vector<int> tab((size_t)J * np.depth * 4, 0);
    for (int j = 0; j < J; ++j)
      for (int L = 0; L < np.depth; ++L) {
        int* ft = &tab[((size_t)j * np.depth + L) * 2];
        int* bt = &tab[(size_t)J * np.depth * 2 + ((size_t)j * np.depth + L) * 2];
        ft[0] = (int)items.size();
        for (int f : np.levels[L]) {
          const d3::NDGeom& g = np.fronts[f];
          const int nf = (g.ns + g.nb) * D.nls[j];
          for (int r0 = 0; r0 < nf; r0 += D.ndlv[L].fwd_rows()) items.push_back(make_int2(f, r0));
        }
        ft[1] = (int)items.size() - ft[0];
        bt[0] = (int)items.size();
        for (int f : np.levels[L]) {
          const d3::NDGeom& g = np.fronts[f];
          if (g.nb == 0) continue;
          const int sv = g.ns * D.nls[j];
          for (int r0 = 0; r0 < sv; r0 += D.ndlv[L].bwd_rows()) items.push_back(make_int2(f, r0));
        }
        bt[1] = (int)items.size() - bt[0];
      }
    if (items.size() != D.nd_nitems) return cleanup(fail(HSP_EINVAL, "internal: nested-dissection items"));
    up(D.o_nditems, items.data(), items.size() * sizeof(int2));
    up(D.o_ndtab, tab.data(), tab.size() * sizeof(int));
    for (hipError_t e : errs)
      if (e != hipSuccess) return cleanup(fail(HSP_EDEVICE, std::string("upload: ") + hipGetErrorString(e)));
    d3::NDSetup Su;
    Su.slabs = D.slabs_dev;
    Su.geom = C->raw<d3::NDGeom>(D.o_ndgeom);
    Su.pts = C->raw<int>(D.o_ndpts);
    Su.lmap = C->raw<int>(D.o_ndlmap);
    Su.chmap = C->raw<int>(D.o_ndchmap);
    Su.cmap = C->raw<int>(D.o_ndcmap);
    Su.fr = C->raw<d3::NDFront>(D.o_ndfr);
    Su.nslabs = J;
    Su.nfronts = nfr;
    Su.m2 = D.dm[1];
    Su.m3 = D.dm[2];
    Su.n_max = D.n_max;
    Su.coef = coefs;
    Su.coef_off = coef_off;
    Su.factors = D.factors;
    Su.jobs = jobs_dev;
    Su.gjobs = gjobs_dev;
    Su.gmax = gmax;
    Su.status = C->raw<int>(D.o_status);
    Su.dbg_slab = debug_knobs().singular_slab;
    Su.dbg_front = np.levels.back()[0];
    CHK(hipMemsetAsync(Su.status, 0, sizeof(int), s));
    CHK(hipMemsetAsync(D.factors, 0, (D.n_fac + kFacTail) * sizeof(cf), s));
    CHK(hipMemsetAsync(gmax, 0, (size_t)J * 2 * sizeof(double), s));
    d3::launch_factor_nd(Su, D.ndlv, s);
    CHK(hipGetLastError());
    std::vector<double> gm(2 * J);
    CHK(hipMemcpyAsync(&hstat, Su.status, sizeof(int), hipMemcpyDeviceToHost, s));
    CHK(hipMemcpyAsync(gm.data(), gmax, 2 * J * sizeof(double), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    for (int j = 0; j < J; ++j) hg[j] = gm[2 * j] > 0 ? std::sqrt(gm[2 * j + 1] / gm[2 * j]) : 0.0;
    // device view for the stages
    D.nds.geom = Su.geom;
    D.nds.maps = C->raw<int>(D.o_ndmaps);
    D.nds.fr = Su.fr;
    D.nds.nfronts = nfr;
    D.nds.depth = np.depth;
    D.nds.items = C->raw<int2>(D.o_nditems);
    D.nds.fwd_tab = C->raw<int>(D.o_ndtab);
    D.nds.bwd_tab = C->raw<int>(D.o_ndtab) + (size_t)J * np.depth * 2;
    D.nds.U = C->at<float>(D.o_ndU);
    D.nds.u_stride = D.nd_u_stride;
  } else {
    d3::Setup3 Su;
    Su.slabs = D.slabs_dev;
    Su.nslabs = J;
    Su.n_max = D.n_max;
    Su.m2 = D.dm[1];
    Su.factors = D.factors;
    {
      Carver sc;
      const size_t nm = (size_t)D.n_max;
      char* base = C->ws + D.o_setup;
      Su.S = reinterpret_cast<cf*>(base + sc.take((size_t)J * nm * nm * sizeof(cf)));
      Su.coef = reinterpret_cast<cf*>(base + sc.take((size_t)J * nm * 27 * sizeof(cf)));
      Su.brow = reinterpret_cast<cf*>(base + sc.take((size_t)J * 32 * nm * sizeof(cf)));
      Su.spr = reinterpret_cast<cf*>(base + sc.take((size_t)J * 32 * 32 * sizeof(cf)));
      Su.piv = reinterpret_cast<int*>(base + sc.take((size_t)J * nm * sizeof(int)));
      Su.col = reinterpret_cast<int*>(base + sc.take((size_t)J * nm * sizeof(int)));
      Su.jobs = reinterpret_cast<d3::GJob*>(base + sc.take((size_t)J * sizeof(d3::GJob)));
      Su.gmax = reinterpret_cast<double*>(base + sc.take((size_t)J * 2 * sizeof(double)));
      if (sc.off > d3::setup3_scratch_bytes(J, D.n_max)) return cleanup(fail(HSP_EINVAL, "internal: setup scratch"));
    }
    std::vector<int> slab_n(J);
    for (int j = 0; j < J; ++j) slab_n[j] = D.slabs_host[j].n;
    std::vector<d3::GJob> jobs(J);
    d3::setup3_jobs(Su, slab_n.data(), jobs.data());
    CHK(hipMemcpyAsync(Su.jobs, jobs.data(), J * sizeof(d3::GJob), hipMemcpyHostToDevice, s));
    Su.status = C->raw<int>(D.o_status);
    Su.dbg_singular = debug_knobs().singular_slab;
    CHK(hipMemsetAsync(Su.status, 0, sizeof(int), s));
    // every factor entry (row padding and the tail included) starts at zero
    CHK(hipMemsetAsync(D.factors, 0, (D.n_fac + kFacTail) * sizeof(cf), s));
    CHK(hipMemsetAsync(Su.gmax, 0, (size_t)J * 2 * sizeof(double), s));
    d3::launch_factor3(Su, s);
    double* growth = C->raw<double>(D.o_growth);
    d3::finish_growth3(Su, growth, s);
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(&hstat, Su.status, sizeof(int), hipMemcpyDeviceToHost, s));
    CHK(hipMemcpyAsync(hg.data(), growth, J * sizeof(double), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
  }
  if (hstat != 0) return cleanup(fail(HSP_ESINGULAR, "zero or non-finite pivot in a slab factorization"));
  C->growth = *std::max_element(hg.begin(), hg.end());
  if (!(C->growth <= growth_limit(sizeof(cf))))
    return cleanup(fail(HSP_ESINGULAR, "growth factor " + std::to_string(C->growth) +
                                           " of the slab Schur complements exceeds the limit " +
                                           std::to_string(growth_limit(sizeof(cf)))));
#undef CHK
  *out = C;
  return HSP_OK;
}

void d3_precond(hsp_ctx* C, const cd* r, cd* z, hipStream_t s) {
  D3Ctx& D = *C->d3;
  const size_t nf = D.nf(), nd = D.nd();
  if (!D.two_grid) {
    cf* fin = C->at<float>(D.o_swf);
    cf* uo = C->at<float>(D.o_tgx0);
    launch_convert<float, double>(r, fin, nf, 0, s);
    run_sweep3(C, fin, uo, s);
    launch_convert<double, float>(uo, z, nf, 0, s);
    return;
  }
  const double wj = C->opt.omega_jac;
  const int nu = C->opt.nu;
  cf* xa = C->at<float>(D.o_tgx0);
  cf* xb = C->at<float>(D.o_tgx1);
  // bytes of one smoothing step: r (complex128), x read and written, k^2
  const double jb = (double)nf * (sizeof(cd) + 2.0 * sizeof(cf) + sizeof(double));
  prof_begin(C, HSP_PROF_SMOOTH, s);
  if (nu > 0) {
    d3::launch_stencil3<float, float, double, float>(D.fine, 2, (const cf*)nullptr, r, xa, wj, s);
    for (int k = 1; k < nu; ++k) {
      d3::launch_stencil3<float, float, double, float>(D.fine, 2, xa, r, xb, wj, s);
      std::swap(xa, xb);
    }
  } else {
    launch_zero<float>(xa, nf, s);
  }
  // coarse-grid correction: r_c = P^T (r - A x) from the complex128 residual
  cd* res = C->at<double>(D.o_tgres);
  d3::launch_stencil3<double, float, double, double>(D.fine, 1, xa, r, res, 0.0, s);
  prof_end(C, HSP_PROF_SMOOTH, s, nu * jb + (double)nf * (2.0 * sizeof(cd) + sizeof(cf) + sizeof(double)));
  cf* rc = C->at<float>(D.o_tgrc);
  cf* ec = C->at<float>(D.o_tgec);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  d3::launch_restrict3<double, float>(D.tr, res, rc, s);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nf * sizeof(cd) + (double)nd * sizeof(cf));
  run_sweep3(C, rc, ec, s);
  prof_begin(C, HSP_PROF_TRANSFER, s);
  d3::launch_prolong_add3<float, float>(D.tr, ec, xa, s);
  prof_end(C, HSP_PROF_TRANSFER, s, (double)nd * sizeof(cf) + 2.0 * nf * sizeof(cf));
  if (nu == 0) {
    launch_convert<double, float>(xa, z, nf, 0, s);
    return;
  }
  prof_begin(C, HSP_PROF_SMOOTH, s);
  for (int k = 0; k < nu; ++k) {
    if (k == nu - 1) {
      d3::launch_stencil3<float, float, double, double>(D.fine, 2, xa, r, z, wj, s);
    } else {
      d3::launch_stencil3<float, float, double, float>(D.fine, 2, xa, r, xb, wj, s);
      std::swap(xa, xb);
    }
  }
  prof_end(C, HSP_PROF_SMOOTH, s, nu * jb);
}

void d3_fine_apply(hsp_ctx* C, int mode, const cd* x, const cd* b, cd* y, hipStream_t s) {
  d3::launch_stencil3<double, double, double, double>(C->d3->fine, mode, x, b, y, 0.0, s);
}

hsp_status d3_rhs(hsp_ctx* C, const cd* f, cd* b, hipStream_t s) {
  D3Ctx& D = *C->d3;
  d3::launch_rhs3(D.m[0], D.m[1], D.m[2], C->h * C->h * C->h, C->at<double>(D.o_ib[0]), C->at<double>(D.o_ib[1]),
                  C->at<double>(D.o_ib[2]), f, b, s);
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status d3_apply_level_operator(hsp_ctx* C, int level, const cd* x, cd* y, hipStream_t s) {
  D3Ctx& D = *C->d3;
  if (level == 0) {
    d3::launch_stencil3<double, double, double, double>(D.fine, 0, x, nullptr, y, 0.0, s);
  } else if (level == 1 && D.two_grid) {
    // the coarse operator in the precision of its use inside the sweep
    const size_t n = D.nd();
    cf* xin = C->at<float>(D.o_cvin);
    cf* yo = C->at<float>(D.o_cvout);
    launch_convert<float, double>(x, xin, n, 0, s);
    d3::launch_stencil3<float, float, float, float>(D.coarse, 0, xin, (const cf*)nullptr, yo, 0.0, s);
    launch_convert<double, float>(yo, y, n, 0, s);
  } else {
    return fail(HSP_EINVAL, "no such level");
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status d3_restrict(hsp_ctx* C, const cd* rf, cd* rc, hipStream_t s) {
  if (!C->d3->two_grid) return fail(HSP_EINVAL, "no coarse level");
  d3::launch_restrict3<double, double>(C->d3->tr, rf, rc, s);
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status d3_prolong_add(hsp_ctx* C, const cd* ec, cd* xf, hipStream_t s) {
  if (!C->d3->two_grid) return fail(HSP_EINVAL, "no coarse level");
  d3::launch_prolong_add3<double, double>(C->d3->tr, ec, xf, s);
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status d3_smooth(hsp_ctx* C, const cd* r, cd* x, int steps, hipStream_t s) {
  D3Ctx& D = *C->d3;
  const double wj = C->opt.omega_jac;
  cd* tmp = C->at<double>(D.o_cvin);
  cd* bufs[2] = {x, tmp};
  int cur = (steps % 2 == 1) ? 0 : 1;
  d3::launch_stencil3<double, double, double, double>(D.fine, 2, (const cd*)nullptr, r, bufs[cur], wj, s);
  for (int k = 1; k < steps; ++k) {
    d3::launch_stencil3<double, double, double, double>(D.fine, 2, bufs[cur], r, bufs[1 - cur], wj, s);
    cur = 1 - cur;
  }
  HIPCHK(hipGetLastError());
  return HSP_OK;
}

hsp_status d3_sweep(hsp_ctx* C, const cd* f, cd* u, hipStream_t s) {
  D3Ctx& D = *C->d3;
  const size_t nd = D.nd();
  cf* fin = C->at<float>(D.o_swf);
  cf* uo = C->at<float>(D.o_swu);
  launch_convert<float, double>(f, fin, nd, 0, s);
  run_sweep3(C, fin, uo, s);
  launch_convert<double, float>(uo, u, nd, 0, s);
  HIPCHK(hipGetLastError());
  return d3_check(C);
}

hsp_status d3_slab_solve(hsp_ctx* C, int j, const cd* b, cd* x, hipStream_t s) {
  D3Ctx& D = *C->d3;
  const size_t n = (size_t)D.nls[j] * D.dm[1] * D.dm[2];
  TaskDev t;
  std::memset(&t, 0, sizeof(t));
  t.slab = j;
  t.mode = 1;
  TaskDev* td = C->tasks_dev + (D.n_tasks - 1);
  HIPCHK(hipMemcpyAsync(td, &t, sizeof(t), hipMemcpyHostToDevice, s));
  cf* fin = C->at<float>(D.o_swf);
  cf* uo = C->at<float>(D.o_swu);
  launch_convert<float, double>(b, fin, n, 0, s);
  d3::Stage3 S;
  S.tasks = td;
  S.slabs = D.slabs_dev;
  S.G = D.dd;
  S.ntasks = 1;
  S.n_max = D.n_max;
  S.nl_max = D.nl_max;
  S.f = fin;
  S.g = fin;
  S.u = uo;
  S.bufs = C->at<float>(D.o_bufs);
  S.fs = C->at<float>(D.o_fs);
  S.ys = C->at<float>(D.o_ys);
  S.factors = D.factors;
  S.nd = D.slab_factor == HSP_SLAB_ND ? &D.nds : nullptr;
  S.nd_lv = &D.ndlv;
  const hipError_t e = d3::launch_stage3(S, s);
  if (e != hipSuccess) return fail(HSP_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
  launch_convert<double, float>(uo, x, n, 0, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));  // the task descriptor is host stack memory
  return HSP_OK;
}

hsp_status d3_check(hsp_ctx* C) {
  D3Ctx& D = *C->d3;
  if (D.launch_err != hipSuccess) {
    const hipError_t e = D.launch_err;
    D.launch_err = hipSuccess;
    return fail(HSP_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
  }
  return HSP_OK;
}

void d3_info(const hsp_ctx* C, hsp_info* info) {
  const D3Ctx& D = *C->d3;
  info->n_fine[0] = D.m[0];
  info->n_fine[1] = D.m[1];
  info->n_fine_z = D.m[2];
  info->n_coarse[0] = D.two_grid ? D.mc[0] : 0;
  info->n_coarse[1] = D.two_grid ? D.mc[1] : 0;
  info->n_coarse_z = D.two_grid ? D.mc[2] : 0;
  info->J = C->J;
  info->max_slab_layers = D.nl_max;
  info->precision = C->opt.precision;
  info->two_grid = D.two_grid;
  info->pivot_growth = C->growth;
  info->dim = 3;
  info->slab_factor = D.slab_factor;
}

}  // namespace hsp
