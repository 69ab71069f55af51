// Nested-dissection (multifrontal) factorization of the three-dimensional
// slabs and its level-synchronous substitutions (Sec. 2.1 subdomains; the
// paper solves the slabs with a sparse multifrontal package, Sec. 5, whose
// nested-dissection cost estimate Sec. 7 quotes).
//
// The plane of a slab is dissected once on the host (nd_plan); every front
// of every slab of a level is then factored by the same launches:
//   kn_assemble  the front matrix: its rows of the slab operator (separator
//                rows against the separator and the ring, ring rows against
//                the separator) plus the Schur complements of its children
//                (extend-add, child by child in a fixed order);
//   Gauss-Jordan the first s columns eliminated (partial pivoting among the
//                separator rows, rank-32 updates on the FP32 matrix cores),
//                which leaves F11^-1, F11^-1 F12, -F21 F11^-1 and the Schur
//                complement F22 - F21 F11^-1 F12 in place;
//   kn_store     GN = [F11^-1 ; -F21 F11^-1] and E = F11^-1 F12 (columns of
//                the inverse un-permuted) into the factor array; the Schur
//                complement stays for the parent.
// The substitutions of one slab solve: forward, leaves to root, each front
// forms v = its separator's right-hand side plus its children's update
// vectors, z = F11^-1 v (kept in the solution vector) and its own update
// vector u = v_ring - F21 F11^-1 v; backward, root to leaves,
// x = z - F11^-1 F12 x_ring.  Both are dense matrix-vector products with
// one wavefront per row, all fronts of a level (and all tasks of a stage) in
// one launch.
#include <algorithm>
#include <cmath>
#include <functional>

#include "d3.h"

namespace hsp {
namespace d3 {

// ---- host plan -----------------------------------------------------------------

bool nd_plan(int m2, int m3, NDPlan& P, std::string* why) {
  P = NDPlan();
  P.m2 = m2;
  P.m3 = m3;
  // rectangles in pre-order (the root first)
  struct Rect {
    int y0, y1, z0, z1, parent, level;
  };
  std::vector<Rect> rects;
  std::vector<std::vector<int>> sep;
  std::function<int(int, int, int, int, int, int)> rec = [&](int y0, int y1, int z0, int z1, int parent,
                                                            int level) -> int {
    if (y1 <= y0 || z1 <= z0) return -1;
    const int id = (int)rects.size();
    rects.push_back({y0, y1, z0, z1, parent, level});
    sep.emplace_back();
    NDGeom g{};
    g.child[0] = g.child[1] = -1;
    g.level = level;
    P.fronts.push_back(g);
    const int h = y1 - y0, w = z1 - z0;
    if (h * w <= kNDLeaf) {
      for (int y = y0; y < y1; ++y)
        for (int z = z0; z < z1; ++z) sep[id].push_back(y * m3 + z);
      return id;
    }
    int c0, c1;
    if (h >= w) {
      const int ys = (y0 + y1) / 2;
      for (int z = z0; z < z1; ++z) sep[id].push_back(ys * m3 + z);
      c0 = rec(y0, ys, z0, z1, id, level + 1);
      c1 = rec(ys + 1, y1, z0, z1, id, level + 1);
    } else {
      const int zs = (z0 + z1) / 2;
      for (int y = y0; y < y1; ++y) sep[id].push_back(y * m3 + zs);
      c0 = rec(y0, y1, z0, zs, id, level + 1);
      c1 = rec(y0, y1, zs + 1, z1, id, level + 1);
    }
    int nc = 0;
    if (c0 >= 0) P.fronts[id].child[nc++] = c0;
    if (c1 >= 0) P.fronts[id].child[nc++] = c1;
    return id;
  };
  rec(0, m2, 0, m3, -1, 0);
  const int nfr = (int)rects.size();
  // separator, ring and the local map over the rectangle and its border
  for (int f = 0; f < nfr; ++f) {
    const Rect& r = rects[f];
    NDGeom& g = P.fronts[f];
    g.y0 = r.y0;
    g.z0 = r.z0;
    g.h = r.y1 - r.y0;
    g.w = r.z1 - r.z0;
    g.ns = (int)sep[f].size();
    g.pt_off = (int)P.pts.size();
    g.lmap_off = (int)P.lmap.size();
    const int W = g.w + 2;
    P.lmap.resize(P.lmap.size() + (size_t)(g.h + 2) * W, -1);
    for (int k = 0; k < g.ns; ++k) {
      const int p2 = sep[f][k], y = p2 / m3, z = p2 % m3;
      P.pts.push_back(p2);
      P.lmap[g.lmap_off + (y - g.y0 + 1) * W + (z - g.z0 + 1)] = k;
    }
    int nb = 0;
    for (int y = r.y0 - 1; y <= r.y1; ++y)
      for (int z = r.z0 - 1; z <= r.z1; ++z) {
        if (y >= r.y0 && y < r.y1 && z >= r.z0 && z < r.z1) continue;
        if (y < 0 || y >= m2 || z < 0 || z >= m3) continue;
        P.pts.push_back(y * m3 + z);
        P.lmap[g.lmap_off + (y - g.y0 + 1) * W + (z - g.z0 + 1)] = g.ns + nb;
        ++nb;
      }
    g.nb = nb;
  }
  auto local = [&](const NDGeom& g, int y, int z) {
    if (y < g.y0 - 1 || y > g.y0 + g.h || z < g.z0 - 1 || z > g.z0 + g.w) return -1;
    return P.lmap[g.lmap_off + (y - g.y0 + 1) * (g.w + 2) + (z - g.z0 + 1)];
  };
  // child maps
  for (int f = 0; f < nfr; ++f) {
    NDGeom& g = P.fronts[f];
    for (int c = 0; c < 2; ++c) {
      g.chmap_off[c] = -1;
      const int ch = g.child[c];
      if (ch < 0) continue;
      const NDGeom& gc = P.fronts[ch];
      g.chmap_off[c] = (int)P.chmap.size();
      for (int k = 0; k < g.ns + g.nb; ++k) {
        const int p2 = P.pts[g.pt_off + k];
        const int v = local(gc, p2 / m3, p2 % m3);
        if (v >= 0 && v < gc.ns) {
          if (why) *why = "nested dissection: a parent node inside a child's separator";
          return false;
        }
        P.chmap.push_back(v >= gc.ns ? v - gc.ns : -1);
      }
    }
  }
  for (int f = 0; f < nfr; ++f) {
    NDGeom& g = P.fronts[f];
    g.cmap_off = (int)P.cmap.size();
    const int par = rects[f].parent;
    for (int q = 0; q < g.nb; ++q) {
      const int p2 = P.pts[g.pt_off + g.ns + q];
      const int v = par >= 0 ? local(P.fronts[par], p2 / m3, p2 % m3) : -1;
      if (v < 0) {
        if (why) *why = "nested dissection: a ring node outside the parent's front";
        return false;
      }
      P.cmap.push_back(v);
    }
  }
  for (int f = 0; f < nfr; ++f) {
    const int L = P.fronts[f].level;
    if ((int)P.levels.size() <= L) P.levels.resize(L + 1);
    P.levels[L].push_back(f);
  }
  P.depth = (int)P.levels.size();
  return true;
}

NDSizes nd_sizes(const NDPlan& P, int nl) {
  NDSizes z;
  for (const NDGeom& g : P.fronts) {
    const size_t s = (size_t)g.ns * nl, b = (size_t)g.nb * nl, nf = s + b;
    z.factor += nf * (s + (s & 1)) + s * (b + (b & 1));
    z.update += b;
    z.rows += (nf + 3) / 4;
    z.s_max = std::max(z.s_max, (int)s);
    z.b_max = std::max(z.b_max, (int)b);
    z.nf_max = std::max(z.nf_max, (int)nf);
  }
  return z;
}

namespace {

inline int nblk(size_t n, int t = 256) { return (int)std::min<size_t>((n + t - 1) / t, (size_t)1 << 20); }

typedef float floatx4 __attribute__((ext_vector_type(4)));

// front variable v -> (x layer, front point)
__device__ __forceinline__ void var_of(int v, int ns, int nb, int nl, int& xl, int& P) {
  const int s = ns * nl;
  if (v < s) {
    xl = v / ns;
    P = v - xl * ns;
  } else {
    const int u = v - s;
    xl = u / nb;
    P = ns + (u - xl * nb);
  }
}
__device__ __forceinline__ int var_idx(int xl, int P, int ns, int nb, int nl) {
  return P < ns ? xl * ns + P : ns * nl + xl * nb + (P - ns);
}

__device__ __forceinline__ void atomic_max_pos(double* a, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(a), (unsigned long long)__double_as_longlong(v));
}

// ---- setup -----------------------------------------------------------------------
constexpr int kAsmRows = 2;  // front rows per workgroup of the assembly (one per wavefront)

// Front matrices of one level: each wavefront builds one row in LDS (zero,
// the slab operator's entries that belong to the front, the children's
// Schur complements in child order) and writes it out.
__global__ void __launch_bounds__(64 * kAsmRows) kn_assemble(NDSetup Su, const NDJob* __restrict__ jobs) {
  const NDJob jb = jobs[blockIdx.y];
  const Slab3 sl = Su.slabs[jb.slab];
  const NDGeom g = Su.geom[jb.front];
  const int nl = sl.nl, m3 = Su.m3, m2 = Su.m2;
  const int s = g.ns * nl, nf = (g.ns + g.nb) * nl;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * kAsmRows + wv;
  const bool ok = r < nf;
  __shared__ cf rowbuf[kAsmRows][kNDMaxFront];
  __shared__ cf cofs[kAsmRows][27];
  cf* row = rowbuf[wv];
  for (int j = lane; j < nf; j += 64) row[j] = mk<float>(0, 0);
  int xl = 0, P = 0;
  if (ok) var_of(r, g.ns, g.nb, nl, xl, P);
  const int p2 = Su.pts[g.pt_off + (ok ? P : 0)];
  const int y = p2 / m3, z = p2 - (p2 / m3) * m3;
  const bool sep_row = ok && r < s;
  double amax = 0;
  if (ok && lane == 0) {
    cd c[27];
    coefs27(sl.op, xl + 1, y + 1, z + 1, c);
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      cofs[wv][k] = cvt<float>(c[k]);
      if (sep_row) amax = fmax(amax, abs2(c[k]));
    }
  }
  __syncthreads();
  if (ok && lane < 27) {
    const int dx = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dz = lane % 3 - 1;
    const int xx = xl + dx, yy = y + dy, zz = z + dz;
    if (xx >= 0 && xx < nl && yy >= 0 && yy < m2 && zz >= 0 && zz < m3 && yy >= g.y0 - 1 && yy <= g.y0 + g.h &&
        zz >= g.z0 - 1 && zz <= g.z0 + g.w) {
      const int Q = Su.lmap[g.lmap_off + (yy - g.y0 + 1) * (g.w + 2) + (zz - g.z0 + 1)];
      // separator rows take their couplings to the separator and the ring,
      // ring rows only those to the separator (the rest belongs to ancestors)
      if (Q >= 0 && (sep_row || Q < g.ns)) {
        const int v = var_idx(xx, Q, g.ns, g.nb, nl);
        row[v] = row[v] + cofs[wv][lane];
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < 2; ++c) {
    const int ch = g.child[c];
    if (ch >= 0 && ok) {
      const int qc = Su.chmap[g.chmap_off[c] + P];
      if (qc >= 0) {
        const NDGeom gc = Su.geom[ch];
        const NDFront fc = Su.fr[(size_t)jb.slab * Su.nfronts + ch];
        const int sc = gc.ns * nl, bc = gc.nb * nl, ldc = sc + bc;
        const cf* crow = fc.F + (size_t)(sc + xl * gc.nb + qc) * ldc + sc;
        for (int j = lane; j < bc; j += 64) {
          const int xj = j / gc.nb, qj = j - xj * gc.nb;
          const int Pp = Su.cmap[gc.cmap_off + qj];
          const int v = var_idx(xj, Pp, g.ns, g.nb, nl);
          row[v] = row[v] + crow[j];
        }
      }
    }
    __syncthreads();
  }
  const bool dbg = sep_row && jb.slab == Su.dbg_slab && jb.front == Su.dbg_front;
  double fmaxv = 0;
  if (ok) {
    const NDFront fr = Su.fr[(size_t)jb.slab * Su.nfronts + jb.front];
    cf* out = fr.F + (size_t)r * nf;
    for (int j = lane; j < nf; j += 64) {
      cf v = row[j];
      if (dbg && j < s) v = mk<float>(0, 0);
      if (sep_row && j < s) fmaxv = fmax(fmaxv, (double)abs2(v));
      out[j] = v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) fmaxv = fmax(fmaxv, __shfl_xor(fmaxv, off, 64));
  if (lane == 0 && ok) {
    if (amax > 0) atomic_max_pos(Su.gmax + 2 * jb.slab, amax);
    if (fmaxv > 0) atomic_max_pos(Su.gmax + 2 * jb.slab + 1, fmaxv);
  }
}

// GN = [F11^-1 ; -F21 F11^-1] (columns un-permuted) and E = F11^-1 F12.
__global__ void __launch_bounds__(256) kn_store(NDSetup Su, const NDJob* __restrict__ jobs,
                                                const GJob* __restrict__ gj) {
  const NDJob jb = jobs[blockIdx.y];
  const GJob G = gj[blockIdx.y];
  const NDFront fr = Su.fr[(size_t)jb.slab * Su.nfronts + jb.front];
  const int s = G.s, nf = G.nf, b = nf - s;
  const size_t ngn = (size_t)nf * s;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  if (idx < ngn) {
    const int i = (int)(idx / s), j = (int)(idx - (idx / s) * s);
    Su.factors[fr.gn + (size_t)i * (s + (s & 1)) + j] = G.F[(size_t)i * G.ld + G.col[j]];
  } else if (idx < ngn + (size_t)s * b) {
    const size_t e = idx - ngn;
    const int i = (int)(e / b), j = (int)(e - (e / b) * b);
    Su.factors[fr.e + (size_t)i * (b + (b & 1)) + j] = G.F[(size_t)i * G.ld + s + j];
  }
}

// ---- substitutions -------------------------------------------------------------
constexpr int kRows = 4;  // rows per workgroup (one per wavefront)

template <int NP>
__device__ __forceinline__ void load_row(floatx4 (&a)[NP], const cf* row, int npair, int lane) {
  const floatx4* w = reinterpret_cast<const floatx4*>(row) + lane;
#pragma unroll
  for (int k = 0; k < NP; ++k)
    a[k] = (lane + 64 * k < npair) ? __builtin_nontemporal_load(w + 64 * k) : floatx4{0.f, 0.f, 0.f, 0.f};
}

template <int NP>
__device__ __forceinline__ cf row_dot(const floatx4 (&a)[NP], const cf* vin, int npair, int lane) {
  const floatx4* vv = reinterpret_cast<const floatx4*>(vin) + lane;
  float ar = 0, ai = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (lane + 64 * k < npair) {
      const floatx4 x = vv[64 * k];
      ar += a[k].x * x.x - a[k].y * x.y + a[k].z * x.z - a[k].w * x.w;
      ai += a[k].x * x.y + a[k].y * x.x + a[k].z * x.w + a[k].w * x.z;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  return mk<float>(ar, ai);
}

// Position of front point P, layer xl, in a task's slab-layout vector.
__device__ __forceinline__ size_t slab_pos(const NDSolve& nd, const NDGeom& g, int xl, int P, int m3, int ldv) {
  const int p2 = nd.pts[g.pt_off + P];
  const int y = p2 / m3, z = p2 - (p2 / m3) * m3;
  return (size_t)y * ldv + (size_t)xl * m3 + z;
}

// Sum of the children's update vectors at front point P, layer xl.
__device__ __forceinline__ cf child_sum(const NDSolve& nd, const NDGeom& g, int slab, int xl, int P, const cf* U) {
  cf v = mk<float>(0, 0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int ch = g.child[c];
    if (ch < 0) continue;
    const int qc = nd.chmap[g.chmap_off[c] + P];
    if (qc < 0) continue;
    const int nbc = nd.geom[ch].nb;
    v = v + U[nd.fr[(size_t)slab * nd.nfronts + ch].u + (size_t)xl * nbc + qc];
  }
  return v;
}

// Forward substitution of one level: rows of GN against v = [f_sep + the
// children's updates]; separator rows give z (into ys), ring rows the
// front's update vector.
template <int NP>
__global__ void __launch_bounds__(256) kn_fwd(Stage3 st, NDSolve nd, int level) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const int* tab = nd.fwd_tab + ((size_t)tk.slab * nd.depth + level) * 2;
  if ((int)blockIdx.x >= tab[1]) return;
  const int2 it = nd.items[tab[0] + blockIdx.x];
  const Slab3 sl = st.slabs[tk.slab];
  const NDGeom g = nd.geom[it.x];
  const NDFront fr = nd.fr[(size_t)tk.slab * nd.nfronts + it.x];
  const int nl = sl.nl, m3 = st.G.m3, m2 = st.G.m2;
  const int s = g.ns * nl, nf = (g.ns + g.nb) * nl;
  const int ldv = st.n_max + (st.n_max & 1);
  const cf* fs = st.fs + (size_t)blockIdx.y * m2 * ldv;
  cf* ys = st.ys + (size_t)blockIdx.y * m2 * ldv;
  cf* U = nd.U + (size_t)blockIdx.y * nd.u_stride;
  __shared__ __align__(16) cf vin[128 * NP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = it.y + wv;
  const bool ok = r < nf;
  const int npair = (s + 1) / 2;
  floatx4 a[NP];
  load_row(a, st.factors + fr.gn + (size_t)(ok ? r : 0) * (s + (s & 1)), npair, lane);
  for (int e = tid; e < 2 * npair; e += 256) {
    cf v = mk<float>(0, 0);
    if (e < s) {
      int xl, P;
      var_of(e, g.ns, g.nb, nl, xl, P);
      v = fs[slab_pos(nd, g, xl, P, m3, ldv)] + child_sum(nd, g, tk.slab, xl, P, U);
    }
    vin[e] = v;
  }
  __syncthreads();
  const cf d = row_dot(a, vin, npair, lane);
  if (lane == 0 && ok) {
    int xl, P;
    var_of(r, g.ns, g.nb, nl, xl, P);
    if (r < s)
      ys[slab_pos(nd, g, xl, P, m3, ldv)] = d;
    else
      U[fr.u + (r - s)] = d + child_sum(nd, g, tk.slab, xl, P, U);
  }
}

// Backward substitution of one level: x_sep = z - E x_ring.
template <int NP>
__global__ void __launch_bounds__(256) kn_bwd(Stage3 st, NDSolve nd, int level) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const int* tab = nd.bwd_tab + ((size_t)tk.slab * nd.depth + level) * 2;
  if ((int)blockIdx.x >= tab[1]) return;
  const int2 it = nd.items[tab[0] + blockIdx.x];
  const Slab3 sl = st.slabs[tk.slab];
  const NDGeom g = nd.geom[it.x];
  const NDFront fr = nd.fr[(size_t)tk.slab * nd.nfronts + it.x];
  const int nl = sl.nl, m3 = st.G.m3, m2 = st.G.m2;
  const int s = g.ns * nl, b = g.nb * nl;
  const int ldv = st.n_max + (st.n_max & 1);
  cf* ys = st.ys + (size_t)blockIdx.y * m2 * ldv;
  __shared__ __align__(16) cf xin[128 * NP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = it.y + wv;
  const bool ok = r < s;
  const int npair = (b + 1) / 2;
  floatx4 a[NP];
  load_row(a, st.factors + fr.e + (size_t)(ok ? r : 0) * (b + (b & 1)), npair, lane);
  for (int e = tid; e < 2 * npair; e += 256) {
    cf v = mk<float>(0, 0);
    if (e < b) {
      const int xl = e / g.nb, q = e - xl * g.nb;
      v = ys[slab_pos(nd, g, xl, g.ns + q, m3, ldv)];
    }
    xin[e] = v;
  }
  __syncthreads();
  const cf d = row_dot(a, xin, npair, lane);
  if (lane == 0 && ok) {
    const int xl = r / g.ns, P = r - xl * g.ns;
    cf* y = ys + slab_pos(nd, g, xl, P, m3, ldv);
    *y = *y - d;
  }
}

}  // namespace

void launch_factor_nd(const NDSetup& Su, const std::vector<NDLevelHost>& lv, hipStream_t s) {
  for (int L = (int)lv.size() - 1; L >= 0; --L) {
    const NDLevelHost& l = lv[L];
    if (l.njobs < 1) continue;
    const NDJob* jobs = Su.jobs + l.first_job;
    const GJob* gj = Su.gjobs + l.first_job;
    hipLaunchKernelGGL(kn_assemble, dim3((l.nf_max + kAsmRows - 1) / kAsmRows, l.njobs), dim3(64 * kAsmRows), 0, s,
                       Su, jobs);
    launch_gauss_jordan(gj, l.njobs, l.s_max, l.b_max, l.nf_max, Su.status, s);
    const size_t cnt = (size_t)l.nf_max * l.s_max + (size_t)l.s_max * l.b_max;
    hipLaunchKernelGGL(kn_store, dim3(nblk(cnt), l.njobs), dim3(256), 0, s, Su, jobs, gj);
  }
}

void launch_nd_solve(const Stage3& st, const NDSolve& nd, const std::vector<NDLevelHost>& lv, hipStream_t s) {
  const int depth = (int)lv.size();
#define ND_FWD(NP) hipLaunchKernelGGL((kn_fwd<NP>), grd, dim3(256), 0, s, st, nd, L)
#define ND_BWD(NP) hipLaunchKernelGGL((kn_bwd<NP>), grd, dim3(256), 0, s, st, nd, L)
  for (int L = depth - 1; L >= 0; --L) {
    const dim3 grd(std::max(lv[L].fwd_items, 1), st.ntasks);
    const int np = (lv[L].s_max + 127) / 128;
    if (np <= 1)
      ND_FWD(1);
    else if (np <= 2)
      ND_FWD(2);
    else if (np <= 4)
      ND_FWD(4);
    else if (np <= 6)
      ND_FWD(6);
    else if (np <= 8)
      ND_FWD(8);
    else
      ND_FWD(12);
  }
  for (int L = 0; L < depth; ++L) {
    if (lv[L].bwd_items < 1) continue;
    const dim3 grd(lv[L].bwd_items, st.ntasks);
    const int np = (lv[L].b_max + 127) / 128;
    if (np <= 1)
      ND_BWD(1);
    else if (np <= 2)
      ND_BWD(2);
    else if (np <= 4)
      ND_BWD(4);
    else if (np <= 6)
      ND_BWD(6);
    else if (np <= 8)
      ND_BWD(8);
    else if (np <= 12)
      ND_BWD(12);
    else
      ND_BWD(16);
  }
#undef ND_FWD
#undef ND_BWD
}

}  // namespace d3
}  // namespace hsp
