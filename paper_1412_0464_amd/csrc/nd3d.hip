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
// x = z - F11^-1 F12 x_ring.  Both are dense matrix-vector products, a
// group of lanes per row sized to the level's row length, all fronts of a
// level (and all tasks of a stage) in one launch; the right-hand side and
// solution entries are found through per-front gather maps built at setup.
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

// Block reduction of a non-negative value into *a (max).
__device__ __forceinline__ void block_max_into(double v, double* a) {
  __shared__ double sh[4];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) m = fmax(m, sh[w]);
    if (m > 0) atomic_max_pos(a, m);
  }
}

// The 27 coefficients of every slab row (slab layout: y-block, x_l m3 + z),
// and the largest |entry| of the slab operator.
__global__ void __launch_bounds__(256) kn_coef(NDSetup Su) {
  const Slab3 sl = Su.slabs[blockIdx.y];
  const int n = sl.n, m3 = Su.m3;
  const size_t idx = blockIdx.x * 256ull + threadIdx.x;
  double amax = 0;
  if (idx < (size_t)n * Su.m2) {
    const int y = (int)(idx / n), q = (int)(idx - (idx / n) * n);
    const int xl = q / m3, z = q - (q / m3) * m3;
    cd c[27];
    coefs27(sl.op, xl + 1, y + 1, z + 1, c);
    cf* o = Su.coef + Su.coef_off[blockIdx.y] + idx * 27;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      o[k] = cvt<float>(c[k]);
      amax = fmax(amax, abs2(c[k]));
    }
  }
  block_max_into(amax, Su.gmax + 2 * blockIdx.y);
}

// Front matrices of one level: each wavefront builds one row in LDS (zero,
// the slab operator's entries that belong to the front, the children's
// Schur complements in child order) and writes it out.  Dynamic LDS:
// kAsmRows rows of the level's largest front.
__global__ void __launch_bounds__(64 * kAsmRows) kn_assemble(NDSetup Su, const NDJob* __restrict__ jobs, int ldr) {
  const NDJob jb = jobs[blockIdx.y];
  const Slab3 sl = Su.slabs[jb.slab];
  const NDGeom g = Su.geom[jb.front];
  const int nl = sl.nl, m3 = Su.m3, m2 = Su.m2;
  const int s = g.ns * nl, nf = (g.ns + g.nb) * nl;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * kAsmRows + wv;
  const bool ok = r < nf;
  extern __shared__ cf rowbuf[];
  cf* row = rowbuf + (size_t)wv * ldr;
  for (int j = lane; j < nf; j += 64) row[j] = mk<float>(0, 0);
  int xl = 0, P = 0;
  if (ok) var_of(r, g.ns, g.nb, nl, xl, P);
  const int p2 = Su.pts[g.pt_off + (ok ? P : 0)];
  const int y = p2 / m3, z = p2 - (p2 / m3) * m3;
  const bool sep_row = ok && r < s;
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
        const size_t ri = (size_t)y * sl.n + (size_t)xl * m3 + z;
        row[v] = row[v] + Su.coef[Su.coef_off[jb.slab] + ri * 27 + lane];
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
  if (lane == 0 && ok && fmaxv > 0) atomic_max_pos(Su.gmax + 2 * jb.slab + 1, fmaxv);
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
// Each row of a factor block is taken by a group of G lanes (64 / G rows
// per wavefront, four wavefronts per workgroup), every lane holding NP
// pairs of complex entries (16 bytes each) of its row; all loads of the
// rows are issued before the input vector is gathered into LDS.

template <int NP, int G>
__device__ __forceinline__ void load_rows(floatx4 (&a)[NP], const cf* row, int npair, int sub) {
  const floatx4* w = reinterpret_cast<const floatx4*>(row) + sub;
#pragma unroll
  for (int k = 0; k < NP; ++k)
    a[k] = (sub + G * k < npair) ? __builtin_nontemporal_load(w + G * k) : floatx4{0.f, 0.f, 0.f, 0.f};
}

template <int NP, int G>
__device__ __forceinline__ cf group_dot(const floatx4 (&a)[NP], const cf* vin, int npair, int sub) {
  const floatx4* vv = reinterpret_cast<const floatx4*>(vin) + sub;
  float ar = 0, ai = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (sub + G * k < npair) {
      const floatx4 x = vv[G * k];
      ar += a[k].x * x.x - a[k].y * x.y + a[k].z * x.z - a[k].w * x.w;
      ai += a[k].x * x.y + a[k].y * x.x + a[k].z * x.w + a[k].w * x.z;
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  return mk<float>(ar, ai);
}

// children's update-vector entries that add to front unknown v
__device__ __forceinline__ cf child_sum(const int* __restrict__ ch, int nf, int v, const cf* U) {
  const int a = ch[v], b = ch[nf + v];
  cf r = mk<float>(0, 0);
  if (a >= 0) r = U[a];
  if (b >= 0) r = r + U[b];
  return r;
}

// Forward substitution of one level: rows of GN against v = [f_sep + the
// children's updates]; separator rows give z (into ys), ring rows the
// front's update vector.
template <int NP, int G>
__global__ void __launch_bounds__(256) kn_fwd(Stage3 st, NDSolve nd, int level) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const int* tab = nd.fwd_tab + ((size_t)tk.slab * nd.depth + level) * 2;
  if ((int)blockIdx.x >= tab[1]) return;
  const int2 it = nd.items[tab[0] + blockIdx.x];
  const Slab3 sl = st.slabs[tk.slab];
  const NDGeom g = nd.geom[it.x];
  const NDFront fr = nd.fr[(size_t)tk.slab * nd.nfronts + it.x];
  const int nl = sl.nl, m2 = st.G.m2;
  const int s = g.ns * nl, b = g.nb * nl, nf = s + b;
  const int ldv = st.n_max + (st.n_max & 1);
  const cf* fs = st.fs + (size_t)blockIdx.y * m2 * ldv;
  cf* ys = st.ys + (size_t)blockIdx.y * m2 * ldv;
  cf* U = nd.U + (size_t)blockIdx.y * nd.u_stride;
  const int* sep = nd.maps + fr.m;
  const int* ch = sep + s + b;
  __shared__ __align__(16) cf vin[2 * G * NP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sub = lane % G;
  const int r = it.y + wv * (64 / G) + lane / G;
  const bool ok = r < nf;
  const int npair = (s + 1) / 2;
  floatx4 a[NP];
  load_rows<NP, G>(a, st.factors + fr.gn + (size_t)(ok ? r : 0) * (s + (s & 1)), npair, sub);
  for (int e = tid; e < 2 * npair; e += 256) vin[e] = e < s ? fs[sep[e]] + child_sum(ch, nf, e, U) : mk<float>(0, 0);
  __syncthreads();
  const cf d = group_dot<NP, G>(a, vin, npair, sub);
  if (sub == 0 && ok) {
    if (r < s)
      ys[sep[r]] = d;
    else
      U[fr.u + (r - s)] = d + child_sum(ch, nf, r, U);
  }
}

// Backward substitution of one level: x_sep = z - E x_ring.
template <int NP, int G>
__global__ void __launch_bounds__(256) kn_bwd(Stage3 st, NDSolve nd, int level) {
  const TaskDev tk = st.tasks[blockIdx.y];
  const int* tab = nd.bwd_tab + ((size_t)tk.slab * nd.depth + level) * 2;
  if ((int)blockIdx.x >= tab[1]) return;
  const int2 it = nd.items[tab[0] + blockIdx.x];
  const Slab3 sl = st.slabs[tk.slab];
  const NDGeom g = nd.geom[it.x];
  const NDFront fr = nd.fr[(size_t)tk.slab * nd.nfronts + it.x];
  const int nl = sl.nl, m2 = st.G.m2;
  const int s = g.ns * nl, b = g.nb * nl;
  const int ldv = st.n_max + (st.n_max & 1);
  cf* ys = st.ys + (size_t)blockIdx.y * m2 * ldv;
  const int* sep = nd.maps + fr.m;
  const int* ring = sep + s;
  __shared__ __align__(16) cf xin[2 * G * NP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sub = lane % G;
  const int r = it.y + wv * (64 / G) + lane / G;
  const bool ok = r < s;
  const int npair = (b + 1) / 2;
  floatx4 a[NP];
  load_rows<NP, G>(a, st.factors + fr.e + (size_t)(ok ? r : 0) * (b + (b & 1)), npair, sub);
  for (int e = tid; e < 2 * npair; e += 256) xin[e] = e < b ? ys[ring[e]] : mk<float>(0, 0);
  __syncthreads();
  const cf d = group_dot<NP, G>(a, xin, npair, sub);
  if (sub == 0 && ok) {
    cf* y = ys + sep[r];
    *y = *y - d;
  }
}

}  // namespace

void launch_factor_nd(const NDSetup& Su, const std::vector<NDLevelHost>& lv, hipStream_t s) {
  hipLaunchKernelGGL(kn_coef, dim3(nblk((size_t)Su.n_max * Su.m2), Su.nslabs), dim3(256), 0, s, Su);
  for (int L = (int)lv.size() - 1; L >= 0; --L) {
    const NDLevelHost& l = lv[L];
    if (l.njobs < 1) continue;
    const NDJob* jobs = Su.jobs + l.first_job;
    const GJob* gj = Su.gjobs + l.first_job;
    const int ldr = l.nf_max + (l.nf_max & 1);
    hipLaunchKernelGGL(kn_assemble, dim3((l.nf_max + kAsmRows - 1) / kAsmRows, l.njobs), dim3(64 * kAsmRows),
                       kAsmRows * ldr * sizeof(cf), s, Su, jobs, ldr);
    launch_gauss_jordan(gj, l.njobs, l.s_max, l.b_max, l.nf_max, Su.status, s);
    const size_t cnt = (size_t)l.nf_max * l.s_max + (size_t)l.s_max * l.b_max;
    hipLaunchKernelGGL(kn_store, dim3(nblk(cnt), l.njobs), dim3(256), 0, s, Su, jobs, gj);
  }
}

void nd_row_shape(int n, int* g, int* np) {
  const int pairs = (n + 1) / 2;
  static const int shapes[][3] = {{16, 16, 1}, {32, 16, 2}, {48, 16, 3}, {64, 32, 2},  {128, 32, 4},
                                  {256, 64, 4}, {384, 64, 6}, {512, 64, 8}, {768, 64, 12}, {1024, 64, 16}};
  for (const auto& sh : shapes)
    if (pairs <= sh[0]) {
      *g = sh[1];
      *np = sh[2];
      return;
    }
  *g = 64;
  *np = 16;
}

void launch_nd_solve(const Stage3& st, const NDSolve& nd, const std::vector<NDLevelHost>& lv, hipStream_t s) {
  const int depth = (int)lv.size();
  auto fwd = [&](int L) {
    const dim3 grd(std::max(lv[L].fwd_items, 1), st.ntasks);
#define ND_F(NP, G)                                                                 \
  if (lv[L].fwd_g == G && lv[L].fwd_np == NP) {                                     \
    hipLaunchKernelGGL((kn_fwd<NP, G>), grd, dim3(256), 0, s, st, nd, L);           \
    return;                                                                         \
  }
    ND_F(1, 16) ND_F(2, 16) ND_F(3, 16) ND_F(2, 32) ND_F(4, 32) ND_F(4, 64) ND_F(6, 64) ND_F(8, 64) ND_F(12, 64)
    ND_F(16, 64)
#undef ND_F
  };
  auto bwd = [&](int L) {
    const dim3 grd(lv[L].bwd_items, st.ntasks);
#define ND_B(NP, G)                                                                 \
  if (lv[L].bwd_g == G && lv[L].bwd_np == NP) {                                     \
    hipLaunchKernelGGL((kn_bwd<NP, G>), grd, dim3(256), 0, s, st, nd, L);           \
    return;                                                                         \
  }
    ND_B(1, 16) ND_B(2, 16) ND_B(3, 16) ND_B(2, 32) ND_B(4, 32) ND_B(4, 64) ND_B(6, 64) ND_B(8, 64) ND_B(12, 64)
    ND_B(16, 64)
#undef ND_B
  };
  for (int L = depth - 1; L >= 0; --L) fwd(L);
  for (int L = 0; L < depth; ++L)
    if (lv[L].bwd_items > 0) bwd(L);
}

}  // namespace d3
}  // namespace hsp
