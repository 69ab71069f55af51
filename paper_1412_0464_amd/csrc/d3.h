// Three-dimensional path: level views, slab views and the kernels of the
// 3-D operators, transfers, slab factorization and sweep stage.  Not part of
// the public ABI.
//
// Vectors are dense over the unknown nodes (i, j, k) of an m1 x m2 x m3 grid
// (x slowest, z fastest): index ((i-1) m2 + (j-1)) m3 + (k-1), x being the
// sweep axis.  A slab of nl x-layers is block tridiagonal along y: block t
// (y node t+1) holds the n = nl m3 unknowns (x_l, z) in the order
// q = x_l m3 + z, so that each x-layer of a block is a contiguous run of m3
// values of the level vector.
#pragma once

#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

namespace hsp {
namespace d3 {

// Compact-stencil Helmholtz operator on a 3-D rectilinear mesh with PML.
//  kind 7  - standard 7-point finite differences (3-D form of eq.
//            define_pml_fd), FE scaled by h^3:
//              A[a][p] = alpha_a at half node p + 1/2 (p = 0..m_a)
//              B[a][i] = 1 / alpha_a at node i       (i = 0..m_a + 1)
//              k2 at unknown nodes (x row stride m2 m3), hs = h.
//  kind 27 - finite-element form H_FE of eq. define_H_FE with the constants
//            of eq. def_IJ_opt:
//              A[a][p] = alpha_a / h_a of cell p, B[a][p] = h_a / alpha_a
//              (p = 0..m_a), k2 and coef (c1..c5) per cell (x row stride
//              (m2+1)(m3+1)).
// xmap (optional) maps the view's x row (node i-1 for kind 7, cell p for
// kind 27) to the row of k2 / coef: a slab reuses the global medium with
// the k continuation of its added layers.
struct Level3 {
  int kind;
  int m1, m2, m3;
  double hs;  // h (kind 7: h^3 / h^2)
  const cd* A[3];
  const cd* B[3];
  const double* k2;
  const double* coef;
  const int* xmap;
};

// Row (i, j, k) (1-based unknown node) of the operator: c[(dx+1)*9 +
// (dy+1)*3 + (dz+1)] multiplies u(i+dx, j+dy, k+dz).  Computed in double.
__device__ __forceinline__ void coefs27(const Level3& L, int i, int j, int k, cd c[27]) {
#pragma unroll
  for (int a = 0; a < 27; ++a) c[a] = mk<double>(0.0, 0.0);
  if (L.kind == 7) {
    const int row = L.xmap ? L.xmap[i - 1] : (i - 1);
    const double k2 = L.k2[((size_t)row * L.m2 + (j - 1)) * L.m3 + (k - 1)];
    const cd ix = L.B[0][i], iy = L.B[1][j], iz = L.B[2][k];
    const double h = L.hs;
    // the 1-D operator of axis a, divided by the alphas of the other axes
    const cd tx = h * (iy * iz), ty = h * (ix * iz), tz = h * (ix * iy);
    const cd xl = -(L.A[0][i - 1] * tx), xr = -(L.A[0][i] * tx);
    const cd yl = -(L.A[1][j - 1] * ty), yr = -(L.A[1][j] * ty);
    const cd zl = -(L.A[2][k - 1] * tz), zr = -(L.A[2][k] * tz);
    c[0 * 9 + 1 * 3 + 1] = xl;
    c[2 * 9 + 1 * 3 + 1] = xr;
    c[1 * 9 + 0 * 3 + 1] = yl;
    c[1 * 9 + 2 * 3 + 1] = yr;
    c[1 * 9 + 1 * 3 + 0] = zl;
    c[1 * 9 + 1 * 3 + 2] = zr;
    c[13] = -(xl + xr + yl + yr + zl + zr) - (h * h * h * k2) * (ix * (iy * iz));
    return;
  }
  // kind 27: the element matrices of the eight cells around the node
  const size_t s2 = (size_t)(L.m2 + 1) * (L.m3 + 1);
#pragma unroll
  for (int px = 0; px < 2; ++px) {
#pragma unroll
    for (int qy = 0; qy < 2; ++qy) {
#pragma unroll
      for (int rz = 0; rz < 2; ++rz) {
        const int p = i - 1 + px, q = j - 1 + qy, r = k - 1 + rz;  // cell
        const int ax = i - p, ay = j - q, az = k - r;               // the node's corner
        const int row = L.xmap ? L.xmap[p] : p;
        const size_t ci = (size_t)row * s2 + (size_t)q * (L.m3 + 1) + r;
        const double k2 = L.k2[ci];
        const double* cf = L.coef + 5 * ci;
        const double I0 = 0.125 * cf[0], I1 = cf[1] / 24.0, I2 = cf[2] / 24.0;
        const double I3 = 0.125 * (1.0 - cf[0] - cf[1] - cf[2]);
        const double J0 = 0.25 * cf[3], J1 = 0.125 * cf[4], J2 = 0.25 * (1.0 - cf[3] - cf[4]);
        const cd ha = L.B[0][p], hb = L.B[1][q], hc = L.B[2][r];
        const cd s1 = L.A[0][p] * (hb * hc), s2v = L.A[1][q] * (ha * hc), s3 = L.A[2][r] * (ha * hb);
        const cd m = k2 * (ha * (hb * hc));
        const double Iv[4] = {I0, I1, I2, I3};
        const double Jv[3] = {J0, J1, J2};
#pragma unroll
        for (int bx = 0; bx < 2; ++bx)
#pragma unroll
          for (int by = 0; by < 2; ++by)
#pragma unroll
            for (int bz = 0; bz < 2; ++bz) {
              const int d1 = bx != ax, d2 = by != ay, d3 = bz != az;
              cd e = -(Iv[d1 + d2 + d3] * m);
              e += (d1 ? -Jv[d2 + d3] : Jv[d2 + d3]) * s1;
              e += (d2 ? -Jv[d1 + d3] : Jv[d1 + d3]) * s2v;
              e += (d3 ? -Jv[d1 + d2] : Jv[d1 + d2]) * s3;
              const int dx = p + bx - i, dy = q + by - j, dz = r + bz - k;
              c[(dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)] += e;
            }
      }
    }
  }
}

// A slab of the DD level (Sec. 2.1, subdomains): x layers x0..x0+nl-1 of
// the level, its own operator view, and the offsets of its factors.
struct Slab3 {
  int x0;         // first global layer (1-based)
  int nl;         // layers
  int n;          // unknowns per block, nl m3
  Level3 op;      // the slab operator A^(j)
  size_t fac_off; // element offset (complex64) of its factors
};

// Factor storage of a slab, complex64, per block t = 0..m2-1:
//   W_t = [G_t | M_t] (n x 2n, row major): G_t = S_t^{-1}, M_t = -G_t L_t,
//   E_t = G_t U_t (n x n, row major),
// with S_t the Schur complements of the block LU along y, L_t and U_t the
// couplings of block t to blocks t-1 and t+1.  Forward substitution:
// y_t = G_t f_t + M_t y_{t-1}; backward: x_t = y_t - E_t x_{t+1}.
inline size_t slab3_factor_elems(int n, int m2) { return (size_t)3 * n * n * m2; }

// One SubdomSolve task of a stage (the fields of TaskDev that the 3-D
// stage uses, with the same meaning).
using TaskDev = hsp::TaskDev;

// ---- kernels (stencil3d.hip) ------------------------------------------------
// y = A x (mode 0), y = b - A x (mode 1), y = x + w D^{-1} (b - A x) (mode 2,
// x == nullptr: x = 0).  Ta is the arithmetic type; Tx, Tb, Ty the storage
// types.
template <class Ta, class Tx, class Tb, class Ty>
void launch_stencil3(const Level3& L, int mode, const cx<Tx>* x, const cx<Tb>* b, cx<Ty>* y, double w,
                     hipStream_t s);

// Tensor-product transfers between the fine grid and the PML-aware coarse
// grid (Sec. 4): per axis, coarse unknown I gathers from up to 3 fine
// unknowns (r[a][3 I + q], weights rw) and fine unknown i from up to 2
// coarse unknowns (p[a][2 i + q], weights pw); index -1 = none.
struct Transfer3 {
  int nf[3], nc[3];
  const int* r[3];
  const double* rw[3];
  const int* p[3];
  const double* pw[3];
};
template <class Tin, class Tout>
void launch_restrict3(const Transfer3& T, const cx<Tin>* rf, cx<Tout>* rc, hipStream_t s);
template <class Tc, class Tf>
void launch_prolong_add3(const Transfer3& T, const cx<Tc>* ec, cx<Tf>* xf, hipStream_t s);

// b = h^3 f / (alpha_1 alpha_2 alpha_3) at the fine unknowns (ib[a] = 1/alpha
// at the nodes 0..m_a+1)
void launch_rhs3(int m1, int m2, int m3, double h3, const cd* ib0, const cd* ib1, const cd* ib2, const cd* f, cd* b,
                 hipStream_t s);
// cell k^2 as the tensor product of 1-D 3-tap averages of the node values
// (boundary nodes take the nearest unknown node's value)
void launch_cell_average3(const double* k2n, const int m[3], const int* x0[3], const double* w[3], const int nc[3],
                          double* k2c, hipStream_t s);
// cell coefficients c1..c5 of Table (b) at 1/G = h_nom k / (2 pi)
void launch_cell_coefs3(const double* k2c, size_t ncell, double h_nom, double* coef, hipStream_t s);

// ---- dense partial Gauss-Jordan elimination (slab3d.hip) -------------------
// One job: the nf x nf complex64 matrix F (row stride ld) whose first s
// columns are eliminated with partial pivoting among rows 0..s-1:
//   [F11 F12; F21 F22]  ->  [F11^-1  F11^-1 F12; -F21 F11^-1  F22 - F21 F11^-1 F12]
// (the row interchanges leave the first s columns permuted: column j of the
// result is column col[j] of F after the elimination).  s = nf inverts F.
// Scratch per job: piv, col (s ints), brow (32 x ld: pivot rows of the
// current panel), spr (32 x 32: the scaled pivot row of every step of the
// current panel, replayed on the rows >= s).
struct GJob {
  cf* F;
  int nf, s, ld;
  int* piv;
  int* col;
  cf* brow;
  cf* spr;
};
// Eliminates the first s columns of every job of the device array (the
// launches cover all jobs; s_max, b_max and nf_max bound s, nf - s and nf over
// the jobs).  status[0] |= 1 for a zero or non-finite pivot.
void launch_gauss_jordan(const GJob* jobs, int njobs, int s_max, int b_max, int nf_max, int* status, hipStream_t s);
constexpr int kGJMaxPivots = 1536;  // s <= 1024 rows in registers + 512 in LDS

// ---- slab factorization and stage (slab3d.hip) ----------------------------
// Setup of all slabs, block by block along y (see slab3d.hip).  Scratch:
// per slab n_max^2 complex64 (S), n_max 27 complex64 (block coefficients),
// 32 n_max complex64 (pivot rows), 32 x 32 complex64 (panel steps), n_max
// ints (pivots, column permutation), one GJob; status[0] |= 1 for a zero or
// non-finite pivot; growth[slab] = max |S_t| / max |D_t|.
struct Setup3 {
  const Slab3* slabs;  // device array
  int nslabs, n_max, m2;
  cf* factors;
  cf* S;       // [slab][n_max][n_max]
  cf* coef;    // [slab][n_max][27]
  cf* brow;    // [slab][32][n_max]
  cf* spr;     // [slab][32][32]
  int* piv;    // [slab][n_max]
  int* col;    // [slab][n_max]
  GJob* jobs;  // [slab]
  double* gmax;  // [slab][2] running max |D|^2, |S|^2
  int* status;
  int dbg_singular;
};
size_t setup3_scratch_bytes(int nslabs, int n_max);
// Fills the job table of Su (host array jobs_host, uploaded by the caller
// to Su.jobs) for the slab sizes n[slab].
void setup3_jobs(const Setup3& Su, const int* n, GJob* jobs_host);
void launch_factor3(const Setup3& Su, hipStream_t s);
void finish_growth3(const Setup3& Su, double* growth, hipStream_t s);

// ---- nested-dissection slab factorization (nd3d.hip) ----------------------
// The (y, z) plane of a slab is cut recursively by lines of nodes (the
// longer side of a rectangle is halved; rectangles of at most kNDLeaf nodes
// are leaves), every cut running through all n_l x-layers.  Each tree node
// is a front: its separator (the cut line, or the whole leaf rectangle) and
// its ring (the nodes of the ancestors' separators next to its rectangle:
// the in-domain nodes of the one-node border around it).  With a stencil
// that couples nodes at most one apart in y and z, the separator couples
// only to its own region and to the ring, so eliminating the fronts from
// the leaves up is block Gaussian elimination in a nested-dissection order
// (multifrontal: the Schur complement of a front is added into its
// parent's front).  Front variables: the separator's n_l ns unknowns
// (x_l ns + point) first, then the ring's n_l nb (x_l nb + point).
constexpr int kNDLeaf = 9;         // nodes per leaf rectangle (at most)
constexpr int kNDMaxFront = 2048;  // unknowns per front

struct NDGeom {       // one front of the plane (shared by all slabs)
  int ns, nb;         // separator and ring nodes
  int pt_off;         // pts[pt_off + P], P < ns + nb: plane index y m3 + z
  int y0, z0, h, w;   // the front's rectangle
  int lmap_off;       // lmap[lmap_off + (y - y0 + 1)(w + 2) + z - z0 + 1]: front point of node (y, z) or -1
  int child[2];       // child fronts (-1: none)
  int chmap_off[2];   // chmap[chmap_off[c] + P]: ring index in child c of front point P, or -1
  int cmap_off;       // cmap[cmap_off + q]: parent front point of ring point q
  int level;          // depth from the root (0)
};

// Per slab and front: factor offsets (complex64 elements) of
//   GN = [F11^-1 ; -F21 F11^-1]   (nf x s, row stride s + (s & 1)) and
//   E  = F11^-1 F12               (s x b, row stride b + (b & 1)),
// the offset of the front's update vector (b entries) in a task's scratch,
// the offset of its gather maps in NDSolve::maps (s + b + 2 nf ints: the
// slab-layout positions of the separator and ring unknowns, then for every
// front unknown the positions of the two children's update-vector entries
// that add to it, -1 for none) and (setup only) its dense front matrix.
struct NDFront {
  size_t gn, e, u, m;
  cf* F;
};
struct NDJob {
  int slab, front;
};

// Device view of the plan for the stage kernels.  Items are (front, first
// row) pairs, a level-dependent number of rows per workgroup: forward items
// cover the nf rows of GN, backward items the s rows of E (fronts with a
// ring); the tables give (offset, count) per slab and level.
struct NDSolve {
  const NDGeom* geom;
  const int* maps;
  const NDFront* fr;  // [slab][front]
  int nfronts, depth;
  const int2* items;
  const int* fwd_tab;  // [slab][level][2]
  const int* bwd_tab;
  cf* U;               // [task][u_stride]
  size_t u_stride;
};

// Host plan of the dissection of an m2 x m3 plane.
struct NDPlan {
  int m2 = 0, m3 = 0, depth = 0;
  std::vector<NDGeom> fronts;
  std::vector<int> pts, lmap, chmap, cmap;
  std::vector<std::vector<int>> levels;  // front indices per level (0: root)
};
// Builds the plan; returns false (with *why) if it breaks an invariant.
bool nd_plan(int m2, int m3, NDPlan& P, std::string* why);

// Sizes per slab of n_l layers.
struct NDSizes {
  size_t factor = 0;   // complex64 elements of GN and E over all fronts
  size_t update = 0;   // complex64 elements of the update vectors
  size_t rows = 0;     // forward items (workgroups) over all levels
  int s_max = 0, b_max = 0, nf_max = 0;
};
NDSizes nd_sizes(const NDPlan& P, int nl);

// Setup scratch of the multifrontal factorization, carved by the caller:
// two level buffers of dense fronts (levels alternate), the Gauss-Jordan
// scratch of the largest level, the job tables.
struct NDSetup {
  const Slab3* slabs;        // device
  const NDGeom* geom;        // device
  const int* pts;
  const int* lmap;
  const int* chmap;
  const int* cmap;
  NDFront* fr;               // device [slab][front]
  int nslabs, nfronts, m2, m3, n_max;
  cf* coef;                  // [slab][m2 n][27]: coefficient rows of every slab
  const size_t* coef_off;    // device [slab]: element offset into coef
  cf* factors;
  const NDJob* jobs;         // device, all levels
  GJob* gjobs;               // device, all levels
  double* gmax;              // [slab][2]: max |A|^2, max |F11|^2
  int* status;
  int dbg_slab, dbg_front;   // a separator block forced to zero (-1: off)
};
// Host description of the levels for the launches.
struct NDLevelHost {
  int first_job = 0, njobs = 0;  // into the job tables
  int s_max = 0, b_max = 0, nf_max = 0;
  int fwd_items = 0, bwd_items = 0;  // max over slabs (grid size)
  int fwd_g = 64, fwd_np = 1;        // lanes per row and pairs per lane of the substitutions
  int bwd_g = 64, bwd_np = 1;
  int fwd_rows() const { return 4 * 64 / fwd_g; }  // rows per workgroup
  int bwd_rows() const { return 4 * 64 / bwd_g; }
};
// Lanes per row and pairs of complex entries per lane for rows of n entries.
void nd_row_shape(int n, int* g, int* np);
void launch_factor_nd(const NDSetup& Su, const std::vector<NDLevelHost>& lv, hipStream_t s);

// One SubdomSolve stage of the 3-D sweep: ntasks tasks, each a slab solve
// (gather + transmission injection, block substitutions along y, scatter-
// add, transmission extraction).  f, g, u: level vectors; bufs: 2 buffers x
// 2 layers x m2 m3; fs, ys: slab scratch per task slot, [m2][n_max] each.
struct Stage3 {
  const TaskDev* tasks;  // device, ntasks
  const Slab3* slabs;    // device
  Level3 G;              // the level operator (transmission couplings)
  int ntasks, n_max, nl_max;
  const cf* f;
  const cf* g;
  cf* u;
  cf* bufs;
  cf* fs;
  cf* ys;
  const cf* factors;
  // nested-dissection factors: the substitutions of the stage run level by
  // level through the fronts instead of block by block along y
  const NDSolve* nd;                      // host pointer, or nullptr
  const std::vector<NDLevelHost>* nd_lv;  // host
};
// Enqueues the stage (one launch per block step, or per level of the
// dissection and direction); returns the launch status.
hipError_t launch_stage3(const Stage3& st, hipStream_t s);
// The level-synchronous substitutions of the nested-dissection factors
// (forward: leaves to root, backward: root to leaves) on the slab-layout
// right-hand sides of the stage (nd3d.hip).
void launch_nd_solve(const Stage3& st, const NDSolve& nd, const std::vector<NDLevelHost>& lv, hipStream_t s);

}  // namespace d3
}  // namespace hsp
