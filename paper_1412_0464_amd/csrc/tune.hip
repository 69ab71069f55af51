// Autotuner of the batched solvers: chunk length of the slab substitutions
// (fixed at setup: the chunk transfer matrices depend on it) and right-hand-
// side tile of the stage launches, chosen jointly by timing.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ctx.h"

namespace hsp {
namespace {

// Candidate chunk lengths with distinct chunk counts for n2 tangential nodes.
std::vector<int> chunk_candidates(int n2) {
  static const int cand[] = {16, 20, 24, 28, 34, 40, 48, 64};
  std::vector<int> out;
  int last_p = -1;
  for (int m : cand) {
    const int mm = std::min(m, n2);
    const int p = (n2 + mm - 1) / mm;
    if (p == last_p) continue;
    last_p = p;
    out.push_back(mm);
  }
  return out;
}

}  // namespace
}  // namespace hsp

using namespace hsp;

extern "C" {

hsp_status hsp_autotune_workspace_size(const hsp_grid* grid, int J, const hsp_options* opt, int nrhs, int restart,
                                       size_t* ws_bytes, size_t* bws_bytes) {
  if (!grid || !opt || !ws_bytes || !bws_bytes) return fail(HSP_EINVAL, "null argument");
  if (grid->dim == 3) return fail(HSP_EINVAL, "the autotuner is implemented for 2-D problems");
  if (nrhs < 1 || restart < 1) return fail(HSP_EINVAL, "nrhs and restart must be >= 1");
  Plan P0;
  hsp_status st = make_plan(grid, J, opt, P0);
  if (st != HSP_OK) return st;
  *ws_bytes = 0;
  *bws_bytes = 0;
  for (int m : chunk_candidates(P0.dd_n2)) {
    hsp_options o = *opt;
    o.chunk = m;
    hsp_ctx tmp;  // host-only: plan and schedule
    if ((st = make_plan(grid, J, &o, tmp.P)) != HSP_OK) return st;
    tmp.opt = o;
    tmp.grid = *grid;
    tmp.J = J;
    build_schedule(&tmp);
    hsp_handle h = &tmp;
    size_t b = 0;
    if ((st = hsp_group_workspace_size(1, &h, &nrhs, restart, &b)) != HSP_OK) return st;
    *ws_bytes = std::max(*ws_bytes, tmp.P.total);
    *bws_bytes = std::max(*bws_bytes, b);
  }
  return HSP_OK;
}

hsp_status hsp_autotune(const double* c_dev, double omega, const hsp_grid* grid, int J, const hsp_options* opt,
                        int nrhs, int restart, void* ws, size_t ws_bytes, void* bws, size_t bws_bytes,
                        int* chunk_out, int* tile_out, double* ms_out, double* table, int* ntable, void* stream) {
  if (!grid || !opt) return fail(HSP_EINVAL, "null argument");
  if (grid->dim == 3) return fail(HSP_EINVAL, "the autotuner is implemented for 2-D problems");
  Plan P0;
  hsp_status st = make_plan(grid, J, opt, P0);
  if (st != HSP_OK) return st;
  int best_m = 0, best_t = 0, n = 0;
  double best_ms = 1e300;
  for (int m : chunk_candidates(P0.dd_n2)) {
    hsp_options o = *opt;
    o.chunk = m;
    hsp_handle hd = nullptr;
    if ((st = hsp_setup(c_dev, omega, grid, J, &o, ws, ws_bytes, stream, &hd)) != HSP_OK) return st;
    int t = 0;
    double ms = 0;
    st = hsp_tune_batch(hd, nrhs, restart, bws, bws_bytes, &t, &ms, stream);
    hsp_destroy(hd);
    if (st != HSP_OK) return st;
    if (table && n < 8) {
      table[3 * n] = m;
      table[3 * n + 1] = t;
      table[3 * n + 2] = ms;
    }
    ++n;
    if (ms < best_ms) {
      best_ms = ms;
      best_m = m;
      best_t = t;
    }
  }
  if (chunk_out) *chunk_out = best_m;
  if (tile_out) *tile_out = best_t;
  if (ms_out) *ms_out = best_ms;
  if (ntable) *ntable = std::min(n, 8);
  return HSP_OK;
}

}  // extern "C"
