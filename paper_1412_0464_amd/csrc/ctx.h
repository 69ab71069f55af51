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

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return hsp::fail(HSP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

using cplx = std::complex<double>;

inline cd to_cd(cplx z) { return mk<double>(z.real(), z.imag()); }

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
  size_t tsize = 16;                      // bytes per preconditioner complex
  int m = 0;                              // FGMRES restart
  // workspace offsets
  size_t o_fxA, o_fxB, o_fyA, o_fyB, o_k2n, o_fk2c, o_fcoef, o_ixn, o_iyn;
  size_t o_cxA, o_cxB, o_cyA, o_cyB, o_ck2c, o_ccoef;
  size_t o_avgx0, o_avgwx, o_avgy0, o_avgwy;
  size_t o_rx, o_rwx, o_ry, o_rwy, o_px, o_pwx, o_py, o_pwy;
  size_t o_slabs, o_slabA, o_slabB, o_xmap, o_fac, o_facscr, o_status, o_tasks, o_tcoef;
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

struct hsp_ctx {
  hsp::Plan P;
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

}  // namespace hsp
