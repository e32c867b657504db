// plan.h -- plan objects of the qdcb runtime (internal).
#pragma once

#include "runtime.h"

namespace qdcb {

// Primitive pairs whose Schwarz weight is below 1e-17 of their row's mean are
// dropped (bounded effect: ~1e-17 of the sum of absolute primitive terms).
constexpr double PRIM_EPS = 1e-17;

// One integral-class pair space: Coulomb (LL and SS pairs) or Gaunt (LS pairs).
struct Space {
  int gaunt = 0;
  int64_t P = 0, Ppad = 0;
  int ntiles = 0;
  std::vector<int32_t> h_cls, h_mu, h_nu;
  std::vector<int64_t> h_key;  // canonical index (Coulomb) or mu*NS + nu (Gaunt)
  DBuf<int32_t> cls, mu, nu;
  DBuf<int64_t> row_first;
  DBuf<double> Q;
  PairStore pp;
  int nK = 1;
  int64_t ldK = 0, ld = 0;
  DBuf<double> D, V, Dmax, Qmax, Bmax;
  DBuf<int32_t> count, tasks, task_bra;
  DBuf<int64_t> slot_base;
  DBuf<double> panel;
  int64_t panel_slots = 0;
  DBuf<unsigned long long> kept;
  DBuf<int64_t> dtotal;     // device copy of the kept-tile total (graph mode)
  DBuf<int32_t> overflow;   // set when the kept tiles exceed the panel (graph mode)
  // per eager transform
  std::vector<int32_t> cnt;
  std::vector<int64_t> base;
  int64_t total = 0;

  size_t bytes() const {
    return cls.bytes() + mu.bytes() + nu.bytes() + row_first.bytes() + Q.bytes() + pp.bytes() +
           D.bytes() + V.bytes() + Dmax.bytes() + Qmax.bytes() + Bmax.bytes() + count.bytes() +
           tasks.bytes() + task_bra.bytes() + slot_base.bytes() + panel.bytes() + kept.bytes() +
           dtotal.bytes() + overflow.bytes();
  }
};

}  // namespace qdcb

struct qdcb_plan {
  qdcb_ctx *ctx = nullptr;
  int64_t nLL = 0, nSS = 0;  // pair counts of the bases (plans do not keep basis pointers)
  qdcb_plan_desc desc{};
  int n = 0, NL = 0, NS = 0;
  int npair_mo = 0;
  int64_t ncol = 0;  // 4 * npair_mo
  int ci = 0;        // MO pairs per column chunk of the first half
  int sc = 0;        // columns per second-half slice
  bool gaunt = false;
  qdcb::Space C, G;
  qdcb::DBuf<int32_t> rs, rowmapL, rowmapS, rowmapLS;
  qdcb::DBuf<double> CLd, CSd, Gd;
  qdcb::DBuf<double> CallL, CallS, ChatL, ChatS;
  qdcb::DBuf<double> AhatK[3], BhatK[3];
  qdcb::DBuf<double> Vfull, W, Gc;
  bool have_last = false;
  // captured transform (re-transforms with new coefficients in the same buffers)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const double *g_CL = nullptr, *g_CS = nullptr;
  double *g_G = nullptr;
  // side stream for integral tiles, overlapping the MFMA contraction of the
  // previous batch (default priority)
  hipStream_t side = nullptr;

  ~qdcb_plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (side) (void)hipStreamDestroy(side);
  }
};
