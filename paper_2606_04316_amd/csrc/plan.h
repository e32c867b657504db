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
  DBuf<int32_t> code;  // per row: pair code of Cartesian bases (else empty)
  int nK = 1;
  // row layout of D~ and V for the current column chunk: nK blocks of ldK
  // columns (ld = nK ldK), packed to the chunk's width; ld_cap = the allocation
  int64_t ldK = 0, ld = 0, ld_cap = 0;
  DBuf<double> D, V, Dmax, Qmax, Bmax, Dtmax;
  // intra-tile row order of the current transform (rows ranked by Q Dmax
  // within each tile) and the row data of the integral tiles in that order
  DBuf<int32_t> perm, wcls, wmu, wnu, wcode;
  DBuf<double> sthr, wQ, wDmax;
  DBuf<int64_t> wrow_first;
  PairStore wpp;
  DBuf<unsigned long long> steps;  // first-half steps of the task lists (eager)
  unsigned long long h_steps = 0;
  // mixed precision: per-tier sub-lists of the directed tasks
  DBuf<int32_t> ttasks, trank, tdesc, tcount, toff;
  DBuf<float> Dlo;  // scaled FP32 copy of D~ (the reduced tiers' density operand)
  std::vector<int32_t> h_tcount;
  DBuf<int32_t> count, tasks, task_bra;
  DBuf<int64_t> slot_base;
  DBuf<double> panel;
  DBuf<double> panel3;  // gauge tiles, six per slot (L-S space of DCB plans)
  int64_t panel_slots = 0;
  // panel of the plain integral tiles: FP64 DCB plans have none of their own
  // and use the gauge panel's memory (the fused Breit tiles replace them; a
  // Gaunt-only transform regenerates its tiles there)
  double *pan() const { return panel.p ? panel.p : panel3.p; }
  DBuf<unsigned long long> kept;
  DBuf<int64_t> dtotal;     // device copy of the kept-tile total (graph mode)
  DBuf<int32_t> overflow;   // set when the kept tiles exceed the panel (graph mode)
  // unique tile pairs (b >= k) of the symmetric integral matrix: one computed
  // tile fills both directed tiles (b, k) and (k, b); dmap = directed slot map
  DBuf<int32_t> ucount, utask_k, utask_b, uslot_bk, uslot_kb, dmap;
  DBuf<int64_t> ubase, udtotal;  // udtotal: device unique-tile total (graph mode)
  DBuf<int32_t> uoverflow;       // set when the unique tiles exceed the panel (graph mode)
  // persistent integral schedule: unique tasks longest first, and the class
  // counts / offsets / queue counter that build and consume that order
  DBuf<int32_t> uorder;
  DBuf<unsigned long long> lpt;
  // per eager transform
  std::vector<int32_t> cnt, ucnt;
  std::vector<int64_t> base, ub;
  int64_t total = 0, utotal = 0;
  bool sym = false;  // this transform computes unique tiles (all directed tiles resident)

  size_t bytes() const {
    return cls.bytes() + mu.bytes() + nu.bytes() + row_first.bytes() + Q.bytes() + pp.bytes() +
           code.bytes() + perm.bytes() + wcls.bytes() + wmu.bytes() + wnu.bytes() + wcode.bytes() +
           sthr.bytes() +
           wQ.bytes() + wDmax.bytes() + wrow_first.bytes() + wpp.bytes() + steps.bytes() +
           D.bytes() + V.bytes() + Dmax.bytes() + Qmax.bytes() + Bmax.bytes() + Dtmax.bytes() +
           ttasks.bytes() + trank.bytes() + tdesc.bytes() + tcount.bytes() + toff.bytes() +
           Dlo.bytes() + count.bytes() +
           tasks.bytes() + task_bra.bytes() + slot_base.bytes() + panel.bytes() + panel3.bytes() + kept.bytes() +
           dtotal.bytes() + overflow.bytes() + ucount.bytes() + utask_k.bytes() +
           utask_b.bytes() + uslot_bk.bytes() + uslot_kb.bytes() + dmap.bytes() + ubase.bytes() + udtotal.bytes() +
           uoverflow.bytes() + uorder.bytes() + lpt.bytes();
  }
};

}  // namespace qdcb

struct qdcb_plan;

namespace qdcb {
// Sized buffers of a plan (plan.hip).
void size_plan(qdcb_plan &p, int64_t slotsC, int64_t slotsG);
bool ensure_residency(qdcb_plan &p, double slack);
// Why a set of launch choices is not valid for the plan, or NULL (tune.hip).
const char *tune_problem(const qdcb_plan &p, const qdcb_tune &t);
}  // namespace qdcb

struct qdcb_plan {
  qdcb_ctx *ctx = nullptr;
  int64_t nLL = 0, nSS = 0;  // pair counts of the bases (plans do not keep basis pointers)
  qdcb_plan_desc desc{};
  int n = 0, NL = 0, NS = 0;
  int npair_mo = 0;
  int64_t ncol = 0;  // 4 * npair_mo
  // general two-spinor plan: n spinors, npair_s pairs c <= d, npair_mo groups
  // of two pairs (four columns: re, im of each)
  bool spinor = false;
  int npair_s = 0;
  int ci = 0;        // MO pairs (spinor mode: groups) per column chunk of the first half
  int mo_batch = 0;  // > 0: MO-driven variant, batches of that many MO pairs
  // first-half MFMA work of the last enqueued transform: row widths summed over
  // the chunks per space, and (MO-driven) width x kept tiles summed per batch
  double ld_sum[2] = {0.0, 0.0};
  double mo_work = 0.0;
  int chunks_run = 0;  // column chunks (MO-driven: batches) of the last transform
  int sc = 0;        // columns per second-half slice
  bool gaunt = false;      // L-S space (Gaunt term; DCG and DCB)
  bool gauge = false;      // gauge term of the Breit operator (DCB)
  bool fused_breit = false;  // FP64 DCB: Gaunt + gauge from one set of Breit tiles
  qdcb_tune tune{};       // launch choices (tile shapes, schedules)
  int n_cu = 0;           // compute units of the device
  std::string tune_key;   // shape key of the tuning cache
  qdcb::Space C, G;
  qdcb::DBuf<int32_t> rs, rowmapL, rowmapS, rowmapLS;
  qdcb::DBuf<double> CLd, CSd, Gd;
  qdcb::DBuf<double> CallL, CallS, ChatL, ChatS;
  qdcb::DBuf<double> AhatK[3], BhatK[3];
  qdcb::DBuf<double> W, Gc;
  qdcb::DBuf<double> Gb;         // block output of qdcb_transform_blocks (made on first use)
  std::vector<double> h_Gb;      // its host copy (host-pointer mode)
  int classes = 3;               // integral classes of the last transform (1 Coulomb, 2 Gaunt,
                                 // 4 gauge)
  std::atomic<int> busy{0};      // a call is using the plan
  qdcb::DBuf<double> boys;   // Taylor table of the Boys function F0
  qdcb::DBuf<double> boys3;  // F0 .. F9 on the same grid (gauge tiles)
  bool cart = false;         // a basis has Cartesian (p, d, f) functions
  bool gen = false;          // a basis has d or f functions: the general integral tiles
  bool gen_f = false;        // ... and f functions (the general tiles' largest orders)
  // integral tiles in the intra-tile row order of each transform, first half
  // skipping masked 16-row steps (environment QDCB_TILE_ORDER=0 at plan
  // creation turns it off, for comparisons)
  bool tile_order = true;
  qdcb::DBuf<double> boysc;  // F0 .. F11 on the same grid (Cartesian tiles)
  qdcb::DBuf<double> boysg;  // F0 .. F19 on the same grid (general tiles: d or f functions)
  bool have_last = false;
  int64_t tiles_made = 0;  // integral tiles generated by the last eager transform
  int v_i0 = 0, v_i1 = 0;  // MO pairs whose first-half columns V holds (last chunk)
  // captured transform (re-transforms with new coefficients in the same buffers)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const double *g_CL = nullptr, *g_CS = nullptr;
  double *g_G = nullptr;
  bool g_sym = false;  // the captured transform uses unique tiles
  // side stream for integral tiles, overlapping the MFMA contraction of the
  // previous batch (default priority)
  hipStream_t side = nullptr;

  // an event after the last work a call enqueued on each stream the plan used
  // (destruction waits for these instead of the whole device)
  std::vector<std::pair<hipStream_t, hipEvent_t>> stream_events;
  void mark_stream(hipStream_t s) {
    for (auto &se : stream_events)
      if (se.first == s) {
        (void)hipEventRecord(se.second, s);
        return;
      }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    stream_events.emplace_back(s, e);
  }
  ~qdcb_plan() {
    for (auto &se : stream_events) (void)hipEventDestroy(se.second);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace qdcb {
// Records the plan's stream event when the scope ends (after the work a call
// enqueued on s).
struct StreamMark {
  qdcb_plan &p;
  hipStream_t s;
  ~StreamMark() { p.mark_stream(s); }
};
// Exclusive use of a plan for the duration of one call: a second call on the
// same plan meanwhile (another thread, or a callback of the first) fails with
// QDCB_E_BUSY instead of racing.
struct PlanUse {
  qdcb_plan &p;
  explicit PlanUse(const qdcb_plan &pl) : p(const_cast<qdcb_plan &>(pl)) {
    int idle = 0;
    if (!p.busy.compare_exchange_strong(idle, 1))
      fail(QDCB_E_BUSY, "the plan is in use by another call");
  }
  ~PlanUse() { p.busy.store(0); }
  PlanUse(const PlanUse &) = delete;
  PlanUse &operator=(const PlanUse &) = delete;
};
}  // namespace qdcb
