// transform.hip -- C ABI: the transformation driver, eager and captured.
//
// One transformation enqueues the paper's four stages (Sec. 3.3.1) on the
// caller's stream: quaternion densities and their bound, screening (task
// lists), AO integral tiles with the first-half contraction, and the second
// half.  Eager mode reads the per-bra-tile counts of kept tiles back to the
// host to size batches that fit the integral panel.  Captured mode keeps every
// step on the device (device-side scan of the counts, one batch, fixed launch
// sizes, no memsets) so the whole transformation can be recorded once into a
// hipGraph and replayed for re-transforms with new coefficients written into
// the same buffers; a replay whose kept tiles exceed the panel sets a flag
// and is redone eagerly.
//
// The autotuner times the launch choices of a plan (integral schedule,
// first-half workgroup order, second-quarter tile) on the plan's own workload,
// one column chunk per trial, and keeps the faster value of each.
#include <cstdlib>
#include <limits>

#include "plan.h"

using namespace qdcb;

namespace {

void check_finite_host(const double *x, size_t n, const char *what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) fail(QDCB_E_INVALID, std::string("non-finite value in ") + what);
}

enum { ST_DENS = 0, ST_SCREEN = 1, ST_ERI = 2, ST_FH = 3, ST_SH = 4, ST_FH32 = 5, ST_FH16 = 6 };

// Stage timing with events read back after the final synchronization;
// disabled (null) while a graph is being captured.
struct StageTimer {
  hipStream_t s;
  bool on;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  hipEvent_t open = nullptr;
  int open_stage = -1;
  bool probe_only = false;  // densities and screening only (sizing before a capture)
  int max_chunks = 0;       // > 0: stop after that many MO-pair column chunks (tuning runs)
  StageTimer(hipStream_t st, bool enabled) : s(st), on(enabled) {}
  ~StageTimer() {
    for (auto e : sync_events) (void)hipEventDestroy(e);
    for (auto &m : marks) {
      (void)hipEventDestroy(m.second.first);
      (void)hipEventDestroy(m.second.second);
    }
    if (open) (void)hipEventDestroy(open);
  }
  void begin(int stage, hipStream_t st = nullptr) {
    if (!on) return;
    HIPC(hipEventCreate(&open));
    HIPC(hipEventRecord(open, st ? st : s));
    open_stage = stage;
  }
  void end(hipStream_t st = nullptr) {
    if (!on) return;
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    HIPC(hipEventRecord(e, st ? st : s));
    marks.push_back({open_stage, {open, e}});
    open = nullptr;
  }
  // ordering events (no timing), destroyed with the timer after the final sync
  std::vector<hipEvent_t> sync_events;
  hipEvent_t record(hipStream_t st) {
    hipEvent_t e;
    HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    sync_events.push_back(e);
    HIPC(hipEventRecord(e, st));
    return e;
  }
  double total(int stage) {
    double t = 0;
    for (auto &m : marks)
      if (m.first == stage) {
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, m.second.first, m.second.second));
        t += ms;
      }
    return t;
  }
  int launches(int stage) {
    int c = 0;
    for (auto &m : marks) c += m.first == stage;
    return c;
  }
};

// The bound pass (bound_only) reads the rows in their own order (Dmax by
// row); the density rows are written in the transform's intra-tile order.
void density(qdcb_plan &p, Space &sp, const double *dCL, const double *dCS, int bound_only,
             int i0, int i1, hipStream_t s) {
  const bool w = p.tile_order && !bound_only;
  DensityArgs da;
  da.gaunt = sp.gaunt;
  da.bound_only = bound_only;
  da.nrows = sp.Ppad;
  da.n = p.n;
  da.npair_mo = p.npair_mo;
  da.i0 = i0;
  da.i1 = i1;
  da.ld = sp.ld;
  da.ldK = sp.ldK;
  da.cls = w ? sp.wcls.p : sp.cls.p;
  da.mu = w ? sp.wmu.p : sp.mu.p;
  da.nu = w ? sp.wnu.p : sp.nu.p;
  da.CL = dCL;
  da.CS = dCS;
  da.NL = p.NL;
  da.NS = p.NS;
  da.rs = p.rs.p;
  da.D = sp.D.p;
  da.Dmax = sp.Dmax.p;
  da.spinor = p.spinor ? 1 : 0;
  da.nspair = p.npair_s;
  launch_density(da, s);
  HIPC(hipGetLastError());
}

// Intra-tile row order after a density bound: rows ranked by Q Dmax within
// each tile, and the integral tiles' row data gathered in that order.
void order_rows(qdcb_plan &p, Space &sp, hipStream_t s) {
  if (!p.tile_order) return;
  launch_tile_order(sp.ntiles, sp.Q.p, sp.Dmax.p, sp.perm.p, sp.sthr.p, s);
  launch_gather_rows(sp.ntiles, sp.perm.p, sp.Q.p, sp.Dmax.p, sp.cls.p, sp.mu.p, sp.nu.p,
                     p.cart ? sp.code.p : nullptr, sp.row_first.p, sp.pp.cview(), sp.wQ.p,
                     sp.wDmax.p, sp.wcls.p, sp.wmu.p, sp.wnu.p, p.cart ? sp.wcode.p : nullptr,
                     sp.wrow_first.p, sp.wpp.view(), s);
  HIPC(hipGetLastError());
}

// Task lists of one space.  Eager: counts to the host, batches sized there.
// Captured: device-side scan, one batch of at most panel_slots tiles.  When
// every directed tile fits the panel (and the plan allows it), the unique
// tile pairs are listed as well, each with its two directed slots.
void screen(qdcb_plan &p, Space &sp, bool captured, hipStream_t s, bool zero_kept = true) {
  const bool want_sym = !(p.desc.flags & QDCB_PLAN_DIRECTED_TILES);
  launch_tile_bounds(sp.ntiles, sp.Q.p, sp.Dmax.p, sp.Qmax.p, sp.Bmax.p, sp.Dtmax.p, s);
  launch_screen_count(sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.count.p, s);
  HIPC(hipGetLastError());
  if (captured) {
    launch_scan_counts(sp.ntiles, sp.count.p, sp.slot_base.p, sp.dtotal.p, sp.panel_slots,
                       sp.overflow.p, s);
  } else {
    sp.cnt.resize(sp.ntiles);
    HIPC(hipMemcpyAsync(sp.cnt.data(), sp.count.p, sp.cnt.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    sp.base.resize(sp.ntiles);
    sp.total = 0;
    for (int b = 0; b < sp.ntiles; ++b) {
      sp.base[b] = sp.total;
      sp.total += sp.cnt[b];
    }
    HIPC(hipMemcpyAsync(sp.slot_base.p, sp.base.data(), sp.base.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
    if ((int64_t)sp.tasks.n < sp.total) fail(QDCB_E_DEVICE, "task list capacity exceeded");
  }
  launch_screen_fill(0, sp.ntiles, sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.slot_base.p,
                     sp.tasks.p, sp.task_bra.p, s);
  if (zero_kept) launch_zero_u64(sp.kept.p, 4, s);
  HIPC(hipGetLastError());
  sp.h_steps = 4ull * (unsigned long long)sp.total;  // every task in full
  if (p.tile_order && !captured) {
    // the steps the first half runs with the intra-tile order (MFMA work)
    launch_zero_u64(sp.steps.p, 1, s);
    launch_step_work(sp.ntiles, sp.slot_base.p, sp.count.p, sp.tasks.p, sp.Qmax.p, sp.sthr.p,
                     p.desc.tau, sp.steps.p, s);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(&sp.h_steps, sp.steps.p, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
  }
  if (p.desc.prec == QDCB_PREC_MIXED) {
    launch_tier_split(sp.ntiles, sp.Qmax.p, sp.Bmax.p, sp.Dtmax.p,
                      p.tile_order ? sp.sthr.p : nullptr, p.desc.tau,
                      (p.desc.flags & QDCB_PLAN_TIER_BY_G) ? 1 : 0, p.desc.tier_fp32,
                      p.desc.tier_bf16, sp.slot_base.p, sp.count.p, sp.tasks.p, sp.ttasks.p,
                      sp.trank.p, sp.tdesc.p, sp.tcount.p, sp.toff.p, s);
    HIPC(hipGetLastError());
    if (!captured) {
      sp.h_tcount.resize(3 * (size_t)sp.ntiles);
      HIPC(hipMemcpyAsync(sp.h_tcount.data(), sp.tcount.p, sp.h_tcount.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    }
  }
  sp.sym = false;
  // directed slots are int32 in the slot map: panel_slots < 2^31 always holds.
  // Eager: the unique lists are built whenever the plan allows them; they are
  // used if every directed tile ends up resident (decided after screening).
  if (!want_sym) return;
  if (!captured && sp.total >= ((int64_t)1 << 31)) return;
  // a captured transform whose directed tiles outgrow the panel writes slots
  // beyond it into dmap; its integral and contraction kernels then do nothing
  launch_screen_fill_map(sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.slot_base.p,
                         sp.dmap.p, s);
  launch_screen_count_u(sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.ucount.p, s);
  HIPC(hipGetLastError());
  if (captured) {
    launch_scan_counts(sp.ntiles, sp.ucount.p, sp.ubase.p, sp.udtotal.p,
                       (int64_t)sp.utask_k.n, sp.uoverflow.p, s);
  } else {
    sp.ucnt.resize(sp.ntiles);
    HIPC(hipMemcpyAsync(sp.ucnt.data(), sp.ucount.p, sp.ucnt.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    sp.ub.resize(sp.ntiles);
    sp.utotal = 0;
    for (int b = 0; b < sp.ntiles; ++b) {
      sp.ub[b] = sp.utotal;
      sp.utotal += sp.ucnt[b];
    }
    if ((int64_t)sp.utask_k.n < sp.utotal) fail(QDCB_E_DEVICE, "unique task capacity exceeded");
    HIPC(hipMemcpyAsync(sp.ubase.p, sp.ub.data(), sp.ub.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  }
  launch_screen_fill_u(sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.ubase.p, sp.dmap.p,
                       sp.utask_k.p, sp.utask_b.p, sp.uslot_bk.p, sp.uslot_kb.p, s);
  if (p.tune.eri_sched == 1)  // persistent integral schedule: longest tiles first
    launch_lpt_order(captured ? 0 : sp.utotal, captured ? sp.udtotal.p : nullptr,
                     (int64_t)sp.utask_k.n, (int64_t)sp.utask_k.n, sp.utask_k.p, sp.utask_b.p,
                     sp.row_first.p, sp.lpt.p, sp.uorder.p, s);
  HIPC(hipGetLastError());
  sp.sym = captured || sp.total <= sp.panel_slots;
}

// gauge: the six-tile gauge panel and its table instead of the integral panel
// (breit: the fused Breit tiles)
EriTileArgs eri_args(qdcb_plan &p, Space &sp, int64_t slot0, bool count, bool gauge = false,
                     bool breit = false) {
  EriTileArgs ea;
  ea.tasks = sp.tasks.p;
  ea.task_bra = sp.task_bra.p;
  ea.slot0 = slot0;
  // the tiles' rows in the transform's intra-tile order (order_rows)
  const bool w = p.tile_order;
  ea.row_first = w ? sp.wrow_first.p : sp.row_first.p;
  ea.pp = w ? sp.wpp.cview() : sp.pp.cview();
  ea.Q = w ? sp.wQ.p : sp.Q.p;
  ea.Dmax = w ? sp.wDmax.p : sp.Dmax.p;
  ea.cls = w ? sp.wcls.p : sp.cls.p;
  ea.tau = p.desc.tau;
  ea.panel = gauge ? sp.panel3.p : sp.pan();
  ea.kept = count ? sp.kept.p : nullptr;
  ea.boys = p.boys.p;
  ea.boys3 = gauge ? p.boys3.p : nullptr;
  ea.code = p.cart ? (w ? sp.wcode.p : sp.code.p) : nullptr;
  ea.boysc = p.cart ? p.boysc.p : nullptr;
  // the general tiles: Coulomb tiles of bases with d or f functions, gauge
  // tiles of every Cartesian basis
  const bool general = p.gen || (p.cart && gauge);
  ea.boysg = general ? p.boysg.p : nullptr;
  ea.gen_tmax = p.gen_f ? 6 : (p.gen ? 4 : 2);
  if (general && !ea.boysg) fail(QDCB_E_DEVICE, "general tiles without their table");
  if (p.cart && (!ea.code || !ea.boysc || !sp.pp.pa.p || !sp.pp.ax.p))
    fail(QDCB_E_DEVICE, "Cartesian tiles without their codes, table or pair data");
  ea.gauge_diag = breit ? 0.5 : -0.5;
  if (gauge && !ea.boys3) fail(QDCB_E_DEVICE, "gauge tiles without their table");
  return ea;
}

FirstHalfArgs fh_args(qdcb_plan &p, Space &sp, int b0, int b1, int64_t slot0,
                      bool gauge = false) {
  FirstHalfArgs fa;
  if (p.tile_order) {
    fa.perm = sp.perm.p;
    fa.sthr = sp.sthr.p;
    fa.tau = p.desc.tau;
    fa.Qmax = sp.Qmax.p;
  }
  fa.b0 = b0;
  fa.b1 = b1;
  fa.slot_base = sp.slot_base.p;
  fa.count = sp.count.p;
  fa.tasks = sp.tasks.p;
  fa.slot0 = slot0;
  fa.panel = gauge ? sp.panel3.p : sp.pan();
  fa.D = sp.D.p;
  fa.V = sp.V.p;
  fa.ld = sp.ld;
  fa.ncol_tiles = (int)((gauge ? sp.ldK : sp.ld) / 128);  // gauge: per K block
  return fa;
}

// First-half contraction of bra tiles [fa.b0, fa.b1): FP64 plans in one
// launch; mixed plans as the FP64 tier (which stores V) followed by the FP32
// and BF16 tiers (which add to it).  Gauge term (gauge >= 0): one FP64
// launch over the directed lists in every precision mode, adding to V when
// gauge = 1 (after the Gaunt term) and storing when gauge = 0.
void contract(qdcb_plan &p, Space &sp, FirstHalfArgs fa, StageTimer &tm, hipStream_t s,
              int gauge = -1) {
  fa.plain_order = p.tune.fh_order;
  if (gauge >= 0) {
    tm.begin(ST_FH);
    launch_first_half_gauge(fa, sp.ldK, gauge, s);
    tm.end();
    HIPC(hipGetLastError());
    return;
  }
  if (p.desc.prec != QDCB_PREC_MIXED) {
    tm.begin(ST_FH);
    launch_first_half(fa, s);
    tm.end();
    HIPC(hipGetLastError());
    return;
  }
  fa.tasks = sp.ttasks.p;
  fa.rank = sp.trank.p;
  fa.Qmax = sp.Qmax.p;
  fa.tdesc = sp.tdesc.p;
  fa.Dlo = sp.Dlo.p;
  const int stage[3] = {ST_FH, ST_FH32, ST_FH16};
  for (int t = 0; t < 3; ++t) {
    fa.count = sp.tcount.p + (size_t)t * sp.ntiles;
    fa.toff = sp.toff.p + (size_t)t * sp.ntiles;
    tm.begin(stage[t]);
    if (t == 0)
      launch_first_half(fa, s);
    else
      launch_first_half_lp(fa, t, s);
    tm.end();
    HIPC(hipGetLastError());
  }
}

// Workgroups of the persistent integral launch: two per compute unit (the
// integral kernel's register and LDS use allow two resident 512-thread
// workgroups per compute unit).
int eri_queue_blocks(const qdcb_plan &p) { return 2 * std::max(p.n_cu, 1); }

// Mixed plans: the reduced-tier tiles of bra tiles [b0, b1), just made into
// the panel at slot0, are rounded in place once (FP32 / BF16 operands of the
// reduced tiers).  The gauge tiles are always FP64.
void round_reduced_tiles(const qdcb_plan &p, Space &sp, int b0, int b1, int64_t slot0,
                         double *panel, const int32_t *overflow, hipStream_t s) {
  if (p.desc.prec != QDCB_PREC_MIXED) return;
  PanelLoArgs la;
  la.overflow = overflow;
  la.b0 = b0;
  la.b1 = b1;
  la.ntiles = sp.ntiles;
  la.slot_base = sp.slot_base.p;
  la.tcount = sp.tcount.p;
  la.toff = sp.toff.p;
  la.rank = sp.trank.p;
  la.tdesc = sp.tdesc.p;
  la.slot0 = slot0;
  la.panel = panel;
  launch_panel_lo(la, s);
  HIPC(hipGetLastError());
}

// Integral tiles + first half of one space over its current column chunk.
// gauge >= 0: the gauge term of the L-S space (its six-tile panel, same task
// lists and batches), adding to V when gauge = 1; breit: the Gaunt and gauge
// terms together from the fused Breit tiles (gauge = 0).
void first_half(qdcb_plan &p, Space &sp, bool make_tiles, bool count, bool captured,
                StageTimer &tm, hipStream_t s, int gauge = -1, bool breit = false) {
  const bool g3 = gauge >= 0;
  const int64_t slot_elems = (g3 ? 6 : 1) * (int64_t)(TILE * TILE);
  if (sp.sym) {
    // every directed tile is resident: the unique tiles are computed once
    // (first chunk) and written to both of their directed slots; then all bra
    // tiles are contracted in one launch
    if (make_tiles) {
      EriTileArgs ea = eri_args(p, sp, 0, count, g3, breit);
      ea.tasks = sp.utask_k.p;
      ea.task_bra = sp.utask_b.p;
      ea.uslot_bk = sp.uslot_bk.p;
      ea.uslot_kb = sp.uslot_kb.p;
      const bool queue = p.tune.eri_sched == 1;
      // the queue counter is zeroed with the order; a second persistent launch
      // over the same order (the gauge tiles) zeroes it again first
      unsigned long long *qctr = sp.lpt.p + 2 * LPT_CLASSES;
      if (queue && g3) launch_zero_u64(qctr, 1, s);
      auto tiles = [&](int64_t n_host, int nblocks, int64_t nlist) {
        if (queue && g3)
          launch_eri_gauge_tiles_queue(ea, sp.uorder.p, qctr, n_host, nblocks, s);
        else if (queue)
          launch_eri_tiles_queue(ea, sp.uorder.p, qctr, n_host, nblocks, s);
        else if (g3)
          launch_eri_gauge_tiles(ea, nlist, s);
        else
          launch_eri_tiles(ea, nlist, s);
      };
      if (captured) {
        ea.overflow = sp.overflow.p;
        ea.d_total = sp.udtotal.p;
        ea.cap = sp.panel_slots;
        tiles(0, eri_queue_blocks(p), std::min<int64_t>(sp.panel_slots, (int64_t)sp.utask_k.n));
        if (!g3) round_reduced_tiles(p, sp, 0, sp.ntiles, 0, sp.pan(), sp.overflow.p, s);
      } else {
        tm.begin(ST_ERI);
        tiles(sp.utotal, (int)std::min<int64_t>(eri_queue_blocks(p), sp.utotal), sp.utotal);
        if (!g3) round_reduced_tiles(p, sp, 0, sp.ntiles, 0, sp.pan(), nullptr, s);
        tm.end();
        if (!g3) p.tiles_made += sp.utotal;
      }
      HIPC(hipGetLastError());
    }
    FirstHalfArgs fa = fh_args(p, sp, 0, sp.ntiles, 0, g3);
    if (captured) fa.overflow = sp.overflow.p;
    contract(p, sp, fa, tm, s, gauge);
    return;
  }
  if (captured) {
    if (make_tiles) {
      EriTileArgs ea = eri_args(p, sp, 0, count, g3, breit);
      ea.d_total = sp.dtotal.p;
      ea.cap = sp.panel_slots;
      const int64_t n = std::min<int64_t>(sp.panel_slots, (int64_t)sp.ntiles * sp.ntiles);
      if (g3) {
        launch_eri_gauge_tiles(ea, n, s);
      } else {
        launch_eri_tiles(ea, n, s);
        round_reduced_tiles(p, sp, 0, sp.ntiles, 0, sp.pan(), sp.overflow.p, s);
      }
    }
    FirstHalfArgs fa = fh_args(p, sp, 0, sp.ntiles, 0, g3);
    fa.overflow = sp.overflow.p;
    contract(p, sp, fa, tm, s, gauge);
    return;
  }
  // Batches of consecutive bra tiles.  When the tiles are generated here, the
  // integral tiles of a batch are made on the side stream while the main
  // stream contracts the previous batch.  With every kept tile resident the
  // batches use disjoint panel slots (about four batches); otherwise the panel
  // is used as two halves and the tiles of batch i wait until the
  // contraction of batch i-2 has released its half.
  const int64_t cap = sp.panel_slots;
  const bool resident_all = sp.total <= cap;
  int maxcnt = 0;
  for (int b = 0; b < sp.ntiles; ++b) maxcnt = std::max(maxcnt, sp.cnt[b]);
  const bool pipe = make_tiles && (resident_all || maxcnt <= cap / 2);
  const int64_t limit = !pipe ? cap : resident_all ? std::max<int64_t>((sp.total + 3) / 4, 1)
                                                   : cap / 2;
  struct Batch {
    int b0, b1;
    int64_t used, off;
  };
  std::vector<Batch> batches;
  for (int b0 = 0; b0 < sp.ntiles;) {
    int b1 = b0;
    int64_t used = 0;
    while (b1 < sp.ntiles && (b1 == b0 || used + sp.cnt[b1] <= limit)) used += sp.cnt[b1++];
    int64_t off = 0;
    if (pipe && !resident_all) off = (batches.size() % 2) * (cap / 2);
    else if (pipe) off = sp.base[b0];
    batches.push_back({b0, b1, used, off});
    b0 = b1;
  }
  hipEvent_t ready = pipe ? tm.record(s) : nullptr;
  std::vector<hipEvent_t> made(batches.size()), done(batches.size());
  for (size_t i = 0; i < batches.size(); ++i) {
    const Batch &B = batches[i];
    double *panel = (g3 ? sp.panel3.p : sp.pan()) + B.off * slot_elems;
    if (make_tiles) {
      hipStream_t es = pipe ? p.side : s;
      if (pipe) {
        HIPC(hipStreamWaitEvent(es, ready, 0));
        if (!resident_all && i >= 2) HIPC(hipStreamWaitEvent(es, done[i - 2], 0));
      }
      EriTileArgs ea = eri_args(p, sp, sp.base[B.b0], count, g3, breit);
      ea.panel = panel;
      tm.begin(ST_ERI, es);
      if (g3) {
        launch_eri_gauge_tiles(ea, B.used, es);
      } else {
        launch_eri_tiles(ea, B.used, es);
        round_reduced_tiles(p, sp, B.b0, B.b1, sp.base[B.b0], panel, nullptr, es);
      }
      if (!g3) p.tiles_made += B.used;
      tm.end(es);
      HIPC(hipGetLastError());
      if (pipe) {
        made[i] = tm.record(es);
        HIPC(hipStreamWaitEvent(s, made[i], 0));
      }
    }
    FirstHalfArgs fa = fh_args(p, sp, B.b0, B.b1, sp.base[B.b0], g3);
    fa.panel = panel;
    contract(p, sp, fa, tm, s, gauge);
    if (pipe && !resident_all) done[i] = tm.record(s);
  }
}

// First quarter of the second half, read straight from V: W[c][b][zq] =
// sum_k V[rowmap[b * sb + k * sk]][col0 + c] Call[k][zq] for batches b < nb.
void gather_quarter(const qdcb_plan &p, const Space &sp, const int32_t *rowmap, int64_t sb,
                    int64_t sk, int nb, int K, const double *Call, int64_t col0, int nc,
                    hipStream_t s) {
  GatherGemmArgs g{};
  g.V = sp.V.p;
  g.ld = sp.ld;
  g.col0 = col0;
  g.rowmap = rowmap;
  g.sb = sb;
  g.sk = sk;
  g.nc = nc;
  g.K = K;
  g.J = 4 * p.n;
  g.nb = nb;
  g.B = Call;
  g.ldb = 4 * p.n;
  g.C = p.W.p;
  g.ldc_c = (int64_t)nb * 4 * p.n;
  g.ldc_b = 4 * p.n;
  g.share_b = 0;  // the J tiles of a batch read the same V rows
  launch_gather_gemm(g, s);
}

// Second quarter for nc columns: Gc[c] (+)= Ahat^T W[c], Ahat [4N][4n] (rows
// (mu, z), columns (x, p)), W[c] [4N][n], Gc[c] [4n][n].  Tile 128: the
// gathered-GEMM kernel with identity rows (A^T rows are Ahat's rows, one
// W block per batch; quaternion plans compute only p <= q when 16 divides n);
// tile 64: the batched GEMM.
void second_quarter(const qdcb_plan &p, const double *Ahat, int N, bool accumulate, int nc,
                    hipStream_t s, bool upper = true) {
  const int n = p.n;
  const int M = (p.spinor ? 2 : 4) * n;  // output planes: re, im (spinors) or x = 0..3
  // quaternion plans: only p <= q (the pack fills p > q by the bra-pair rule)
  const int tri_n = upper && !p.spinor && n % 16 == 0 ? n : 0;
  if (p.tune.sq_tile == 128) {
    GatherGemmArgs g{};
    g.V = Ahat;
    g.ld = 4 * n;
    g.col0 = 0;
    g.rowmap = nullptr;
    g.nc = M;
    g.K = 4 * N;
    g.J = n;
    g.nb = nc;
    g.B = p.W.p;
    g.ldb = n;
    g.sbB = (int64_t)N * 4 * n;
    g.C = p.Gc.p;
    g.ldc_c = n;
    g.ldc_b = (int64_t)4 * n * n;
    g.accumulate = accumulate ? 1 : 0;
    g.share_b = 1;  // the (x, p) tiles of a column read the same W_c
    g.tri_n = tri_n;
    launch_gather_gemm(g, s);
  } else {
    launch_dgemm_batched(1, M, n, 4 * N, 1.0, Ahat, 4 * n, 0, p.W.p, n, (int64_t)N * 4 * n,
                         accumulate ? 1.0 : 0.0, p.Gc.p, n, (int64_t)4 * n * n, nc, s, tri_n);
  }
}

// Receiver of the blocked output: after each second-half slice the stream is
// synchronized and the slice's MO pairs are handed to the callback.
struct BlockSink {
  qdcb_block_cb cb = nullptr;
  void *user = nullptr;
  bool on_device = true;
  int64_t pairs = 1;  // MO pairs per block (the block buffer's capacity)
  void deliver(qdcb_plan &p, int64_t i0, int64_t i1, hipStream_t s) {
    const size_t nb = (size_t)(i1 - i0) * p.n * p.n * 32;
    const double *B = p.Gb.p;
    if (!on_device) {
      if (p.h_Gb.size() < nb) p.h_Gb.resize(nb);
      HIPC(hipMemcpyAsync(p.h_Gb.data(), p.Gb.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
      B = p.h_Gb.data();
    }
    HIPC(hipStreamSynchronize(s));
    if (cb(user, i0, i1, B, on_device ? 1 : 0) != 0)
      fail(QDCB_E_ABORTED, "the block callback asked to stop");
  }
};

enum { CLS_COULOMB = 1, CLS_GAUNT = 2, CLS_GAUGE = 4, CLS_LS = CLS_GAUNT | CLS_GAUGE };

// Every integral class of the plan's Hamiltonian.
int all_classes(const qdcb_plan &p) {
  return CLS_COULOMB | (p.gaunt ? CLS_GAUNT : 0) | (p.gauge ? CLS_GAUGE : 0);
}

// classes: the V of the L-S space holds the Gaunt and / or gauge terms, whose
// second halves are the same.
void second_half(qdcb_plan &p, int i0, int i1, double *dG, hipStream_t s, int classes,
                 BlockSink *sink = nullptr) {
  const int n = p.n;
  const int64_t cend = 4LL * i1;
  const bool do_c = classes & CLS_COULOMB, do_g = p.gaunt && (classes & CLS_LS);
  // slices of whole MO pairs; with blocked output, of at most one block
  const int64_t step = sink ? std::min<int64_t>(p.sc, 4 * sink->pairs) : p.sc;
  for (int64_t c0 = 4LL * i0; c0 < cend; c0 += step) {
    const int nc = (int)std::min<int64_t>(step, cend - c0);
    const int64_t lc0 = c0 - 4LL * i0;
    auto pack = [&](double mirror, int accumulate) {
      if (p.spinor)  // (pq|dc) = A - iB for both classes; blocks are not offered
        launch_pack_spinor(n, p.rs.p, p.npair_s, c0, nc, p.Gc.p, dG, accumulate, s);
      else if (sink)
        launch_pack_block(n, p.rs.p, c0, nc, p.Gc.p, p.Gb.p, c0 / 4, mirror, accumulate, s);
      else
        launch_pack(n, p.rs.p, c0, nc, p.Gc.p, dG, mirror, accumulate, s);
    };
    for (int cls = 0; do_c && cls < (p.NS ? 2 : 1); ++cls) {
      const int N = cls ? p.NS : p.NL;
      // W_c = V_c C (V_c the symmetric N x N first-half matrix of column c)
      gather_quarter(p, p.C, cls ? p.rowmapS.p : p.rowmapL.p, N, 1, N, N,
                     cls ? p.CallS.p : p.CallL.p, lc0, nc, s);
      // G_c (+)= Chat^T W_c
      second_quarter(p, cls ? p.ChatS.p : p.ChatL.p, N, cls != 0, nc, s);
    }
    if (do_c) pack(1.0, 0);
    if (do_g) {
      const int NL = p.NL, NS = p.NS;
      for (int K = 0; K < 3; ++K) {
        const int64_t col0 = K * p.G.ldK + lc0;
        if (p.spinor) {
          // -c^L(mu)^dagger (V sigma_K c^S): batches mu in L, sum over nu in S
          // (AhatK / BhatK hold the planes of -sigma_K c^L / -sigma_K c^S)
          gather_quarter(p, p.G, p.rowmapLS.p, NS, 1, NL, NS, p.BhatK[K].p, col0, nc, s);
          second_quarter(p, p.ChatL.p, NL, K != 0, nc, s);
          // -c^S(nu)^dagger (V^T sigma_K c^L): batches nu in S, sum over mu in L
          gather_quarter(p, p.G, p.rowmapLS.p, 1, NS, NS, NL, p.AhatK[K].p, col0, nc, s);
          second_quarter(p, p.ChatS.p, NS, true, nc, s);
          continue;
        }
        // T = conj(C^L) e_K (V C^S): batches mu in L, sum over nu in S, every
        // (p, q); the term conj(C^S) e_K C^L follows from T in the pack
        gather_quarter(p, p.G, p.rowmapLS.p, NS, 1, NL, NS, p.CallS.p, col0, nc, s);
        second_quarter(p, p.AhatK[K].p, NL, K != 0, nc, s, false);
      }
      pack(-1.0, do_c ? 1 : 0);
    }
    HIPC(hipGetLastError());
    if (sink) sink->deliver(p, c0 / 4, (c0 + nc) / 4, s);
  }
}

// Enqueue one whole transformation of device inputs into device G.
void enqueue(qdcb_plan &p, const double *dCL, const double *dCS, double *dG, bool captured,
             StageTimer &tm, hipStream_t s, int classes = -1, BlockSink *sink = nullptr) {
  if (classes < 0) classes = all_classes(p);
  std::vector<Space *> spaces;
  if (classes & CLS_COULOMB) spaces.push_back(&p.C);
  else launch_zero_u64(p.C.kept.p, 4, s);
  if (p.gaunt && (classes & CLS_LS)) spaces.push_back(&p.G);
  else if (p.gaunt) launch_zero_u64(p.G.kept.p, 4, s);
  const bool gaunt_term = classes & CLS_GAUNT, gauge_term = p.gauge && (classes & CLS_GAUGE);
  const bool fused = p.fused_breit && gaunt_term && gauge_term;
  p.classes = classes;
  p.tiles_made = 0;
  for (Space *sp : spaces) {
    tm.begin(ST_DENS);
    density(p, *sp, dCL, dCS, 1, 0, p.npair_mo, s);
    tm.end();
    tm.begin(ST_SCREEN);
    order_rows(p, *sp, s);
    screen(p, *sp, captured, s);
    tm.end();
  }
  if (!captured && !tm.probe_only) {
    (void)ensure_residency(p, 1.0);
    // the panels may have been resized: the unique path applies when every
    // directed tile is resident (its lists exist whenever that can hold)
    for (Space *sp : spaces)
      sp->sym = !(p.desc.flags & QDCB_PLAN_DIRECTED_TILES) && sp->total <= sp->panel_slots;
  }
  if (tm.probe_only) return;
  if (p.spinor) {
    launch_build_spinor_mats(p.NL, p.n, dCL, -1, p.CallL.p, p.ChatL.p, s);
    if (p.NS) launch_build_spinor_mats(p.NS, p.n, dCS, -1, p.CallS.p, p.ChatS.p, s);
    if (p.gaunt)
      for (int K = 0; K < 3; ++K) {
        launch_build_spinor_mats(p.NL, p.n, dCL, K, p.AhatK[K].p, nullptr, s);
        launch_build_spinor_mats(p.NS, p.n, dCS, K, p.BhatK[K].p, nullptr, s);
      }
  } else {
    launch_build_coef_mats(p.NL, p.n, dCL, -1, p.CallL.p, p.ChatL.p, s);
    if (p.NS) launch_build_coef_mats(p.NS, p.n, dCS, -1, p.CallS.p, p.ChatS.p, s);
    if (p.gaunt)
      for (int K = 0; K < 3; ++K) {
        launch_build_coef_mats(p.NL, p.n, dCL, K, p.CallL.p, p.AhatK[K].p, s);
        launch_build_coef_mats(p.NS, p.n, dCS, K, p.CallS.p, p.BhatK[K].p, s);
      }
  }
  HIPC(hipGetLastError());
  // MO-driven variant: batches of mo_batch MO pairs, each screened with the
  // density bound of its own pairs and with its own integral tiles (the
  // panels, sized for the all-pairs bound above, hold every batch's subset)
  const bool mo = p.mo_batch > 0 && !captured;
  const int step = mo ? std::min(p.ci, p.mo_batch) : p.ci;
  p.ld_sum[0] = p.ld_sum[1] = 0.0;
  p.mo_work = 0.0;
  p.chunks_run = 0;
  for (int i0 = 0, k = 0; i0 < p.npair_mo && (tm.max_chunks <= 0 || k < tm.max_chunks);
       i0 += step, ++k) {
    const int i1 = std::min(p.npair_mo, i0 + step);
    p.v_i0 = i0;
    p.v_i1 = i1;
    ++p.chunks_run;
    // D~ and V rows packed to this chunk's width: a narrower chunk (the last
    // one, or an MO-driven batch) contracts only its own column tiles
    for (Space *sp : spaces) {
      sp->ldK = round_up(4LL * (i1 - i0), 128);
      sp->ld = sp->nK * sp->ldK;
      if (sp->ld > sp->ld_cap) fail(QDCB_E_DEVICE, "column chunk wider than its buffers");
    }
    if (mo)
      for (Space *sp : spaces) {
        tm.begin(ST_DENS);
        density(p, *sp, dCL, dCS, 1, i0, i1, s);
        tm.end();
        tm.begin(ST_SCREEN);
        order_rows(p, *sp, s);
        screen(p, *sp, false, s, false);  // kept counts add up over the batches
        tm.end();
        sp->sym = !(p.desc.flags & QDCB_PLAN_DIRECTED_TILES) && sp->total <= sp->panel_slots;
      }
    for (Space *sp : spaces) {
      p.ld_sum[sp == &p.G ? 1 : 0] += (double)sp->ld;
      if (mo) p.mo_work += (double)sp->ld * 0.25 * (double)sp->h_steps;
      tm.begin(ST_DENS);
      density(p, *sp, dCL, dCS, 0, i0, i1, s);
      // the reduced tiers' scaled FP32 copy of the density rows
      if (p.desc.prec == QDCB_PREC_MIXED)
        launch_density_lo(sp->Ppad, sp->ld, sp->D.p, sp->Dtmax.p, sp->Dlo.p, s);
      tm.end();
      // captured mode keeps the tiles of the first chunk (one batch, resident)
      const bool resident = captured || sp->sym || sp->total <= sp->panel_slots;
      const bool make = mo || !resident || i0 == 0, count = mo || i0 == 0;
      if (sp == &p.G && fused) {
        // Gaunt + gauge: one pass over the Breit tiles B_KL + delta_KL (mn|kl)
        first_half(p, *sp, make, count, captured, tm, s, 0, true);
        continue;
      }
      if (sp != &p.G || gaunt_term) first_half(p, *sp, make, count, captured, tm, s);
      // gauge term: its own tiles and contraction over the same lists, added
      // to the Gaunt term's V (counted here only without the Gaunt term)
      if (sp == &p.G && gauge_term)
        first_half(p, *sp, make, count && !gaunt_term, captured, tm, s, gaunt_term ? 1 : 0);
    }
    tm.begin(ST_SH);
    second_half(p, i0, i1, dG, s, classes, sink);
    tm.end();
  }
}

void fill_stats(qdcb_plan &p, qdcb_stats *stats, StageTimer *tm, double ms_total,
                const unsigned long long kc[4], const unsigned long long kg[4], int64_t tiles_c,
                int64_t tiles_g) {
  std::memset(stats, 0, sizeof(*stats));
  const int n = p.n;
  if (tm) {
    stats->ms_density = tm->total(ST_DENS);
    stats->ms_screen = tm->total(ST_SCREEN);
    stats->ms_eri = tm->total(ST_ERI);
    stats->ms_first_half = tm->total(ST_FH) + tm->total(ST_FH32) + tm->total(ST_FH16);
    stats->ms_second_half = tm->total(ST_SH);
    stats->n_batches = tm->launches(ST_FH);
    stats->ms_tier[0] = tm->total(ST_FH);
    stats->ms_tier[1] = tm->total(ST_FH32);
    stats->ms_tier[2] = tm->total(ST_FH16);
  }
  stats->ms_total = ms_total;
  double ktot = 0;
  for (int c = 0; c < 4; ++c) {
    stats->kept[c] = (int64_t)kc[c];
    ktot += (double)kc[c];
  }
  if (p.classes & CLS_COULOMB) {
    stats->total[0] = p.nLL * p.nLL;
    stats->total[1] = p.nLL * p.nSS;
    stats->total[2] = p.nSS * p.nLL;
    stats->total[3] = p.nSS * p.nSS;
  }
  const bool ls = p.gaunt && (p.classes & CLS_LS);
  // first-half products per kept L-S contribution and MO-pair column: 3 (Gaunt,
  // one per K) and 9 (gauge, K x L)
  const bool gt = p.classes & CLS_GAUNT, gg = p.gauge && (p.classes & CLS_GAUGE);
  const double ls_mult = p.fused_breit && gt && gg ? 9.0 : (gt ? 3.0 : 0.0) + (gg ? 9.0 : 0.0);
  stats->kept_gaunt = (int64_t)kg[0];
  stats->total_gaunt = ls ? p.G.P * p.G.P : 0;
  stats->tiles_kept = tiles_c + tiles_g;
  stats->tiles_total = ((p.classes & CLS_COULOMB) ? (int64_t)p.C.ntiles * p.C.ntiles : 0) +
                       (ls ? (int64_t)p.G.ntiles * p.G.ntiles : 0);
  stats->flops_first_half =
      2.0 * (double)p.ncol * ktot + 2.0 * ls_mult * (double)p.ncol * (double)kg[0];
  double f2 = 0;
  // per column: first quarter 2 N N 4n, second quarter 2 (4n or 2n output
  // rows) (4N) n; quaternion plans take the Coulomb second quarter over p <= q
  // and one of the two Gaunt chains (the other follows from it)
  for (int cls = 0; (p.classes & CLS_COULOMB) && cls < (p.NS ? 2 : 1); ++cls) {
    double N = cls ? p.NS : p.NL;
    const double sq = p.spinor ? 16.0 * N * n * n : 16.0 * N * n * (n + 1.0);
    f2 += (8.0 * N * N * n + sq) * (double)p.ncol;
  }
  if (ls)
    f2 += 3.0 *
          (p.spinor ? 16.0 * p.NL * (double)p.NS * n + 16.0 * (p.NL + p.NS) * (double)n * n
                    : 8.0 * p.NL * (double)p.NS * n + 32.0 * p.NL * (double)n * n) *
          (double)p.ncol;
  stats->flops_second_half = f2;
  stats->n_chunks = p.chunks_run;
  // MFMA flops issued by the first half: every kept directed tile times the
  // row width of each chunk (per batch for the MO-driven variant); the L-S
  // row width (3 K blocks) counts once for Gaunt and three times for the gauge
  // term (three L blocks per K block)
  const double gw = ls_mult / 3.0;
  // (tiles as run: with the intra-tile order, the steps each task runs / 4)
  const double run_c = p.tile_order && tm ? 0.25 * (double)p.C.h_steps : (double)tiles_c;
  const double run_g = p.tile_order && tm ? 0.25 * (double)p.G.h_steps : (double)tiles_g;
  stats->flops_mfma = 2.0 * TILE * TILE *
                      (p.mo_batch > 0 && tm ? p.mo_work
                                            : p.ld_sum[0] * run_c + gw * p.ld_sum[1] * run_g);
  stats->classes = p.classes;
  if (p.desc.prec == QDCB_PREC_MIXED) {
    for (Space *sp : {&p.C, &p.G}) {
      if (sp == &p.G && !(p.gaunt && (p.classes & CLS_GAUNT))) continue;  // tiers: Gaunt only
      if (sp == &p.C && !(p.classes & CLS_COULOMB)) continue;
      if (sp->h_tcount.size() != 3 * (size_t)sp->ntiles) continue;
      for (int t = 0; t < 3; ++t)
        for (int b = 0; b < sp->ntiles; ++b)
          stats->tiles_tier[t] += sp->h_tcount[(size_t)t * sp->ntiles + b];
    }
  }
}

void read_counters(qdcb_plan &p, hipStream_t s, unsigned long long kc[4],
                   unsigned long long kg[4]) {
  for (int c = 0; c < 4; ++c) kc[c] = kg[c] = 0;
  HIPC(hipMemcpyAsync(kc, p.C.kept.p, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (p.gaunt)
    HIPC(hipMemcpyAsync(kg, p.G.kept.p, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                        s));
}

void run_eager(qdcb_plan &p, const double *dCL, const double *dCS, double *dG, hipStream_t s,
               qdcb_stats *stats, int classes = -1, BlockSink *sink = nullptr) {
  if (classes < 0) classes = all_classes(p);
  StageTimer tm(s, true);
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  HIPC(hipEventRecord(e0, s));
  enqueue(p, dCL, dCS, dG, false, tm, s, classes, sink);
  HIPC(hipEventRecord(e1, s));
  unsigned long long kc[4], kg[4];
  read_counters(p, s, kc, kg);
  HIPC(hipStreamSynchronize(s));
  float ms = 0;
  HIPC(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p.have_last = true;
  if (stats) {
    fill_stats(p, stats, &tm, ms, kc, kg, (classes & CLS_COULOMB) ? p.C.total : 0,
               p.gaunt && (classes & CLS_LS) ? p.G.total : 0);
    stats->tiles_made = p.tiles_made;
  }
}

// Integral classes selected by transform flags.
int class_mask(const qdcb_plan &p, uint32_t flags) {
  if (flags &
      ~(uint32_t)(QDCB_PTR_DEVICE | QDCB_CLASS_COULOMB | QDCB_CLASS_GAUNT | QDCB_CLASS_GAUGE))
    fail(QDCB_E_INVALID, "unknown transform flag");
  int m = 0;
  if (flags & QDCB_CLASS_COULOMB) m |= CLS_COULOMB;
  if (flags & QDCB_CLASS_GAUNT) m |= CLS_GAUNT;
  if (flags & QDCB_CLASS_GAUGE) m |= CLS_GAUGE;
  const int all = all_classes(p);
  if (!m) return all;
  // classes the plan lacks are ignored beside one it has
  if (!(m & all))
    fail(QDCB_E_INVALID, (m & CLS_GAUGE) ? "QDCB_CLASS_GAUGE needs a DCB plan"
                                         : "QDCB_CLASS_GAUNT needs a DCG or DCB plan");
  return m & all;
}

// Device copies of host inputs (QDCB_PTR_DEVICE unset): CL, CS into the
// plan's coefficient buffers, G into its staging buffer.
struct DevIO {
  const double *CL, *CS;
  double *G;
};
DevIO device_io(qdcb_plan &p, const double *CL, const double *CS, double *G, bool dev,
                hipStream_t s) {
  if (dev) return {CL, CS, G};
  const size_t nG = (size_t)p.n * p.n * p.n * p.n * (p.spinor ? 2 : 16);
  check_finite_host(CL, (size_t)4 * p.NL * p.n, "CL");
  if (p.NS) check_finite_host(CS, (size_t)4 * p.NS * p.n, "CS");
  HIPC(hipMemcpyAsync(p.CLd.p, CL, p.CLd.bytes(), hipMemcpyHostToDevice, s));
  DevIO io{p.CLd.p, nullptr, nullptr};
  if (p.NS) {
    HIPC(hipMemcpyAsync(p.CSd.p, CS, p.CSd.bytes(), hipMemcpyHostToDevice, s));
    io.CS = p.CSd.p;
  }
  if (p.Gd.n != nG) p.Gd.alloc(p.ctx, nG);
  io.G = p.Gd.p;
  return io;
}

}  // namespace

extern "C" {

qdcb_status qdcb_plan_autotune(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                               uint32_t flags, void *hip_stream, const char *cache_path,
                               qdcb_tune_report *report) {
  return guarded([&] {
    if (!plan || !CL || !G) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    PlanUse use(p);
    if (p.NS && !CS) fail(QDCB_E_INVALID, "CS is required for this Hamiltonian");
    const char *path = cache_path ? cache_path : std::getenv("QDCB_TUNE_CACHE");
    if (path && !*path) path = nullptr;
    qdcb_tune_report rep{};
    for (int v = 0; v < 2; ++v)
      rep.ms_eri[v] = rep.ms_first_half[v] = rep.ms_second_half[v] = std::nan("");
    if (path) {
      qdcb_tune t{};
      int32_t found = 0;
      const qdcb_status st = qdcb_tune_cache_lookup(path, p.tune_key.c_str(), &t, &found);
      if (st != QDCB_OK) fail(st, qdcb_last_error());
      if (found && !tune_problem(p, t)) {
        p.tune = t;
        rep.chosen = p.tune;
        rep.from_cache = 1;
        if (report) *report = rep;
        return;
      }
    }
    DeviceGuard g(p.ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    StreamMark mark{p, s};  // after this call's work on s
    const DevIO io = device_io(p, CL, CS, G, flags & QDCB_PTR_DEVICE, s);
    const qdcb_tune saved = p.tune;
    // the two candidates differ in every choice; alternating them gives each
    // value of each choice two timings of its own stage
    const qdcb_tune cand[2] = {{0, 0, 64, 0}, {1, 1, p.n % 2 ? 64 : 128, 0}};
    const double inf = std::numeric_limits<double>::infinity();
    double best[3][2] = {{inf, inf}, {inf, inf}, {inf, inf}};
    auto trial = [&](const qdcb_tune &t, bool keep) {
      p.tune = t;
      StageTimer tm(s, true);
      tm.max_chunks = 1;
      enqueue(p, io.CL, io.CS, io.G, false, tm, s);
      HIPC(hipStreamSynchronize(s));
      if (!keep) return;
      const double ms[3] = {tm.total(ST_ERI),
                            tm.total(ST_FH) + tm.total(ST_FH32) + tm.total(ST_FH16),
                            tm.total(ST_SH)};
      const int val[3] = {t.eri_sched, t.fh_order, t.sq_tile == 128 ? 1 : 0};
      for (int c = 0; c < 3; ++c) best[c][val[c]] = std::min(best[c][val[c]], ms[c]);
    };
    try {
      trial(saved, false);  // warm-up: panel sizing, first launches of every kernel
      for (int r = 0; r < 4; ++r) trial(cand[r & 1], true);
    } catch (...) {
      p.tune = saved;
      throw;
    }
    auto pick = [&](int c) { return best[c][1] < 0.99 * best[c][0] ? 1 : 0; };
    qdcb_tune t{};
    t.eri_sched = pick(0);
    t.fh_order = pick(1);
    t.sq_tile = pick(2) ? 128 : 64;
    p.tune = t;
    rep.chosen = t;
    rep.trials = 4;
    for (int v = 0; v < 2; ++v) {
      if (best[0][v] < inf) rep.ms_eri[v] = best[0][v];
      if (best[1][v] < inf) rep.ms_first_half[v] = best[1][v];
      if (best[2][v] < inf) rep.ms_second_half[v] = best[2][v];
    }
    if (path) {
      const qdcb_status st = qdcb_tune_cache_store(path, p.tune_key.c_str(), &t);
      if (st != QDCB_OK) fail(st, qdcb_last_error());
    }
    if (report) *report = rep;
  });
}

qdcb_status qdcb_transform(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                           uint32_t flags, void *hip_stream, qdcb_stats *stats) {
  return guarded([&] {
    if (!plan || !CL || !G) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    PlanUse use(p);
    if (p.NS && !CS) fail(QDCB_E_INVALID, "CS is required for this Hamiltonian");
    DeviceGuard g(p.ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    StreamMark mark{p, s};  // after this call's work on s
    const bool dev = flags & QDCB_PTR_DEVICE;
    const int classes = class_mask(p, flags);
    const int n = p.n;
    const size_t nG = (size_t)n * n * n * n * (p.spinor ? 2 : 16);
    const DevIO io = device_io(p, CL, CS, G, dev, s);
    double *dG = io.G;
    run_eager(p, io.CL, io.CS, dG, s, stats, classes);
    if (!dev) {
      HIPC(hipMemcpyAsync(G, dG, nG * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
    }
  });
}

qdcb_status qdcb_transform_blocks(qdcb_plan *plan, const double *CL, const double *CS,
                                  qdcb_block_cb cb, void *user, uint32_t flags,
                                  void *hip_stream, qdcb_stats *stats) {
  return guarded([&] {
    if (!plan || !CL || !cb) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    PlanUse use(p);
    if (p.NS && !CS) fail(QDCB_E_INVALID, "CS is required for this Hamiltonian");
    if (p.spinor) fail(QDCB_E_UNSUPPORTED, "blocked output is offered for quaternion plans");
    DeviceGuard g(p.ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    StreamMark mark{p, s};  // after this call's work on s
    const bool dev = flags & QDCB_PTR_DEVICE;
    const int classes = class_mask(p, flags);
    // block buffer: at most one second-half slice of MO pairs, both (r, s)
    // and (s, r), within what the context budget leaves
    const size_t pair_doubles = (size_t)p.n * p.n * 32;
    int64_t pairs = p.sc / 4;
    if (p.Gb.n < (size_t)pairs * pair_doubles) {
      const size_t room = p.ctx->room() + p.Gb.bytes();
      pairs = std::min<int64_t>(pairs, (int64_t)(room / (pair_doubles * sizeof(double))));
      if (pairs < 1) fail(QDCB_E_NOMEM, "no room for the block buffer of one MO pair");
      if (p.Gb.n < (size_t)pairs * pair_doubles) {
        p.Gb.free();
        p.Gb.alloc(p.ctx, (size_t)pairs * pair_doubles);
      }
    }
    BlockSink sink;
    sink.cb = cb;
    sink.user = user;
    sink.on_device = dev;
    sink.pairs = (int64_t)(p.Gb.n / pair_doubles);
    // the host-pointer path needs device copies of CL and CS only (no G)
    const double *dCL = CL, *dCS = CS;
    if (!dev) {
      check_finite_host(CL, (size_t)4 * p.NL * p.n, "CL");
      if (p.NS) check_finite_host(CS, (size_t)4 * p.NS * p.n, "CS");
      HIPC(hipMemcpyAsync(p.CLd.p, CL, p.CLd.bytes(), hipMemcpyHostToDevice, s));
      dCL = p.CLd.p;
      if (p.NS) {
        HIPC(hipMemcpyAsync(p.CSd.p, CS, p.CSd.bytes(), hipMemcpyHostToDevice, s));
        dCS = p.CSd.p;
      }
    }
    run_eager(p, dCL, dCS, nullptr, s, stats, classes, &sink);
  });
}

qdcb_status qdcb_plan_capture(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                              void *hip_stream) {
  return guarded([&] {
    if (!plan || !CL || !G || !hip_stream) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    PlanUse use(p);
    if (p.mo_batch > 0) fail(QDCB_E_UNSUPPORTED, "the MO-driven variant is not captured");
    if (p.NS && !CS) fail(QDCB_E_INVALID, "CS is required for this Hamiltonian");
    DeviceGuard g(p.ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    if (p.graph_exec) {
      (void)hipGraphExecDestroy(p.graph_exec);
      p.graph_exec = nullptr;
    }
    if (p.graph) {
      (void)hipGraphDestroy(p.graph);
      p.graph = nullptr;
    }
    // size the panels for the capture-time kept tiles (with 25% slack for
    // re-transforms whose screening keeps more), so that replays stay resident
    {
      StageTimer probe(s, false);
      probe.probe_only = true;
      enqueue(p, CL, CS, G, false, probe, s);
      HIPC(hipStreamSynchronize(s));
      (void)ensure_residency(p, 1.25);
    }
    StageTimer tm(s, false);
    HIPC(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      enqueue(p, CL, CS, G, true, tm, s);
    } catch (...) {
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(s, &dead);
      if (dead) (void)hipGraphDestroy(dead);
      throw;
    }
    HIPC(hipStreamEndCapture(s, &p.graph));
    HIPC(hipGraphInstantiate(&p.graph_exec, p.graph, nullptr, nullptr, 0));
    p.g_CL = CL;
    p.g_CS = CS;
    p.g_G = G;
    p.g_sym = p.C.sym;
  });
}

qdcb_status qdcb_plan_replay(qdcb_plan *plan, void *hip_stream, qdcb_stats *stats) {
  return guarded([&] {
    if (!plan) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    PlanUse use(p);
    if (!p.graph_exec) fail(QDCB_E_INVALID, "no captured transform (call qdcb_plan_capture)");
    DeviceGuard g(p.ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    StreamMark mark{p, s};  // after this call's work on s
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    HIPC(hipEventRecord(e0, s));
    HIPC(hipGraphLaunch(p.graph_exec, s));
    HIPC(hipEventRecord(e1, s));
    int32_t ovf[2] = {0, 0};
    int64_t tot[2] = {0, 0}, made[2] = {0, 0};
    const int nsp = p.gaunt ? 2 : 1;
    for (int i = 0; i < nsp; ++i) {
      const Space &sp = i ? p.G : p.C;
      HIPC(hipMemcpyAsync(&ovf[i], sp.overflow.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(&tot[i], sp.dtotal.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(&made[i], p.g_sym ? sp.udtotal.p : sp.dtotal.p, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    }
    unsigned long long kc[4], kg[4];
    read_counters(p, s, kc, kg);
    HIPC(hipStreamSynchronize(s));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ovf[0] || ovf[1]) {  // the kept tiles outgrew the panel: redo eagerly
      run_eager(p, p.g_CL, p.g_CS, p.g_G, s, stats);
      if (stats) stats->graph_fallback = 1;
      return;
    }
    p.have_last = true;
    if (stats) {
      fill_stats(p, stats, nullptr, ms, kc, kg, tot[0], tot[1]);
      stats->tiles_made = made[0] + made[1];
      stats->graph_replay = 1;
    }
  });
}

}  // extern "C"
