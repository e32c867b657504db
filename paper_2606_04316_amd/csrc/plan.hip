// plan.hip -- C ABI: plans and the transformation driver.
//
// A plan holds one or two pair spaces:
//   Coulomb  LL pairs (mu <= nu) and, for DC/DCG, SS pairs: the classes of
//            Eq. (DCInt); one AO integral tile serves every class pair because
//            the stand-in small-component functions are scalar s Gaussians.
//   Gaunt    ordered LS pairs (mu in L, nu in S) of Eq. (GauntInt), with three
//            Pauli components K per MO-pair column.
// Rows of a space are ordered by decreasing Schwarz factor and padded to a
// multiple of 64.  A transformation runs the paper's four stages (Sec. 3.3.1):
// quaternion densities (and their bound), screening, AO integral tiles with the
// first-half contraction, and the second half -- all on the GPU; the host only
// sizes batches from the per-bra-tile counts of kept tiles.
#include "runtime.h"

using namespace qdcb;

namespace {

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
  // per transform
  std::vector<int32_t> cnt;
  std::vector<int64_t> base;
  int64_t total = 0;

  size_t bytes() const {
    size_t b = cls.bytes() + mu.bytes() + nu.bytes() + row_first.bytes() + Q.bytes() +
               pp.bytes() + D.bytes() + V.bytes() + Dmax.bytes() + Qmax.bytes() + Bmax.bytes() +
               count.bytes() + tasks.bytes() + task_bra.bytes() + slot_base.bytes() +
               panel.bytes() + kept.bytes();
    return b;
  }
};

// Primitive pairs whose Schwarz weight is below 1e-17 of their row's mean are
// dropped (bounded effect: ~1e-17 of the sum of absolute primitive terms).
constexpr double PRIM_EPS = 1e-17;

// Sorted rows of a space: order by decreasing Q (stable in the input order).
struct RowSrc {
  double Q;
  int32_t cls, mu, nu;
  int64_t key;
  int64_t src_first;
  int32_t cnt;
  int which;  // which source store
};

void build_space(qdcb_ctx *ctx, Space &sp, std::vector<RowSrc> &rows,
                 const std::vector<const PairStore *> &stores) {
  std::stable_sort(rows.begin(), rows.end(),
                   [](const RowSrc &a, const RowSrc &b) { return a.Q > b.Q; });
  sp.P = (int64_t)rows.size();
  sp.Ppad = std::max<int64_t>(round_up(sp.P, TILE), TILE);
  if (sp.Ppad / TILE > (1 << 30)) fail(QDCB_E_INVALID, "too many pairs");
  sp.ntiles = (int)(sp.Ppad / TILE);
  sp.h_cls.assign(sp.Ppad, -1);
  sp.h_mu.assign(sp.Ppad, 0);
  sp.h_nu.assign(sp.Ppad, 0);
  sp.h_key.assign(sp.Ppad, -1);
  std::vector<double> hQ(sp.Ppad, 0.0);
  const size_t ns = stores.size();
  std::vector<std::vector<int64_t>> src(ns), dst(ns), rowidx(ns);
  std::vector<std::vector<int32_t>> cnt(ns);
  for (int64_t r = 0; r < sp.P; ++r) {
    const RowSrc &s = rows[r];
    sp.h_cls[r] = s.cls;
    sp.h_mu[r] = s.mu;
    sp.h_nu[r] = s.nu;
    sp.h_key[r] = s.key;
    hQ[r] = s.Q;
    src[s.which].push_back(s.src_first);
    cnt[s.which].push_back(s.cnt);
    rowidx[s.which].push_back(r);
  }
  // primitive pairs kept per row after primitive screening
  std::vector<DBuf<int64_t>> dsrc(ns);
  std::vector<DBuf<int32_t>> dcnt(ns);
  std::vector<int32_t> kept_prims(sp.Ppad, 0);
  for (size_t w = 0; w < ns; ++w) {
    if (src[w].empty()) continue;
    dsrc[w].upload(ctx, src[w]);
    dcnt[w].upload(ctx, cnt[w]);
    DBuf<int32_t> dk;
    dk.alloc(ctx, src[w].size());
    launch_prim_count((int64_t)src[w].size(), dsrc[w].p, dcnt[w].p, stores[w]->cview(),
                      PRIM_EPS, dk.p, nullptr);
    HIPC(hipGetLastError());
    std::vector<int32_t> k(src[w].size());
    HIPC(hipMemcpy(k.data(), dk.p, k.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < k.size(); ++i) kept_prims[rowidx[w][i]] = k[i];
  }
  std::vector<int64_t> rf(sp.Ppad + 1, 0);
  for (int64_t r = 0; r < sp.Ppad; ++r) rf[r + 1] = rf[r] + kept_prims[r];
  for (size_t w = 0; w < ns; ++w)
    for (int64_t r : rowidx[w]) dst[w].push_back(rf[r]);
  sp.cls.upload(ctx, sp.h_cls);
  sp.mu.upload(ctx, sp.h_mu);
  sp.nu.upload(ctx, sp.h_nu);
  sp.Q.upload(ctx, hQ);
  sp.row_first.upload(ctx, rf);
  sp.pp.alloc(ctx, (size_t)std::max<int64_t>(rf[sp.Ppad], 1));
  for (size_t w = 0; w < ns; ++w) {
    if (src[w].empty()) continue;
    DBuf<int64_t> dd;
    dd.upload(ctx, dst[w]);
    launch_gather_pairs((int64_t)src[w].size(), dsrc[w].p, dcnt[w].p, dd.p, stores[w]->cview(),
                        sp.pp.view(), PRIM_EPS, nullptr);
    HIPC(hipGetLastError());
    HIPC(hipDeviceSynchronize());
  }
  sp.Dmax.alloc(ctx, sp.Ppad);
  sp.Qmax.alloc(ctx, sp.ntiles);
  sp.Bmax.alloc(ctx, sp.ntiles);
  sp.count.alloc(ctx, sp.ntiles);
  sp.slot_base.alloc(ctx, sp.ntiles);
  sp.kept.alloc(ctx, 4);
}

}  // namespace

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
  Space C, G;
  DBuf<int32_t> rs, rowmapL, rowmapS, rowmapLS;
  DBuf<double> CLd, CSd, Gd;
  DBuf<double> CallL, CallS, ChatL, ChatS;
  DBuf<double> AhatK[3], BhatK[3];
  DBuf<double> Vfull, W, Gc;
  bool have_last = false;
};

extern "C" {

qdcb_status qdcb_plan_create(qdcb_ctx *ctx, const qdcb_basis *L, const qdcb_basis *S,
                             const qdcb_plan_desc *desc, qdcb_plan **out) {
  return guarded([&] {
    if (!ctx || !L || !desc || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (desc->ham != QDCB_HAM_LL && desc->ham != QDCB_HAM_DC && desc->ham != QDCB_HAM_DCG)
      fail(QDCB_E_INVALID, "unknown Hamiltonian");
    if (desc->prec != QDCB_PREC_FP64)
      fail(QDCB_E_UNSUPPORTED, "only QDCB_PREC_FP64 is available in this build");
    if ((desc->ham == QDCB_HAM_LL) != (S == nullptr))
      fail(QDCB_E_INVALID, "S must be NULL exactly for QDCB_HAM_LL");
    if (desc->n_mo < 1 || desc->n_mo > 512) fail(QDCB_E_INVALID, "n_mo must be in [1, 512]");
    if (!std::isfinite(desc->tau) || desc->tau < 0) fail(QDCB_E_INVALID, "tau must be >= 0");
    if (L->ctx != ctx || (S && S->ctx != ctx)) fail(QDCB_E_INVALID, "basis of another context");
    DeviceGuard g(ctx->device);
    std::unique_ptr<qdcb_plan> pl(new qdcb_plan());
    qdcb_plan &p = *pl;
    p.ctx = ctx;
    p.nLL = L->npairs;
    p.nSS = S ? S->npairs : 0;
    p.desc = *desc;
    p.n = desc->n_mo;
    p.NL = L->nfunc;
    p.NS = S ? S->nfunc : 0;
    p.gaunt = desc->ham == QDCB_HAM_DCG;
    p.npair_mo = p.n * (p.n + 1) / 2;
    p.ncol = 4LL * p.npair_mo;

    // --- Coulomb space: LL pairs, then SS pairs
    {
      std::vector<RowSrc> rows;
      rows.reserve(L->npairs + (S ? S->npairs : 0));
      auto add = [&](const qdcb_basis *B, int cls, int which) {
        for (int nu = 0; nu < B->nfunc; ++nu)
          for (int mu = 0; mu <= nu; ++mu) {
            int64_t c = qdcb_basis::canon(mu, nu);
            rows.push_back(RowSrc{B->Q[c], cls, mu, nu, c, B->pair_first[c],
                                  (int32_t)(B->pair_first[c + 1] - B->pair_first[c]), which});
          }
      };
      add(L, 0, 0);
      std::vector<const PairStore *> stores{&L->pp};
      if (S) {
        add(S, 1, 1);
        stores.push_back(&S->pp);
      }
      p.C.gaunt = 0;
      p.C.nK = 1;
      build_space(ctx, p.C, rows, stores);
    }
    // --- Gaunt space: ordered LS pairs (mu in L, nu in S), key mu*NS + nu
    if (p.gaunt) {
      int64_t nls = (int64_t)p.NL * p.NS;
      std::vector<int32_t> pm(nls), pn(nls);
      std::vector<int64_t> pf(nls + 1, 0);
      for (int mu = 0; mu < p.NL; ++mu)
        for (int nu = 0; nu < p.NS; ++nu) {
          int64_t i = (int64_t)mu * p.NS + nu;
          pm[i] = mu;
          pn[i] = nu;
          pf[i + 1] = pf[i] + (int64_t)L->nprim[mu] * S->nprim[nu];
        }
      PairStore ls;
      DBuf<int32_t> dm, dn;
      DBuf<int64_t> dpf;
      DBuf<double> dQ;
      dm.upload(ctx, pm);
      dn.upload(ctx, pn);
      dpf.upload(ctx, pf);
      ls.alloc(ctx, (size_t)pf[nls]);
      launch_pair_data(nls, dm.p, dn.p, dpf.p, L->cent.p, L->dfirst.p, L->exps.p, L->nc.p,
                       S->cent.p, S->dfirst.p, S->exps.p, S->nc.p, ls.view(), nullptr);
      dQ.alloc(ctx, nls);
      launch_schwarz(nls, dpf.p, ls.cview(), dQ.p, nullptr);
      HIPC(hipGetLastError());
      std::vector<double> hQ(nls);
      HIPC(hipMemcpy(hQ.data(), dQ.p, nls * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<RowSrc> rows(nls);
      for (int64_t i = 0; i < nls; ++i)
        rows[i] = RowSrc{hQ[i], 0, pm[i], pn[i], i, pf[i], (int32_t)(pf[i + 1] - pf[i]), 0};
      p.G.gaunt = 1;
      p.G.nK = 3;
      build_space(ctx, p.G, rows, {&ls});
    }

    // --- index tables
    std::vector<int32_t> rs(p.npair_mo);
    {
      int k = 0;
      for (int r = 0; r < p.n; ++r)
        for (int s = r; s < p.n; ++s) rs[k++] = r | (s << 16);
    }
    p.rs.upload(ctx, rs);
    {
      std::vector<int32_t> mL((size_t)p.NL * p.NL), mS((size_t)p.NS * p.NS);
      for (int64_t r = 0; r < p.C.P; ++r) {
        int a = p.C.h_mu[r], b = p.C.h_nu[r];
        if (p.C.h_cls[r] == 0)
          mL[(size_t)a * p.NL + b] = mL[(size_t)b * p.NL + a] = (int32_t)r;
        else
          mS[(size_t)a * p.NS + b] = mS[(size_t)b * p.NS + a] = (int32_t)r;
      }
      p.rowmapL.upload(ctx, mL);
      if (p.NS) p.rowmapS.upload(ctx, mS);
      if (p.gaunt) {
        std::vector<int32_t> mLS((size_t)p.NL * p.NS);
        for (int64_t r = 0; r < p.G.P; ++r) mLS[p.G.h_key[r]] = (int32_t)r;
        p.rowmapLS.upload(ctx, mLS);
      }
    }
    // --- coefficient buffers
    p.CLd.alloc(ctx, (size_t)4 * p.NL * p.n);
    p.CallL.alloc(ctx, (size_t)p.NL * 4 * p.n);
    p.ChatL.alloc(ctx, (size_t)4 * p.NL * 4 * p.n);
    if (p.NS) {
      p.CSd.alloc(ctx, (size_t)4 * p.NS * p.n);
      p.CallS.alloc(ctx, (size_t)p.NS * 4 * p.n);
      p.ChatS.alloc(ctx, (size_t)4 * p.NS * 4 * p.n);
    }
    if (p.gaunt)
      for (int K = 0; K < 3; ++K) {
        p.AhatK[K].alloc(ctx, (size_t)4 * p.NL * 4 * p.n);
        p.BhatK[K].alloc(ctx, (size_t)4 * p.NS * 4 * p.n);
      }

    // --- task lists: one slot per (bra tile, ket tile), the worst case
    for (Space *sp : {&p.C, &p.G}) {
      if (sp == &p.G && !p.gaunt) continue;
      size_t cap = (size_t)sp->ntiles * (size_t)sp->ntiles;
      sp->tasks.alloc(ctx, cap);
      sp->task_bra.alloc(ctx, cap);
    }
    // room left for the sized buffers, keeping space for the G staging buffer
    // of host-pointer transforms
    const size_t g_stage = sizeof(double) * (size_t)p.n * p.n * p.n * p.n * 16;
    auto room = [&]() -> size_t {
      size_t r = ctx->room();
      return r > g_stage ? r - g_stage : 0;
    };
    // --- first-half column chunk: D~ and V of both spaces within ~45% of the room
    auto dv_bytes = [&](int64_t ci) {
      int64_t ldK = round_up(4 * ci, 128);
      return (double)16 * ((double)p.C.Ppad * ldK + (p.gaunt ? 3.0 * p.G.Ppad * ldK : 0.0));
    };
    int64_t ci = p.npair_mo;
    const double room0 = (double)room();
    while (ci > 32 && dv_bytes(ci) > 0.45 * room0) ci = std::max<int64_t>(32, (ci / 2) / 32 * 32);
    if (dv_bytes(ci) > 0.6 * room0) fail(QDCB_E_NOMEM, "no room for a 32-MO-pair column chunk");
    p.ci = (int)ci;
    for (Space *sp : {&p.C, &p.G}) {
      if (sp == &p.G && !p.gaunt) continue;
      sp->ldK = round_up(4 * ci, 128);
      sp->ld = sp->nK * sp->ldK;
      sp->D.alloc(ctx, (size_t)sp->Ppad * sp->ld);
      HIPC(hipMemset(sp->D.p, 0, sp->D.bytes()));
      sp->V.alloc(ctx, (size_t)sp->Ppad * sp->ld);
    }
    // --- second-half slice: dense V, W and G slices within ~1/8 of the room
    {
      int64_t vmax = std::max<int64_t>((int64_t)p.NL * p.NL, (int64_t)p.NS * p.NS);
      if (p.gaunt) vmax = std::max<int64_t>(vmax, (int64_t)p.NL * p.NS);
      int64_t wmax = (int64_t)std::max(p.NL, p.NS) * 4 * p.n;
      size_t per_col = sizeof(double) * (size_t)(vmax + wmax + (int64_t)4 * p.n * p.n);
      int64_t sc = (int64_t)(room() / 8 / per_col);
      sc = std::min<int64_t>(sc, 4 * ci);
      sc = std::min<int64_t>(sc, 65532);
      sc = sc >= 64 ? sc / 64 * 64 : sc / 4 * 4;  // whole MO pairs (4 columns each)
      if (sc < 4) fail(QDCB_E_NOMEM, "no room for a second-half slice");
      p.sc = (int)sc;
      p.Vfull.alloc(ctx, (size_t)p.sc * vmax);
      p.W.alloc(ctx, (size_t)p.sc * wmax);
      p.Gc.alloc(ctx, (size_t)p.sc * 4 * p.n * p.n);
    }
    // --- integral panels: a quarter of what is left, split between the spaces
    {
      size_t slot_bytes = sizeof(double) * TILE * TILE;
      int nsp = p.gaunt ? 2 : 1;
      for (Space *sp : {&p.C, &p.G}) {
        if (sp == &p.G && !p.gaunt) continue;
        int64_t slots = (int64_t)(room() / 4 / nsp / slot_bytes);
        if (sp == &p.G) slots = (int64_t)(room() / 4 / slot_bytes);
        slots = std::min<int64_t>(slots, (int64_t)1 << 22);
        if (slots < sp->ntiles) fail(QDCB_E_NOMEM, "no room for one bra row of integral tiles");
        sp->panel_slots = slots;
        sp->panel.alloc(ctx, (size_t)slots * TILE * TILE);
      }
    }
    ctx->retain();
    *out = pl.release();
  });
}

void qdcb_plan_destroy(qdcb_plan *p) {
  if (!p) return;
  qdcb_ctx *ctx = p->ctx;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  delete p;
  if (prev >= 0) (void)hipSetDevice(prev);
  qdcb_ctx::release_ref(ctx);
}

qdcb_status qdcb_plan_footprint(const qdcb_plan *p, size_t *bytes) {
  return guarded([&] {
    if (!p || !bytes) fail(QDCB_E_INVALID, "NULL argument");
    size_t b = p->C.bytes() + p->G.bytes();
    for (auto *x : {&p->CLd, &p->CSd, &p->Gd, &p->CallL, &p->CallS, &p->ChatL, &p->ChatS,
                    &p->Vfull, &p->W, &p->Gc})
      b += x->bytes();
    for (int K = 0; K < 3; ++K) b += p->AhatK[K].bytes() + p->BhatK[K].bytes();
    b += p->rs.bytes() + p->rowmapL.bytes() + p->rowmapS.bytes() + p->rowmapLS.bytes();
    *bytes = b;
  });
}

}  // extern "C"

namespace {

void check_finite_host(const double *x, size_t n, const char *what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) fail(QDCB_E_INVALID, std::string("non-finite value in ") + what);
}

// Stage timing with events read back after the final synchronization.
struct StageTimer {
  hipStream_t s;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  hipEvent_t open = nullptr;
  int open_stage = -1;
  explicit StageTimer(hipStream_t st) : s(st) {}
  ~StageTimer() {
    for (auto &m : marks) {
      (void)hipEventDestroy(m.second.first);
      (void)hipEventDestroy(m.second.second);
    }
    if (open) (void)hipEventDestroy(open);
  }
  void begin(int stage) {
    HIPC(hipEventCreate(&open));
    HIPC(hipEventRecord(open, s));
    open_stage = stage;
  }
  void end() {
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    HIPC(hipEventRecord(e, s));
    marks.push_back({open_stage, {open, e}});
    open = nullptr;
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

enum { ST_DENS = 0, ST_SCREEN = 1, ST_ERI = 2, ST_FH = 3, ST_SH = 4, ST_ALL = 5 };

void density(qdcb_plan &p, Space &sp, const double *dCL, const double *dCS, int bound_only,
             int i0, int i1, hipStream_t s) {
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
  da.cls = sp.cls.p;
  da.mu = sp.mu.p;
  da.nu = sp.nu.p;
  da.CL = dCL;
  da.CS = dCS;
  da.NL = p.NL;
  da.NS = p.NS;
  da.rs = p.rs.p;
  da.D = sp.D.p;
  da.Dmax = sp.Dmax.p;
  launch_density(da, s);
  HIPC(hipGetLastError());
}

void screen(qdcb_plan &p, Space &sp, hipStream_t s) {
  launch_tile_bounds(sp.ntiles, sp.Q.p, sp.Dmax.p, sp.Qmax.p, sp.Bmax.p, s);
  launch_screen_count(sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau, sp.count.p, s);
  HIPC(hipGetLastError());
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
  launch_screen_fill(0, sp.ntiles, sp.ntiles, sp.Qmax.p, sp.Bmax.p, p.desc.tau,
                     sp.slot_base.p, sp.tasks.p, sp.task_bra.p, s);
  HIPC(hipMemsetAsync(sp.kept.p, 0, sp.kept.bytes(), s));
  HIPC(hipGetLastError());
}

// Integral tiles + first half of one space over its current column chunk.
int first_half(qdcb_plan &p, Space &sp, bool make_tiles, bool count, StageTimer &tm,
               hipStream_t s) {
  int nb = 0;
  for (int b0 = 0; b0 < sp.ntiles;) {
    int b1 = b0;
    int64_t used = 0;
    while (b1 < sp.ntiles && used + sp.cnt[b1] <= sp.panel_slots) used += sp.cnt[b1++];
    if (make_tiles) {
      EriTileArgs ea;
      ea.tasks = sp.tasks.p;
      ea.task_bra = sp.task_bra.p;
      ea.slot0 = sp.base[b0];
      ea.row_first = sp.row_first.p;
      ea.pp = sp.pp.cview();
      ea.Q = sp.Q.p;
      ea.Dmax = sp.Dmax.p;
      ea.cls = sp.cls.p;
      ea.tau = p.desc.tau;
      ea.panel = sp.panel.p;
      ea.kept = count ? sp.kept.p : nullptr;
      tm.begin(ST_ERI);
      launch_eri_tiles(ea, used, s);
      tm.end();
      HIPC(hipGetLastError());
    }
    FirstHalfArgs fa;
    fa.b0 = b0;
    fa.b1 = b1;
    fa.slot_base = sp.slot_base.p;
    fa.count = sp.count.p;
    fa.tasks = sp.tasks.p;
    fa.slot0 = sp.base[b0];
    fa.panel = sp.panel.p;
    fa.D = sp.D.p;
    fa.V = sp.V.p;
    fa.ld = sp.ld;
    fa.ncol_tiles = (int)(sp.ld / 128);
    tm.begin(ST_FH);
    launch_first_half(fa, s);
    tm.end();
    HIPC(hipGetLastError());
    ++nb;
    b0 = b1;
  }
  return nb;
}

}  // namespace

extern "C" {

qdcb_status qdcb_transform(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                           uint32_t flags, void *hip_stream, qdcb_stats *stats) {
  return guarded([&] {
    if (!plan || !CL || !G) fail(QDCB_E_INVALID, "NULL argument");
    qdcb_plan &p = *plan;
    if (p.NS && !CS) fail(QDCB_E_INVALID, "CS is required for this Hamiltonian");
    qdcb_ctx *ctx = p.ctx;
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const bool dev = flags & QDCB_PTR_DEVICE;
    const int n = p.n;
    const size_t nG = (size_t)n * n * n * n * 16;
    const double *dCL = CL, *dCS = CS;
    double *dG = G;
    if (!dev) {
      check_finite_host(CL, (size_t)4 * p.NL * n, "CL");
      if (p.NS) check_finite_host(CS, (size_t)4 * p.NS * n, "CS");
      HIPC(hipMemcpyAsync(p.CLd.p, CL, p.CLd.bytes(), hipMemcpyHostToDevice, s));
      dCL = p.CLd.p;
      if (p.NS) {
        HIPC(hipMemcpyAsync(p.CSd.p, CS, p.CSd.bytes(), hipMemcpyHostToDevice, s));
        dCS = p.CSd.p;
      }
      if (p.Gd.n != nG) p.Gd.alloc(ctx, nG);
      dG = p.Gd.p;
    }
    std::vector<Space *> spaces{&p.C};
    if (p.gaunt) spaces.push_back(&p.G);
    StageTimer tm(s);
    hipEvent_t ev_start;
    HIPC(hipEventCreate(&ev_start));
    HIPC(hipEventRecord(ev_start, s));

    // density bounds and screening (the kept set is the same for every chunk)
    for (Space *sp : spaces) {
      tm.begin(ST_DENS);
      density(p, *sp, dCL, dCS, 1, 0, p.npair_mo, s);
      tm.end();
      tm.begin(ST_SCREEN);
      screen(p, *sp, s);
      tm.end();
    }
    // second-half coefficient matrices
    launch_build_coef_mats(p.NL, n, dCL, -1, p.CallL.p, p.ChatL.p, s);
    if (p.NS) launch_build_coef_mats(p.NS, n, dCS, -1, p.CallS.p, p.ChatS.p, s);
    if (p.gaunt)
      for (int K = 0; K < 3; ++K) {
        launch_build_coef_mats(p.NL, n, dCL, K, p.CallL.p, p.AhatK[K].p, s);
        launch_build_coef_mats(p.NS, n, dCS, K, p.CallS.p, p.BhatK[K].p, s);
      }
    HIPC(hipGetLastError());

    int nb = 0;
    double mfma = 0;
    for (int i0 = 0; i0 < p.npair_mo; i0 += p.ci) {
      const int i1 = std::min(p.npair_mo, i0 + p.ci);
      for (Space *sp : spaces) {
        tm.begin(ST_DENS);
        density(p, *sp, dCL, dCS, 0, i0, i1, s);
        tm.end();
        const bool resident = sp->total <= sp->panel_slots;
        nb += first_half(p, *sp, !resident || i0 == 0, i0 == 0, tm, s);
        mfma += 2.0 * TILE * TILE * (double)sp->ld * (double)sp->total;
      }
      // second half of this chunk's columns, slice by slice
      tm.begin(ST_SH);
      const int64_t cend = 4LL * i1;
      for (int64_t c0 = 4LL * i0; c0 < cend; c0 += p.sc) {
        const int nc = (int)std::min<int64_t>(p.sc, cend - c0);
        const int64_t lc0 = c0 - 4LL * i0;
        for (int cls = 0; cls < (p.NS ? 2 : 1); ++cls) {
          const int N = cls ? p.NS : p.NL;
          launch_unpack(N, N, cls ? p.rowmapS.p : p.rowmapL.p, p.C.V.p, p.C.ld, lc0, nc,
                        p.Vfull.p, s);
          launch_dgemm_batched(0, N, 4 * n, N, 1.0, p.Vfull.p, N, (int64_t)N * N,
                               cls ? p.CallS.p : p.CallL.p, 4 * n, 0, 0.0, p.W.p, 4 * n,
                               (int64_t)N * 4 * n, nc, s);
          launch_dgemm_batched(1, 4 * n, n, 4 * N, 1.0, cls ? p.ChatS.p : p.ChatL.p, 4 * n, 0,
                               p.W.p, n, (int64_t)N * 4 * n, cls ? 1.0 : 0.0, p.Gc.p, n,
                               (int64_t)4 * n * n, nc, s);
        }
        launch_pack(n, p.rs.p, c0, nc, p.Gc.p, dG, 1.0, 0, s);
        if (p.gaunt) {
          const int NL = p.NL, NS = p.NS;
          for (int K = 0; K < 3; ++K) {
            launch_unpack(NL, NS, p.rowmapLS.p, p.G.V.p, p.G.ld, K * p.G.ldK + lc0, nc,
                          p.Vfull.p, s);
            // conj(C^L) e_K (V C^S)
            launch_dgemm_batched(0, NL, 4 * n, NS, 1.0, p.Vfull.p, NS, (int64_t)NL * NS,
                                 p.CallS.p, 4 * n, 0, 0.0, p.W.p, 4 * n, (int64_t)NL * 4 * n, nc,
                                 s);
            launch_dgemm_batched(1, 4 * n, n, 4 * NL, 1.0, p.AhatK[K].p, 4 * n, 0, p.W.p, n,
                                 (int64_t)NL * 4 * n, K ? 1.0 : 0.0, p.Gc.p, n,
                                 (int64_t)4 * n * n, nc, s);
            // conj(C^S) e_K (V^T C^L)
            launch_dgemm_batched(1, NS, 4 * n, NL, 1.0, p.Vfull.p, NS, (int64_t)NL * NS,
                                 p.CallL.p, 4 * n, 0, 0.0, p.W.p, 4 * n, (int64_t)NS * 4 * n, nc,
                                 s);
            launch_dgemm_batched(1, 4 * n, n, 4 * NS, 1.0, p.BhatK[K].p, 4 * n, 0, p.W.p, n,
                                 (int64_t)NS * 4 * n, 1.0, p.Gc.p, n, (int64_t)4 * n * n, nc,
                                 s);
          }
          launch_pack(n, p.rs.p, c0, nc, p.Gc.p, dG, -1.0, 1, s);
        }
        HIPC(hipGetLastError());
      }
      tm.end();
    }
    hipEvent_t ev_end;
    HIPC(hipEventCreate(&ev_end));
    HIPC(hipEventRecord(ev_end, s));
    tm.marks.push_back({ST_ALL, {ev_start, ev_end}});
    if (!dev) HIPC(hipMemcpyAsync(G, dG, nG * sizeof(double), hipMemcpyDeviceToHost, s));
    unsigned long long kc[4] = {0, 0, 0, 0}, kg[4] = {0, 0, 0, 0};
    HIPC(hipMemcpyAsync(kc, p.C.kept.p, sizeof(kc), hipMemcpyDeviceToHost, s));
    if (p.gaunt) HIPC(hipMemcpyAsync(kg, p.G.kept.p, sizeof(kg), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    p.have_last = true;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->ms_density = tm.total(ST_DENS);
      stats->ms_screen = tm.total(ST_SCREEN);
      stats->ms_eri = tm.total(ST_ERI);
      stats->ms_first_half = tm.total(ST_FH);
      stats->ms_second_half = tm.total(ST_SH);
      stats->ms_total = tm.total(ST_ALL);
      double ktot = 0;
      for (int c = 0; c < 4; ++c) {
        stats->kept[c] = (int64_t)kc[c];
        ktot += (double)kc[c];
      }
      const int64_t nLL = p.nLL, nSS = p.nSS;
      stats->total[0] = nLL * nLL;
      stats->total[1] = nLL * nSS;
      stats->total[2] = nSS * nLL;
      stats->total[3] = nSS * nSS;
      stats->kept_gaunt = (int64_t)kg[0];
      stats->total_gaunt = p.gaunt ? p.G.P * p.G.P : 0;
      stats->tiles_kept = p.C.total + (p.gaunt ? p.G.total : 0);
      stats->tiles_total = (int64_t)p.C.ntiles * p.C.ntiles +
                           (p.gaunt ? (int64_t)p.G.ntiles * p.G.ntiles : 0);
      stats->flops_first_half =
          2.0 * (double)p.ncol * ktot + 2.0 * 3.0 * (double)p.ncol * (double)kg[0];
      double f2 = 0;
      for (int cls = 0; cls < (p.NS ? 2 : 1); ++cls) {
        double N = cls ? p.NS : p.NL;
        f2 += (8.0 * N * N * n + 32.0 * N * n * n) * (double)p.ncol;
      }
      if (p.gaunt)
        f2 += 3.0 * (16.0 * p.NL * (double)p.NS * n + 32.0 * (p.NL + p.NS) * (double)n * n) *
              (double)p.ncol;
      stats->flops_second_half = f2;
      stats->flops_mfma = mfma;
      stats->n_batches = tm.launches(ST_FH);
      stats->n_chunks = (p.npair_mo + p.ci - 1) / p.ci;
      (void)nb;
    }
  });
}

qdcb_status qdcb_plan_fetch(const qdcb_plan *p, int32_t what, void *host_out, size_t bytes) {
  return guarded([&] {
    if (!p || !host_out) fail(QDCB_E_INVALID, "NULL argument");
    DeviceGuard g(p->ctx->device);
    const bool gaunt_item = what == QDCB_FETCH_DMAX_GAUNT || what == QDCB_FETCH_Q_GAUNT;
    if (what != QDCB_FETCH_DMAX && what != QDCB_FETCH_Q && !gaunt_item)
      fail(QDCB_E_INVALID, "unknown item");
    if (gaunt_item && !p->gaunt) fail(QDCB_E_INVALID, "the plan has no Gaunt classes");
    const Space &sp = gaunt_item ? p->G : p->C;
    if (bytes < (size_t)sp.P * sizeof(double)) fail(QDCB_E_INVALID, "output too small");
    const bool dm = what == QDCB_FETCH_DMAX || what == QDCB_FETCH_DMAX_GAUNT;
    if (dm && !p->have_last) fail(QDCB_E_INVALID, "no transform yet");
    std::vector<double> sorted(sp.Ppad);
    HIPC(hipMemcpy(sorted.data(), dm ? sp.Dmax.p : sp.Q.p, sp.Ppad * sizeof(double),
                   hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_out);
    const int64_t nLL = p->nLL;
    for (int64_t r = 0; r < sp.P; ++r) {
      int64_t idx = sp.h_key[r];
      if (!gaunt_item && sp.h_cls[r] == 1) idx += nLL;
      o[idx] = sorted[r];
    }
  });
}

}  // extern "C"
