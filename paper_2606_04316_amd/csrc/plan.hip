// plan.hip -- C ABI: plans (pair spaces, buffers, sizing) and fetches.
//
// A plan holds one or two pair spaces:
//   Coulomb  LL pairs (mu <= nu) and, for DC/DCG, SS pairs: the classes of
//            Eq. (DCInt); one AO integral tile serves every class pair because
//            the stand-in small-component functions are scalar s Gaussians.
//   Gaunt    ordered LS pairs (mu in L, nu in S) of Eq. (GauntInt), with three
//            Pauli components K per MO-pair column.
// Rows of a space are ordered by decreasing Schwarz factor and padded to a
// multiple of 64.  The transformation itself is driven by transform.hip.
#include <chrono>
#include <deque>
#include <cstdlib>

#include "plan.h"

using namespace qdcb;

namespace {

// Sorted rows of a space: order by decreasing Q (stable in the input order).
struct RowSrc {
  double Q;
  int32_t cls, mu, nu;
  int64_t key;
  int64_t src_first;
  int32_t cnt;
  int which;        // which source store
  int32_t kept = 0;  // primitive pairs kept by primitive screening
  int32_t code = 0;  // pair_code(cf, cg) of Cartesian bases (0: s s)
};

// Rows ordered by Schwarz factor; band_rows > 0: within each band of that many
// rows, by the number of primitive pairs kept by primitive screening
// (decreasing, Schwarz order among equals).
void build_space(qdcb_ctx *ctx, Space &sp, std::vector<RowSrc> &rows,
                 const std::vector<const PairStore *> &stores, int64_t band_rows) {
  // primitive pairs kept per row (rows in their input order)
  for (size_t w = 0; w < stores.size(); ++w) {
    std::vector<int64_t> idx, first;
    std::vector<int32_t> cnt, code;
    for (size_t i = 0; i < rows.size(); ++i)
      if (rows[i].which == (int)w) {
        idx.push_back((int64_t)i);
        first.push_back(rows[i].src_first);
        cnt.push_back(rows[i].cnt);
        code.push_back(rows[i].code);
      }
    if (idx.empty()) continue;
    DBuf<int64_t> dfirst(POOLED);
    DBuf<int32_t> dcnt(POOLED), dk(POOLED), dcode(POOLED);
    dfirst.upload(ctx, first);
    dcnt.upload(ctx, cnt);
    dcode.upload(ctx, code);
    dk.alloc(ctx, idx.size());
    launch_prim_count((int64_t)idx.size(), dfirst.p, dcnt.p, dcode.p, stores[w]->cview(),
                      PRIM_EPS, dk.p, nullptr);
    HIPC(hipGetLastError());
    std::vector<int32_t> k(idx.size());
    HIPC(hipMemcpy(k.data(), dk.p, k.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < idx.size(); ++i) rows[idx[i]].kept = k[i];
  }
  std::stable_sort(rows.begin(), rows.end(),
                   [](const RowSrc &a, const RowSrc &b) { return a.Q > b.Q; });
  for (int64_t b0 = 0; band_rows > 0 && b0 < (int64_t)rows.size(); b0 += band_rows) {
    const int64_t b1 = std::min<int64_t>((int64_t)rows.size(), b0 + band_rows);
    std::stable_sort(rows.begin() + b0, rows.begin() + b1,
                     [](const RowSrc &a, const RowSrc &b) { return a.kept > b.kept; });
  }
  sp.P = (int64_t)rows.size();
  sp.Ppad = std::max<int64_t>(round_up(sp.P, TILE), TILE);
  // unique-tile slot numbers are int32: ntiles (ntiles + 1) / 2 < 2^31
  if (sp.Ppad / TILE > 65535) fail(QDCB_E_INVALID, "too many pairs (at most 65535 tiles)");
  sp.ntiles = (int)(sp.Ppad / TILE);
  sp.h_cls.assign(sp.Ppad, -1);
  sp.h_mu.assign(sp.Ppad, 0);
  sp.h_nu.assign(sp.Ppad, 0);
  sp.h_key.assign(sp.Ppad, -1);
  std::vector<double> hQ(sp.Ppad, 0.0);
  std::vector<int32_t> hcode(sp.Ppad, 0);
  const size_t ns = stores.size();
  std::vector<std::vector<int64_t>> src(ns), dst(ns), rowidx(ns);
  std::vector<std::vector<int32_t>> cnt(ns), scode(ns);
  bool cart = false;
  for (int64_t r = 0; r < sp.P; ++r) {
    const RowSrc &s = rows[r];
    sp.h_cls[r] = s.cls;
    sp.h_mu[r] = s.mu;
    sp.h_nu[r] = s.nu;
    sp.h_key[r] = s.key;
    hQ[r] = s.Q;
    hcode[r] = s.code;
    cart = cart || s.code != 0;
    src[s.which].push_back(s.src_first);
    cnt[s.which].push_back(s.cnt);
    scode[s.which].push_back(s.code);
    rowidx[s.which].push_back(r);
  }
  for (const PairStore *st : stores) cart = cart || st->pa.p;
  if (cart) sp.code.upload(ctx, hcode);
  // primitive pairs kept per row after primitive screening
  std::deque<DBuf<int64_t>> dsrc;  // deque: its elements never move
  std::deque<DBuf<int32_t>> dcnt, dscode;
  for (size_t w = 0; w < ns; ++w) {
    dsrc.emplace_back(POOLED);
    dcnt.emplace_back(POOLED);
    dscode.emplace_back(POOLED);
  }
  std::vector<int32_t> kept_prims(sp.Ppad, 0);
  for (int64_t r = 0; r < sp.P; ++r) kept_prims[r] = rows[r].kept;
  for (size_t w = 0; w < ns; ++w) {
    if (src[w].empty()) continue;
    dsrc[w].upload(ctx, src[w]);
    dcnt[w].upload(ctx, cnt[w]);
    dscode[w].upload(ctx, scode[w]);
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
  sp.pp.alloc(ctx, (size_t)std::max<int64_t>(rf[sp.Ppad], 1), cart);
  for (size_t w = 0; w < ns; ++w) {
    if (src[w].empty()) continue;
    DBuf<int64_t> dd(POOLED);
    dd.upload(ctx, dst[w]);
    launch_gather_pairs((int64_t)src[w].size(), dsrc[w].p, dcnt[w].p, dscode[w].p, dd.p,
                        stores[w]->cview(), sp.pp.view(), PRIM_EPS, nullptr);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(nullptr));
  }
  sp.Dmax.alloc(ctx, sp.Ppad);
  // intra-tile row order buffers (row data of the integral tiles in that order)
  sp.perm.alloc(ctx, sp.Ppad);
  sp.sthr.alloc(ctx, (size_t)sp.ntiles * 4);
  sp.wQ.alloc(ctx, sp.Ppad);
  sp.wDmax.alloc(ctx, sp.Ppad);
  sp.wcls.alloc(ctx, sp.Ppad);
  sp.wmu.alloc(ctx, sp.Ppad);
  sp.wnu.alloc(ctx, sp.Ppad);
  if (cart) sp.wcode.alloc(ctx, sp.Ppad);
  sp.wrow_first.alloc(ctx, sp.Ppad + 1);
  sp.wpp.alloc(ctx, (size_t)std::max<int64_t>(rf[sp.Ppad], 1), cart);
  sp.steps.alloc(ctx, 1);
  sp.Qmax.alloc(ctx, sp.ntiles);
  sp.Bmax.alloc(ctx, sp.ntiles);
  sp.count.alloc(ctx, sp.ntiles);
  sp.slot_base.alloc(ctx, sp.ntiles);
  sp.kept.alloc(ctx, 4);
  sp.dtotal.alloc(ctx, 1);
  sp.overflow.alloc(ctx, 1);
}

// Stage times of plan creation on stderr when QDCB_TRACE_PLAN is set (host
// wall clock, after a device synchronization at each mark).
struct PlanTrace {
  bool on = std::getenv("QDCB_TRACE_PLAN") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  std::string line;
  void mark(const char *what) {
    if (!on) return;
    (void)hipDeviceSynchronize();
    const auto now = std::chrono::steady_clock::now();
    char b[96];
    std::snprintf(b, sizeof b, " %s %.2f", what,
                  std::chrono::duration<double, std::milli>(now - t).count());
    line += b;
    t = now;
  }
  ~PlanTrace() {
    if (on && !line.empty()) std::fprintf(stderr, "qdcb plan ms:%s\n", line.c_str());
  }
};

// Taylor table of the Boys function, tab[8 i + k] = (2/sqrt(pi)) (-1)^k F_k(T_i) / k! at
// T_i = i / 8: F_7 from its series e^-T sum_j (2T)^j / ((2m+1)(2m+3)...(2m+2j+1)),
// then the stable downward recursion F_{m-1} = (2 T F_m + e^-T) / (2m - 1),
// in long double.
std::vector<double> boys_table() {
  std::vector<double> tab((size_t)BOYS_N * 8);
  for (int i = 0; i < BOYS_N; ++i) {
    const long double T = (long double)i / 8.0L, eT = expl(-T);
    long double term = 1.0L / 15.0L, sum = term;  // m = 7: first term 1/(2m+1)
    for (int j = 1; j < 400; ++j) {
      term *= 2.0L * T / (15.0L + 2.0L * j);
      sum += term;
      if (term < 1e-22L * sum) break;
    }
    long double F[8];
    F[7] = eT * sum;
    for (int m = 7; m >= 1; --m) F[m - 1] = (2.0L * T * F[m] + eT) / (2.0L * m - 1.0L);
    // scaled by 2 / sqrt(pi), the factor of the kernel erf(sqrt(rho) R) / R
    const long double two_over_sqrtpi = 2.0L / sqrtl(3.14159265358979323846264338327950288L);
    long double fact = 1.0L;
    for (int k = 0; k < 8; ++k) {
      if (k) fact *= k;
      tab[(size_t)8 * i + k] = (double)(two_over_sqrtpi * (k & 1 ? -F[k] : F[k]) / fact);
    }
  }
  return tab;
}

// Table of the gauge tiles: tab[BOYS_LD i + k] = (2/sqrt(pi)) F_k(T_i), k = 0 .. 9,
// T_i = i / 8, by the same series and downward recursion (long double).
std::vector<double> boys_table3() {
  std::vector<double> tab((size_t)BOYS_N * BOYS_LD);
  const long double two_over_sqrtpi = 2.0L / sqrtl(3.14159265358979323846264338327950288L);
  for (int i = 0; i < BOYS_N; ++i) {
    const long double T = (long double)i / 8.0L, eT = expl(-T);
    long double term = 1.0L / 19.0L, sum = term;  // m = 9
    for (int j = 1; j < 400; ++j) {
      term *= 2.0L * T / (19.0L + 2.0L * j);
      sum += term;
      if (term < 1e-22L * sum) break;
    }
    long double F[10];
    F[9] = eT * sum;
    for (int m = 9; m >= 1; --m) F[m - 1] = (2.0L * T * F[m] + eT) / (2.0L * m - 1.0L);
    for (int k = 0; k < 10; ++k) tab[(size_t)BOYS_LD * i + k] = (double)(two_over_sqrtpi * F[k]);
  }
  return tab;
}

// Table of the Cartesian tiles: tab[LD i + k] = (2/sqrt(pi)) F_k(T_i), k < LD
// (BOYS_LDC for s/p tiles, BOYS_LDG for the general tiles), T_i = i / 8, by the
// same series and downward recursion (long double).
template <int LD = BOYS_LDC>
std::vector<double> boys_table_cart() {
  std::vector<double> tab((size_t)BOYS_N * LD);
  const long double two_over_sqrtpi = 2.0L / sqrtl(3.14159265358979323846264338327950288L);
  constexpr int M = LD - 1;
  for (int i = 0; i < BOYS_N; ++i) {
    const long double T = (long double)i / 8.0L, eT = expl(-T);
    long double term = 1.0L / (2.0L * M + 1.0L), sum = term;
    for (int j = 1; j < 400; ++j) {
      term *= 2.0L * T / (2.0L * M + 1.0L + 2.0L * j);
      sum += term;
      if (term < 1e-22L * sum) break;
    }
    long double F[LD];
    F[M] = eT * sum;
    for (int m = M; m >= 1; --m) F[m - 1] = (2.0L * T * F[m] + eT) / (2.0L * m - 1.0L);
    for (int k = 0; k < LD; ++k) tab[(size_t)LD * i + k] = (double)(two_over_sqrtpi * F[k]);
  }
  return tab;
}

}  // namespace

namespace qdcb {

double dv_bytes(const qdcb_plan &p, int64_t ci) {
  const int64_t ldK = round_up(4 * ci, 128);
  // D~ and V in FP64, and (mixed precision) the FP32 copy of D~
  const double per = p.desc.prec == QDCB_PREC_MIXED ? 20.0 : 16.0;
  return per * ((double)p.C.Ppad * ldK + (p.gaunt ? 3.0 * p.G.Ppad * ldK : 0.0));
}

size_t g_stage_bytes(const qdcb_plan &p) {
  return sizeof(double) * (size_t)p.n * p.n * p.n * p.n * (p.spinor ? 2 : 16);
}

// (Re)allocate the sized buffers: D~ and V of the column chunk, the
// second-half slices and the integral panels.  slotsC, slotsG = 0: the
// default split (D~ and V within ~45% of the room, the slices ~1/8 of the
// rest, the panels a quarter of what is left); otherwise panels of exactly
// that many slots and the largest column chunk that fits beside them.  The
// G staging buffer of host-pointer transforms is kept out of the room.
void size_plan(qdcb_plan &p, int64_t slotsC, int64_t slotsG) {
  qdcb_ctx *ctx = p.ctx;
  for (Space *sp : {&p.C, &p.G}) {
    sp->D.free();
    sp->Dlo.free();
    sp->V.free();
    sp->panel.free();
    sp->panel3.free();
    sp->panel_slots = 0;
  }
  p.W.free();
  p.Gc.free();
  const size_t g_stage = g_stage_bytes(p);
  auto room = [&]() -> size_t {
    size_t r = ctx->room();
    return r > g_stage ? r - g_stage : 0;
  };
  const size_t slot_bytes = sizeof(double) * TILE * TILE;
  const int64_t wmax = (int64_t)std::max(p.NL, p.NS) * 4 * p.n;
  const size_t per_col = sizeof(double) * (size_t)(wmax + (int64_t)4 * p.n * p.n);
  // an L-S slot of a DCB plan holds six gauge (or Breit) tiles, and the Gaunt
  // tile too when the two terms are contracted apart (mixed precision)
  const int gmul = p.gauge ? (p.fused_breit ? 6 : 7) : 1;
  const bool fixed = slotsC > 0;
  const double panels = fixed ? (double)slot_bytes * (slotsC + gmul * slotsG) : 0.0;
  // --- first-half column chunk
  int64_t ci = p.npair_mo;
  const double room0 = (double)room();
  if (fixed) {
    // beside the panels, keep ~1/8 of the remainder for the second-half slices
    const double avail = (room0 - panels) * 0.85;
    while (ci > 32 && dv_bytes(p, ci) > avail) ci = std::max<int64_t>(32, (ci / 2) / 32 * 32);
    if (dv_bytes(p, ci) > avail) fail(QDCB_E_NOMEM, "no room for the panels and a column chunk");
  } else {
    while (ci > 32 && dv_bytes(p, ci) > 0.45 * room0) ci = std::max<int64_t>(32, (ci / 2) / 32 * 32);
    if (dv_bytes(p, ci) > 0.6 * room0) fail(QDCB_E_NOMEM, "no room for a 32-MO-pair column chunk");
  }
  p.ci = (int)ci;
  for (Space *sp : {&p.C, &p.G}) {
    if (sp == &p.G && !p.gaunt) continue;
    sp->ldK = round_up(4 * ci, 128);
    sp->ld = sp->nK * sp->ldK;
    sp->ld_cap = sp->ld;
    sp->D.alloc(ctx, (size_t)sp->Ppad * sp->ld);
    HIPC(hipMemset(sp->D.p, 0, sp->D.bytes()));
    if (p.desc.prec == QDCB_PREC_MIXED) sp->Dlo.alloc(ctx, (size_t)sp->Ppad * sp->ld);
    sp->V.alloc(ctx, (size_t)sp->Ppad * sp->ld);
  }
  // the zeroing runs on the null stream, which is not ordered with the
  // caller's (non-blocking) streams, and may wait there behind other threads'
  // set-up work: it must be complete before a transform on another stream
  // writes the densities (a resize happens inside the first transform)
  HIPC(hipStreamSynchronize(nullptr));
  // --- second-half slice: W and G slices
  {
    const double avail = fixed ? (double)room() - panels : (double)room() / 8;
    int64_t sc = avail > 0 ? (int64_t)(avail / per_col) : 0;
    sc = std::min<int64_t>(sc, 4 * ci);
    sc = std::min<int64_t>(sc, 65532);
    sc = sc >= 64 ? sc / 64 * 64 : sc / 4 * 4;  // whole MO pairs (4 columns each)
    if (sc < 4) fail(QDCB_E_NOMEM, "no room for a second-half slice");
    p.sc = (int)sc;
    p.W.alloc(ctx, (size_t)p.sc * wmax);
    p.Gc.alloc(ctx, (size_t)p.sc * 4 * p.n * p.n);
  }
  // --- integral panels
  const int nsp = p.gaunt ? 2 : 1;
  for (Space *sp : {&p.C, &p.G}) {
    if (sp == &p.G && !p.gaunt) continue;
    int64_t slots;
    if (fixed) {
      slots = sp == &p.G ? slotsG : slotsC;
    } else {
      slots = (int64_t)(room() / 4 / nsp / slot_bytes);
      if (sp == &p.G) slots = (int64_t)(room() / 4 / (gmul * slot_bytes));
    }
    slots = std::min<int64_t>(slots, (int64_t)1 << 23);
    if (slots < sp->ntiles) fail(QDCB_E_NOMEM, "no room for one bra row of integral tiles");
    sp->panel_slots = slots;
    if (!(sp == &p.G && p.fused_breit)) sp->panel.alloc(ctx, (size_t)slots * TILE * TILE);
    if (sp == &p.G && p.gauge) sp->panel3.alloc(ctx, (size_t)slots * 6 * TILE * TILE);
  }
}

// Make every kept directed tile of both spaces resident (slack x the kept
// counts of the current screening) when the budget allows it with a column
// chunk of at least 32 MO pairs; otherwise keep the current sizing (panel
// batches).  Returns true when the buffers were reallocated.
bool ensure_residency(qdcb_plan &p, double slack) {
  const int64_t needC = std::max<int64_t>((int64_t)(p.C.total * slack) + 1, p.C.ntiles);
  const int64_t needG = p.gaunt ? std::max<int64_t>((int64_t)(p.G.total * slack) + 1, p.G.ntiles) : 0;
  if (needC <= p.C.panel_slots && (!p.gaunt || needG <= p.G.panel_slots)) return false;
  if (needC > ((int64_t)1 << 23) || needG > ((int64_t)1 << 23)) return false;
  // memory the resizable buffers may use: what they hold now plus the free room
  size_t held = p.W.bytes() + p.Gc.bytes();
  for (const Space *sp : {&p.C, &p.G})
    held += sp->D.bytes() + sp->Dlo.bytes() + sp->V.bytes() + sp->panel.bytes() +
            sp->panel3.bytes();
  const size_t g_stage = g_stage_bytes(p);
  // within the context budget and within what the device has free now (other
  // allocations of the process, such as the caller's G, count against it)
  size_t fr = 0, tot = 0;
  HIPC(hipMemGetInfo(&fr, &tot));
  fr += dev_cached(p.ctx->device);  // cached blocks are reusable
  const double room0 = std::min((double)p.ctx->room(), 0.95 * (double)fr) + (double)held -
                       (double)g_stage;
  const double panels = (double)sizeof(double) * TILE * TILE *
                        (needC + (p.gauge ? (p.fused_breit ? 6 : 7) : 1) * needG);
  const int64_t wmax = (int64_t)std::max(p.NL, p.NS) * 4 * p.n;
  const double per_col = (double)sizeof(double) * (wmax + 4.0 * p.n * p.n);
  if (panels + dv_bytes(p, 32) + 64.0 * per_col > 0.85 * room0) return false;
  HIPC(hipDeviceSynchronize());
  try {
    size_plan(p, needC, needG);
  } catch (const Fail &) {
    // the device could not hold the resident sizing after all: return to the
    // default sizing (panel batches) so that the plan stays usable
    (void)hipGetLastError();
    size_plan(p, 0, 0);
    return false;
  }
  return true;
}

}  // namespace qdcb

extern "C" {

qdcb_status qdcb_plan_create(qdcb_ctx *ctx, const qdcb_basis *L, const qdcb_basis *S,
                             const qdcb_plan_desc *desc, qdcb_plan **out) {
  return guarded([&] {
    if (!ctx || !L || !desc || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (desc->ham != QDCB_HAM_LL && desc->ham != QDCB_HAM_DC && desc->ham != QDCB_HAM_DCG &&
        desc->ham != QDCB_HAM_DCB)
      fail(QDCB_E_INVALID, "unknown Hamiltonian");
    if (desc->prec != QDCB_PREC_FP64 && desc->prec != QDCB_PREC_MIXED)
      fail(QDCB_E_INVALID, "unknown precision mode");
    if (desc->prec == QDCB_PREC_MIXED &&
        !(std::isfinite(desc->tier_fp32) && std::isfinite(desc->tier_bf16) &&
          desc->tier_bf16 >= 0 && desc->tier_bf16 <= desc->tier_fp32))
      fail(QDCB_E_INVALID, "mixed precision needs finite tiers 0 <= tier_bf16 <= tier_fp32");
    if ((desc->ham == QDCB_HAM_LL) != (S == nullptr))
      fail(QDCB_E_INVALID, "S must be NULL exactly for QDCB_HAM_LL");
    if (desc->n_mo < 1 || desc->n_mo > 512) fail(QDCB_E_INVALID, "n_mo must be in [1, 512]");
    if (!std::isfinite(desc->tau) || desc->tau < 0) fail(QDCB_E_INVALID, "tau must be >= 0");
    if (desc->flags &
        ~(int32_t)(QDCB_PLAN_DIRECTED_TILES | QDCB_PLAN_TIER_BY_G | QDCB_PLAN_SPINOR |
                   QDCB_PLAN_PRIM_BANDS | QDCB_PLAN_SCHWARZ_ROWS))
      fail(QDCB_E_INVALID, "unknown plan flag");
    if ((desc->flags & QDCB_PLAN_PRIM_BANDS) && (desc->flags & QDCB_PLAN_SCHWARZ_ROWS))
      fail(QDCB_E_INVALID, "QDCB_PLAN_PRIM_BANDS and QDCB_PLAN_SCHWARZ_ROWS exclude each other");
    // bases may belong to another context (resident, shared) on the same device
    if (L->ctx->device != ctx->device || (S && S->ctx->device != ctx->device))
      fail(QDCB_E_INVALID, "basis on another device");
    DeviceGuard g(ctx->device);
    PlanTrace trace;
    std::unique_ptr<qdcb_plan> pl(new qdcb_plan());
    qdcb_plan &p = *pl;
    p.ctx = ctx;
    p.nLL = L->npairs;
    p.nSS = S ? S->npairs : 0;
    p.desc = *desc;
    p.n = desc->n_mo;
    p.NL = L->nfunc;
    p.NS = S ? S->nfunc : 0;
    p.gaunt = desc->ham == QDCB_HAM_DCG || desc->ham == QDCB_HAM_DCB;
    p.gauge = desc->ham == QDCB_HAM_DCB;
    p.fused_breit = p.gauge && desc->prec == QDCB_PREC_FP64;
    p.cart = L->has_p() || (S && S->has_p());
    p.gen = L->has_gen() || (S && S->has_gen());
    p.gen_f = L->has_f() || (S && S->has_f());
    {
      const char *e = std::getenv("QDCB_TILE_ORDER");
      p.tile_order = !(e && e[0] == '0');
    }
    p.spinor = desc->flags & QDCB_PLAN_SPINOR;
    if (p.spinor) {  // pairs of spinors c <= d, two pairs per four-column group
      p.npair_s = p.n * (p.n + 1) / 2;
      p.npair_mo = (p.npair_s + 1) / 2;
    } else {
      p.npair_mo = p.n * (p.n + 1) / 2;
    }
    p.ncol = 4LL * p.npair_mo;
    // row order: primitive bands of 8 tiles (default), or plain Schwarz order
    const int64_t bands = (desc->flags & QDCB_PLAN_SCHWARZ_ROWS) ? 0 : 8 * TILE;

    // --- Coulomb space: LL pairs, then SS pairs
    {
      std::vector<RowSrc> rows;
      rows.reserve(L->npairs + (S ? S->npairs : 0));
      auto add = [&](const qdcb_basis *B, int cls, int which) {
        for (int nu = 0; nu < B->nfunc; ++nu)
          for (int mu = 0; mu <= nu; ++mu) {
            int64_t c = qdcb_basis::canon(mu, nu);
            RowSrc r{B->Q[c], cls, mu, nu, c, B->pair_first[c],
                     (int32_t)(B->pair_first[c + 1] - B->pair_first[c]), which};
            r.code = pair_code(B->cart_of(mu), B->cart_of(nu));
            rows.push_back(r);
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
      build_space(ctx, p.C, rows, stores, bands);
      trace.mark("coulomb_space");
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
      PairStore ls(POOLED);
      DBuf<int32_t> dm(POOLED), dn(POOLED);
      DBuf<int64_t> dpf(POOLED);
      DBuf<double> dQ(POOLED);
      dm.upload(ctx, pm);
      dn.upload(ctx, pn);
      dpf.upload(ctx, pf);
      ls.alloc(ctx, (size_t)pf[nls], p.cart);
      launch_pair_data(nls, dm.p, dn.p, dpf.p, L->cent.p, L->dfirst.p, L->exps.p, L->nc.p,
                       L->dcart.p, S->cent.p, S->dfirst.p, S->exps.p, S->nc.p, S->dcart.p,
                       ls.view(), nullptr);
      std::vector<int32_t> lcode(p.cart ? nls : 0);
      for (int64_t i = 0; p.cart && i < nls; ++i)
        lcode[i] = pair_code(L->cart_of(pm[i]), S->cart_of(pn[i]));
      DBuf<int32_t> dlcode(POOLED);
      if (p.cart) dlcode.upload(ctx, lcode);
      dQ.alloc(ctx, nls);
      launch_schwarz(nls, dpf.p, ls.cview(), dlcode.p, dQ.p, nullptr);
      HIPC(hipGetLastError());
      std::vector<double> hQ(nls);
      HIPC(hipMemcpy(hQ.data(), dQ.p, nls * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<RowSrc> rows(nls);
      for (int64_t i = 0; i < nls; ++i) {
        rows[i] = RowSrc{hQ[i], 0, pm[i], pn[i], i, pf[i], (int32_t)(pf[i + 1] - pf[i]), 0};
        rows[i].code = p.cart ? lcode[i] : 0;
      }
      p.G.gaunt = 1;
      p.G.nK = 3;
      build_space(ctx, p.G, rows, {&ls}, bands);
      trace.mark("gaunt_space");
    }

    // --- index tables
    std::vector<int32_t> rs(p.spinor ? 2 * (size_t)p.npair_mo : (size_t)p.npair_mo, -1);
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
    trace.mark("index_tables");
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
      size_t ucap = (size_t)sp->ntiles * (size_t)(sp->ntiles + 1) / 2;
      sp->ucount.alloc(ctx, sp->ntiles);
      sp->ubase.alloc(ctx, sp->ntiles);
      sp->utask_k.alloc(ctx, ucap);
      sp->utask_b.alloc(ctx, ucap);
      sp->Dtmax.alloc(ctx, sp->ntiles);
      if (desc->prec == QDCB_PREC_MIXED) {
        sp->ttasks.alloc(ctx, cap);
        sp->trank.alloc(ctx, cap);
        sp->tdesc.alloc(ctx, cap);
        sp->tcount.alloc(ctx, 3 * (size_t)sp->ntiles);
        sp->toff.alloc(ctx, 3 * (size_t)sp->ntiles);
      }
      sp->uslot_bk.alloc(ctx, ucap);
      sp->uslot_kb.alloc(ctx, ucap);
      sp->dmap.alloc(ctx, cap);
      sp->udtotal.alloc(ctx, 1);
      sp->uoverflow.alloc(ctx, 1);
      sp->uorder.alloc(ctx, ucap);
      sp->lpt.alloc(ctx, LPT_WORK);
    }
    trace.mark("coef_and_task_buffers");
    // --- launch choices and the shape key of the tuning cache
    HIPC(hipDeviceGetAttribute(&p.n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    p.tune.eri_sched = 1;  // faster or equal on every workload measured
    p.tune.fh_order = 0;
    p.tune.sq_tile = (p.n % 2 == 0 && p.n >= 128) ? 128 : 64;
    {
      int kL = *std::max_element(L->nprim.begin(), L->nprim.end());
      int kS = S ? *std::max_element(S->nprim.begin(), S->nprim.end()) : 0;
      char key[256];
      std::snprintf(key, sizeof key,
                    "v1 ham=%d prec=%d fl=%d n=%d NL=%d NS=%d kL=%d kS=%d tau=%.3e tC=%d "
                    "tG=%d cu=%d%s",
                    (int)desc->ham, (int)desc->prec, (int)desc->flags, p.n, p.NL, p.NS, kL, kS,
                    desc->tau,
                    p.C.ntiles, p.gaunt ? p.G.ntiles : 0, p.n_cu, p.cart ? " p=1" : "");
      p.tune_key = key;
    }
    size_plan(p, 0, 0);
    trace.mark("size_plan");
    p.boys.upload(ctx, boys_table());
    if (p.gauge) p.boys3.upload(ctx, boys_table3());
    if (p.cart) p.boysc.upload(ctx, boys_table_cart());
    // general tiles: Coulomb tiles of d / f bases, gauge tiles of Cartesian bases
    if (p.gen || (p.cart && p.gauge)) p.boysg.upload(ctx, boys_table_cart<BOYS_LDG>());
    trace.mark("tables");
    HIPC(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));
    trace.mark("stream");
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
  // wait only for this plan's own work (the last enqueued call on each stream
  // it used, and its side stream); its buffers then go to the allocator's
  // cache without the device-wide wait of hipFree
  bool idle = true;
  for (auto &se : p->stream_events) idle = idle && hipEventSynchronize(se.second) == hipSuccess;
  if (p->side) idle = idle && hipStreamSynchronize(p->side) == hipSuccess;
  if (idle) {
    CacheReleases cache;
    delete p;
  } else {
    (void)hipGetLastError();
    delete p;  // hipFree: waits for the whole device
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  qdcb_ctx::release_ref(ctx);
}

qdcb_status qdcb_plan_estimate(const qdcb_basis *L, const qdcb_basis *S,
                               const qdcb_plan_desc *desc, size_t *bytes) {
  return guarded([&] {
    if (!L || !desc || !bytes) fail(QDCB_E_INVALID, "NULL argument");
    if ((desc->ham == QDCB_HAM_LL) != (S == nullptr))
      fail(QDCB_E_INVALID, "S must be NULL exactly for QDCB_HAM_LL");
    if (desc->n_mo < 1 || desc->n_mo > 512) fail(QDCB_E_INVALID, "n_mo must be in [1, 512]");
    const bool gaunt = desc->ham == QDCB_HAM_DCG || desc->ham == QDCB_HAM_DCB;
    // gauge (or fused Breit) tiles: six per slot, plus the Gaunt tile when mixed
    const double gmul =
        desc->ham == QDCB_HAM_DCB ? (desc->prec == QDCB_PREC_MIXED ? 7.0 : 6.0) : 1.0;
    const double n = desc->n_mo, NL = L->nfunc, NS = S ? S->nfunc : 0;
    const bool spinor = desc->flags & QDCB_PLAN_SPINOR;
    // MO-pair columns: 4 per quaternion pair, 2 per spinor pair (in groups of two)
    const double npair = spinor ? std::ceil(n * (n + 1) / 4) : n * (n + 1) / 2;
    const double ldK = (double)round_up((int64_t)(4 * npair), 128);
    const double PC = (double)round_up(L->npairs + (S ? S->npairs : 0), TILE);
    const double PG = gaunt ? (double)round_up((int64_t)(NL * NS), TILE) : 0.0;
    const double ntC = PC / TILE, ntG = PG / TILE;
    double prims = (double)L->pair_first.back() + (S ? (double)S->pair_first.back() : 0.0);
    if (gaunt) prims += 2.0 * (double)L->first.back() * (double)S->first.back();
    const bool cart = L->has_p() || (S && S->has_p());
    double b = 2.0 * (cart ? 272.0 : 40.0) * prims;       // primitive-pair data (two orders)
    b += 88.0 * (PC + PG);                                // row metadata
    b += (desc->prec == QDCB_PREC_MIXED ? 20.0 : 16.0) *
         (PC * ldK + 3.0 * PG * ldK);                     // D~, V (and FP32 D~), all columns
    b += 22.0 * (ntC * ntC + ntG * ntG);                  // task lists, unique pairs, slot map
    if (desc->prec == QDCB_PREC_MIXED) b += 12.0 * (ntC * ntC + ntG * ntG);  // tier sub-lists
    b += 8.0 * 256 * (std::max(NL, NS) * 4 * n + 4 * n * n);  // second-half slice
    b += 8.0 * 20.0 * (NL + NS) * n * 4;                  // coefficient matrices
    auto slots = [](double nt) { return std::min(nt * nt, std::max(nt, 65536.0)); };
    b += 8.0 * TILE * TILE * (slots(ntC) + (gaunt ? gmul * slots(ntG) : 0.0));  // integral panels
    b += 8.0 * (spinor ? 2.0 : 16.0) * n * n * n * n;     // host-path G staging
    *bytes = (size_t)(b * 1.05);
  });
}

qdcb_status qdcb_plan_footprint(const qdcb_plan *p, size_t *bytes) {
  return guarded([&] {
    if (!p || !bytes) fail(QDCB_E_INVALID, "NULL argument");
    size_t b = p->C.bytes() + p->G.bytes();
    for (auto *x : {&p->CLd, &p->CSd, &p->Gd, &p->CallL, &p->CallS, &p->ChatL, &p->ChatS, &p->boys,
                    &p->boys3, &p->boysc, &p->boysg, &p->W, &p->Gc})
      b += x->bytes();
    for (int K = 0; K < 3; ++K) b += p->AhatK[K].bytes() + p->BhatK[K].bytes();
    b += p->rs.bytes() + p->rowmapL.bytes() + p->rowmapS.bytes() + p->rowmapLS.bytes();
    *bytes = b;
  });
}

}  // extern "C"

extern "C" {
qdcb_status qdcb_plan_fetch(const qdcb_plan *p, int32_t what, void *host_out, size_t bytes) {
  return guarded([&] {
    if (!p || !host_out) fail(QDCB_E_INVALID, "NULL argument");
    PlanUse use(*p);
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

qdcb_status qdcb_plan_fetch_v(const qdcb_plan *p, const int64_t *pairs, int64_t npairs,
                              double *out) {
  return guarded([&] {
    if (!p || !pairs || !out || npairs < 0) fail(QDCB_E_INVALID, "NULL argument");
    if (!p->have_last) fail(QDCB_E_INVALID, "no transform yet");
    PlanUse use(*p);
    DeviceGuard g(p->ctx->device);
    const int64_t c0 = 4LL * p->v_i0, nc = 4LL * (p->v_i1 - p->v_i0);  // resident columns
    const int64_t nLL = p->nLL, nSS = p->nSS, nLS = p->gaunt ? (int64_t)p->NL * p->NS : 0;
    const int64_t wK = 4LL * p->npair_mo, width = (p->gaunt ? 3 : 1) * wK;
    // sorted row of every pair of the concatenated list
    std::vector<int64_t> rowC(nLL + nSS, -1), rowG(nLS, -1);
    for (int64_t r = 0; r < p->C.P; ++r)
      rowC[p->C.h_key[r] + (p->C.h_cls[r] == 1 ? nLL : 0)] = r;
    for (int64_t r = 0; r < p->G.P && p->gaunt; ++r) rowG[p->G.h_key[r]] = r;
    for (int64_t i = 0; i < npairs; ++i) {
      const int64_t k = pairs[i];
      if (k < 0 || k >= nLL + nSS + nLS) fail(QDCB_E_INVALID, "pair index out of range");
      double *o = out + i * width;
      const bool gaunt_row = k >= nLL + nSS;
      const int nK = gaunt_row ? 3 : 1;
      std::fill(o, o + width, 0.0);
      for (int K = 0; K < nK; ++K) {  // columns outside the resident chunk
        std::fill(o + K * wK, o + K * wK + c0, std::nan(""));
        std::fill(o + K * wK + c0 + nc, o + (K + 1) * wK, std::nan(""));
      }
      const Space &sp = gaunt_row ? p->G : p->C;
      const int64_t r = gaunt_row ? rowG[k - nLL - nSS] : rowC[k];
      for (int K = 0; K < nK; ++K)
        HIPC(hipMemcpy(o + K * wK + c0, sp.V.p + r * sp.ld + K * sp.ldK, nc * sizeof(double),
                       hipMemcpyDeviceToHost));
    }
  });
}

}  // extern "C"
