// runtime.hip -- host runtime behind the C ABI in include/qdcb.h.
//
// Objects: context (device + memory budget), basis (device primitive-pair
// data and Schwarz factors of its own pairs), plan (pairs of the
// Hamiltonian's classes ordered by decreasing Schwarz factor, per-transform
// buffers).  A transform runs the paper's four stages (Sec. 3.3.1): quaternion
// densities, screening, integral tiles + first half, second half.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qdcb.h"
#include "kernels.h"

using namespace qdcb;

namespace {

thread_local std::string g_err;

struct Fail {
  qdcb_status st;
  std::string msg;
};

[[noreturn]] void fail(qdcb_status st, const std::string &m) { throw Fail{st, m}; }

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(QDCB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPC(x) hip_check((x), #x)

template <class F>
qdcb_status guarded(F &&f) {
  try {
    f();
    g_err.clear();
    return QDCB_OK;
  } catch (const Fail &e) {
    g_err = e.msg;
    return e.st;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return QDCB_E_NOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return QDCB_E_DEVICE;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    HIPC(hipGetDevice(&prev));
    if (prev != dev) HIPC(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct qdcb_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;

  void *alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (used + bytes > budget)
      fail(QDCB_E_NOMEM, "device memory budget exceeded (" + std::to_string(used + bytes) +
                             " > " + std::to_string(budget) + " bytes)");
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) fail(QDCB_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    used += bytes;
    return p;
  }
  void release(void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    used -= bytes;
  }
};

// Device buffer owned by a context.
template <class T>
struct DBuf {
  qdcb_ctx *ctx = nullptr;
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { free(); }
  void alloc(qdcb_ctx *c, size_t count) {
    free();
    ctx = c;
    n = count;
    p = static_cast<T *>(c->alloc(count * sizeof(T)));
  }
  void upload(qdcb_ctx *c, const std::vector<T> &v) {
    alloc(c, v.size());
    if (!v.empty()) HIPC(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  void free() {
    if (ctx && p) ctx->release(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

struct PairStore {
  DBuf<double> p, x, y, z, e;
  void alloc(qdcb_ctx *c, size_t n) {
    p.alloc(c, n);
    x.alloc(c, n);
    y.alloc(c, n);
    z.alloc(c, n);
    e.alloc(c, n);
  }
  PrimPairs view() { return PrimPairs{p.p, x.p, y.p, z.p, e.p}; }
  PrimPairsC cview() const { return PrimPairsC(PrimPairs{p.p, x.p, y.p, z.p, e.p}); }
  void free() {
    p.free();
    x.free();
    y.free();
    z.free();
    e.free();
  }
  size_t bytes() const { return p.bytes() * 5; }
};

struct qdcb_basis {
  qdcb_ctx *ctx = nullptr;
  int nfunc = 0;
  std::vector<int32_t> first;      // primitive offsets [nfunc+1]
  std::vector<int64_t> pair_first; // canonical pairs (mu <= nu, nu-major) [npairs+1]
  std::vector<double> Q;           // host copy of the Schwarz factors
  int64_t npairs = 0;
  DBuf<double> cent, exps, coefs, nc;
  DBuf<int32_t> dfirst;
  DBuf<int64_t> dpair_first;
  PairStore pp;
  DBuf<double> dQ;

  static int64_t canon(int mu, int nu) {
    if (mu > nu) std::swap(mu, nu);
    return (int64_t)nu * (nu + 1) / 2 + mu;
  }
  ~qdcb_basis() {
    cent.free();
    exps.free();
    coefs.free();
    nc.free();
    dfirst.free();
    dpair_first.free();
    pp.free();
    dQ.free();
  }
};

struct qdcb_plan {
  qdcb_ctx *ctx = nullptr;
  const qdcb_basis *L = nullptr, *S = nullptr;
  qdcb_plan_desc desc{};
  int n = 0, NL = 0, NS = 0;
  int npair_mo = 0;
  int64_t ncol = 0, ld = 0;
  int64_t P = 0, Ppad = 0;
  int ntiles = 0;
  int64_t nLL = 0, nSS = 0;

  // sorted pair rows
  std::vector<int32_t> h_cls, h_mu, h_nu;
  std::vector<int64_t> h_canon;  // canonical index within its class basis
  DBuf<int32_t> cls, mu, nu, rs, rowmapL, rowmapS;
  DBuf<int64_t> row_first;
  DBuf<double> Q;
  PairStore pp;

  // per-transform buffers
  DBuf<double> D, V, Dmax, Qmax, Bmax;
  DBuf<int32_t> count, tasks, task_bra;
  DBuf<int64_t> slot_base;
  DBuf<double> panel;
  int64_t panel_slots = 0;
  DBuf<unsigned long long> kept;
  DBuf<double> CLd, CSd, Gd;
  DBuf<double> CallL, ChatL, CallS, ChatS;
  DBuf<double> Vfull, W, Gc;
  int chunk = 0;
  bool have_last = false;

  ~qdcb_plan() {
    for (auto *b : {&D, &V, &Dmax, &Qmax, &Bmax, &panel, &CLd, &CSd, &Gd, &CallL, &ChatL,
                    &CallS, &ChatS, &Vfull, &W, &Gc, &Q})
      b->free();
    for (auto *b : {&cls, &mu, &nu, &rs, &rowmapL, &rowmapS, &count, &tasks, &task_bra})
      b->free();
    row_first.free();
    slot_base.free();
    kept.free();
    pp.free();
  }
};

// ---------------------------------------------------------------------------
extern "C" {

int qdcb_abi_version(void) { return QDCB_ABI_VERSION; }

const char *qdcb_last_error(void) { return g_err.c_str(); }

qdcb_status qdcb_ctx_create(int device, size_t budget, qdcb_ctx **out) {
  return guarded([&] {
    if (!out) fail(QDCB_E_INVALID, "out is NULL");
    int ndev = 0;
    HIPC(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(QDCB_E_INVALID, "no such HIP device");
    DeviceGuard g(device);
    size_t fr = 0, tot = 0;
    HIPC(hipMemGetInfo(&fr, &tot));
    auto *c = new qdcb_ctx();
    c->device = device;
    c->budget = budget ? budget : (size_t)(0.9 * (double)tot);
    *out = c;
  });
}

void qdcb_ctx_destroy(qdcb_ctx *ctx) { delete ctx; }

qdcb_status qdcb_basis_create(qdcb_ctx *ctx, int32_t nfunc, const double *centers,
                              const int32_t *nprim, const double *exps, const double *coefs,
                              qdcb_basis **out) {
  return guarded([&] {
    if (!ctx || !out || !centers || !nprim || !exps || !coefs)
      fail(QDCB_E_INVALID, "NULL argument");
    if (nfunc <= 0 || nfunc > 65535) fail(QDCB_E_INVALID, "nfunc must be in [1, 65535]");
    std::vector<int32_t> first(nfunc + 1, 0);
    for (int f = 0; f < nfunc; ++f) {
      if (nprim[f] < 1 || nprim[f] > 64) fail(QDCB_E_INVALID, "nprim must be in [1, 64]");
      first[f + 1] = first[f] + nprim[f];
    }
    for (int f = 0; f < 3 * nfunc; ++f)
      if (!std::isfinite(centers[f])) fail(QDCB_E_INVALID, "non-finite center");
    for (int i = 0; i < first[nfunc]; ++i) {
      if (!std::isfinite(exps[i]) || !(exps[i] > 0)) fail(QDCB_E_INVALID, "exponent <= 0");
      if (!std::isfinite(coefs[i])) fail(QDCB_E_INVALID, "non-finite coefficient");
    }
    DeviceGuard g(ctx->device);
    std::unique_ptr<qdcb_basis> b(new qdcb_basis());
    b->ctx = ctx;
    b->nfunc = nfunc;
    b->first = first;
    int np = first[nfunc];
    b->cent.upload(ctx, std::vector<double>(centers, centers + 3 * nfunc));
    b->exps.upload(ctx, std::vector<double>(exps, exps + np));
    b->coefs.upload(ctx, std::vector<double>(coefs, coefs + np));
    b->dfirst.upload(ctx, first);
    b->nc.alloc(ctx, np);
    launch_norm_coefs(nfunc, b->dfirst.p, b->exps.p, b->coefs.p, b->nc.p, nullptr);
    HIPC(hipGetLastError());
    // canonical pairs mu <= nu, index nu(nu+1)/2 + mu
    int64_t npairs = (int64_t)nfunc * (nfunc + 1) / 2;
    b->npairs = npairs;
    std::vector<int32_t> pm(npairs), pn(npairs);
    std::vector<int64_t> pf(npairs + 1, 0);
    for (int nu = 0; nu < nfunc; ++nu)
      for (int mu = 0; mu <= nu; ++mu) {
        int64_t i = qdcb_basis::canon(mu, nu);
        pm[i] = mu;
        pn[i] = nu;
      }
    for (int64_t i = 0; i < npairs; ++i)
      pf[i + 1] = pf[i] + (int64_t)nprim[pm[i]] * nprim[pn[i]];
    b->pair_first = pf;
    DBuf<int32_t> dm, dn;
    dm.upload(ctx, pm);
    dn.upload(ctx, pn);
    b->dpair_first.upload(ctx, pf);
    b->pp.alloc(ctx, (size_t)pf[npairs]);
    launch_pair_data(npairs, dm.p, dn.p, b->dpair_first.p, b->cent.p, b->dfirst.p, b->exps.p,
                     b->nc.p, b->cent.p, b->dfirst.p, b->exps.p, b->nc.p, b->pp.view(), nullptr);
    HIPC(hipGetLastError());
    b->dQ.alloc(ctx, npairs);
    launch_schwarz(npairs, b->dpair_first.p, b->pp.cview(), b->dQ.p, nullptr);
    HIPC(hipGetLastError());
    b->Q.resize(npairs);
    HIPC(hipMemcpy(b->Q.data(), b->dQ.p, npairs * sizeof(double), hipMemcpyDeviceToHost));
    dm.free();
    dn.free();
    *out = b.release();
  });
}

void qdcb_basis_destroy(qdcb_basis *b) {
  if (!b) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->ctx->device);
  delete b;
  if (prev >= 0) (void)hipSetDevice(prev);
}

qdcb_status qdcb_basis_schwarz(const qdcb_basis *b, double *Q) {
  return guarded([&] {
    if (!b || !Q) fail(QDCB_E_INVALID, "NULL argument");
    int N = b->nfunc;
    for (int mu = 0; mu < N; ++mu)
      for (int nu = 0; nu < N; ++nu) Q[(int64_t)mu * N + nu] = b->Q[qdcb_basis::canon(mu, nu)];
  });
}

qdcb_status qdcb_eri_quartets(const qdcb_basis *A, const qdcb_basis *B, int64_t nq,
                              const int32_t *idx, double *out) {
  return guarded([&] {
    if (!A || !B || (nq > 0 && (!idx || !out))) fail(QDCB_E_INVALID, "NULL argument");
    if (A->ctx != B->ctx) fail(QDCB_E_INVALID, "bases belong to different contexts");
    if (nq <= 0) return;
    std::vector<int64_t> af(nq), bf(nq);
    std::vector<int32_t> ac(nq), bc(nq);
    for (int64_t q = 0; q < nq; ++q) {
      const int32_t *i4 = idx + 4 * q;
      if (i4[0] < 0 || i4[1] < 0 || i4[0] >= A->nfunc || i4[1] >= A->nfunc || i4[2] < 0 ||
          i4[3] < 0 || i4[2] >= B->nfunc || i4[3] >= B->nfunc)
        fail(QDCB_E_INVALID, "quartet index out of range");
      int64_t pa = qdcb_basis::canon(i4[0], i4[1]), pb = qdcb_basis::canon(i4[2], i4[3]);
      af[q] = A->pair_first[pa];
      ac[q] = (int32_t)(A->pair_first[pa + 1] - af[q]);
      bf[q] = B->pair_first[pb];
      bc[q] = (int32_t)(B->pair_first[pb + 1] - bf[q]);
    }
    qdcb_ctx *ctx = A->ctx;
    DeviceGuard g(ctx->device);
    DBuf<int64_t> daf, dbf;
    DBuf<int32_t> dac, dbc;
    DBuf<double> dout;
    daf.upload(ctx, af);
    dbf.upload(ctx, bf);
    dac.upload(ctx, ac);
    dbc.upload(ctx, bc);
    dout.alloc(ctx, nq);
    launch_eri_list(nq, daf.p, dbf.p, dac.p, dbc.p, A->pp.cview(), B->pp.cview(), dout.p, nullptr);
    HIPC(hipGetLastError());
    HIPC(hipMemcpy(out, dout.p, nq * sizeof(double), hipMemcpyDeviceToHost));
    daf.free();
    dbf.free();
    dac.free();
    dbc.free();
    dout.free();
  });
}

qdcb_status qdcb_plan_create(qdcb_ctx *ctx, const qdcb_basis *L, const qdcb_basis *S,
                             const qdcb_plan_desc *desc, qdcb_plan **out) {
  return guarded([&] {
    if (!ctx || !L || !desc || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (desc->ham != QDCB_HAM_LL && desc->ham != QDCB_HAM_DC && desc->ham != QDCB_HAM_DCG)
      fail(QDCB_E_INVALID, "unknown Hamiltonian");
    if (desc->ham == QDCB_HAM_DCG)
      fail(QDCB_E_UNSUPPORTED, "the Gaunt classes are not available in this build");
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
    p.L = L;
    p.S = S;
    p.desc = *desc;
    p.n = desc->n_mo;
    p.NL = L->nfunc;
    p.NS = S ? S->nfunc : 0;
    p.nLL = L->npairs;
    p.nSS = S ? S->npairs : 0;
    p.P = p.nLL + p.nSS;
    p.Ppad = (p.P + TILE - 1) / TILE * TILE;
    if (p.Ppad / TILE > (1 << 30)) fail(QDCB_E_INVALID, "too many pairs");
    p.ntiles = (int)(p.Ppad / TILE);
    p.npair_mo = p.n * (p.n + 1) / 2;
    p.ncol = 4LL * p.npair_mo;
    p.ld = (p.ncol + 127) / 128 * 128;

    // rows ordered by decreasing Schwarz factor (ties: class, canonical index)
    std::vector<int64_t> order(p.P);
    std::iota(order.begin(), order.end(), 0);
    auto qof = [&](int64_t i) { return i < p.nLL ? L->Q[i] : S->Q[i - p.nLL]; };
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return qof(a) > qof(b); });
    p.h_cls.assign(p.Ppad, -1);
    p.h_mu.assign(p.Ppad, 0);
    p.h_nu.assign(p.Ppad, 0);
    p.h_canon.assign(p.Ppad, -1);
    std::vector<double> hQ(p.Ppad, 0.0);
    std::vector<int64_t> rf(p.Ppad + 1, 0);
    std::vector<int32_t> rowmapL((size_t)p.NL * p.NL), rowmapS((size_t)p.NS * p.NS);
    // source rows for the gather, per class
    std::vector<int64_t> srcL, dstL, srcS, dstS;
    std::vector<int32_t> cntL, cntS;
    for (int64_t r = 0; r < p.P; ++r) {
      int64_t i = order[r];
      const qdcb_basis *B = i < p.nLL ? L : S;
      int64_t ci = i < p.nLL ? i : i - p.nLL;
      int cls = i < p.nLL ? 0 : 1;
      int nu = (int)std::floor((std::sqrt(8.0 * (double)ci + 1.0) - 1.0) / 2.0);
      while ((int64_t)nu * (nu + 1) / 2 > ci) --nu;
      while ((int64_t)(nu + 1) * (nu + 2) / 2 <= ci) ++nu;
      int mu = (int)(ci - (int64_t)nu * (nu + 1) / 2);
      p.h_cls[r] = cls;
      p.h_mu[r] = mu;
      p.h_nu[r] = nu;
      p.h_canon[r] = ci;
      hQ[r] = B->Q[ci];
      int64_t cnt = B->pair_first[ci + 1] - B->pair_first[ci];
      rf[r + 1] = rf[r] + cnt;
      if (cls == 0) {
        srcL.push_back(B->pair_first[ci]);
        dstL.push_back(rf[r]);
        cntL.push_back((int32_t)cnt);
        rowmapL[(size_t)mu * p.NL + nu] = rowmapL[(size_t)nu * p.NL + mu] = (int32_t)r;
      } else {
        srcS.push_back(B->pair_first[ci]);
        dstS.push_back(rf[r]);
        cntS.push_back((int32_t)cnt);
        rowmapS[(size_t)mu * p.NS + nu] = rowmapS[(size_t)nu * p.NS + mu] = (int32_t)r;
      }
    }
    for (int64_t r = p.P; r < p.Ppad; ++r) rf[r + 1] = rf[r];
    p.cls.upload(ctx, p.h_cls);
    p.mu.upload(ctx, p.h_mu);
    p.nu.upload(ctx, p.h_nu);
    p.Q.upload(ctx, hQ);
    p.row_first.upload(ctx, rf);
    p.rowmapL.upload(ctx, rowmapL);
    if (p.NS) p.rowmapS.upload(ctx, rowmapS);
    p.pp.alloc(ctx, (size_t)std::max<int64_t>(rf[p.Ppad], 1));
    for (int c = 0; c < 2; ++c) {
      auto &src = c ? srcS : srcL;
      auto &dst = c ? dstS : dstL;
      auto &cnt = c ? cntS : cntL;
      if (src.empty()) continue;
      DBuf<int64_t> ds, dd;
      DBuf<int32_t> dc;
      ds.upload(ctx, src);
      dd.upload(ctx, dst);
      dc.upload(ctx, cnt);
      launch_gather_pairs((int64_t)src.size(), ds.p, dc.p, dd.p, (c ? S : L)->pp.cview(),
                          p.pp.view(), nullptr);
      HIPC(hipGetLastError());
      HIPC(hipDeviceSynchronize());
      ds.free();
      dd.free();
      dc.free();
    }
    // MO pair table r <= s
    std::vector<int32_t> rs(p.npair_mo);
    {
      int k = 0;
      for (int r = 0; r < p.n; ++r)
        for (int s = r; s < p.n; ++s) rs[k++] = r | (s << 16);
    }
    p.rs.upload(ctx, rs);

    // per-transform buffers
    p.D.alloc(ctx, (size_t)p.Ppad * p.ld);
    HIPC(hipMemset(p.D.p, 0, p.D.bytes()));
    p.V.alloc(ctx, (size_t)p.Ppad * p.ld);
    p.Dmax.alloc(ctx, p.Ppad);
    p.Qmax.alloc(ctx, p.ntiles);
    p.Bmax.alloc(ctx, p.ntiles);
    p.count.alloc(ctx, p.ntiles);
    p.slot_base.alloc(ctx, p.ntiles);
    p.kept.alloc(ctx, 4);
    p.CLd.alloc(ctx, (size_t)4 * p.NL * p.n);
    if (p.NS) p.CSd.alloc(ctx, (size_t)4 * p.NS * p.n);
    p.CallL.alloc(ctx, (size_t)p.NL * 4 * p.n);
    p.ChatL.alloc(ctx, (size_t)4 * p.NL * 4 * p.n);
    if (p.NS) {
      p.CallS.alloc(ctx, (size_t)p.NS * 4 * p.n);
      p.ChatS.alloc(ctx, (size_t)4 * p.NS * 4 * p.n);
    }
    // second-half column chunk: dense V, W and G slices within ~1/8 of the free budget
    int Nmax = std::max(p.NL, p.NS);
    size_t per_col = sizeof(double) * ((size_t)Nmax * Nmax + (size_t)Nmax * 4 * p.n +
                                       (size_t)4 * p.n * p.n);
    size_t room = (ctx->budget - ctx->used) / 8;
    int64_t chunk = (int64_t)(room / per_col) / 64 * 64;
    chunk = std::min<int64_t>(chunk, (p.ncol + 63) / 64 * 64);
    chunk = std::min<int64_t>(chunk, 65535 * 64);
    if (chunk < 64) fail(QDCB_E_NOMEM, "no room for a 64-column second-half slice");
    p.chunk = (int)chunk;
    p.Vfull.alloc(ctx, (size_t)chunk * Nmax * Nmax);
    p.W.alloc(ctx, (size_t)chunk * Nmax * 4 * p.n);
    p.Gc.alloc(ctx, (size_t)chunk * 4 * p.n * p.n);
    // integral panel: a quarter of what is left, at least one full bra row of tiles
    size_t slot_bytes = sizeof(double) * TILE * TILE;
    int64_t slots = (int64_t)((ctx->budget - ctx->used) / 4 / slot_bytes);
    slots = std::min<int64_t>(slots, (int64_t)1 << 22);
    if (slots < p.ntiles) fail(QDCB_E_NOMEM, "no room for one bra row of integral tiles");
    p.panel_slots = slots;
    p.panel.alloc(ctx, (size_t)slots * TILE * TILE);
    *out = pl.release();
  });
}

void qdcb_plan_destroy(qdcb_plan *p) {
  if (!p) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(p->ctx->device);
  delete p;
  if (prev >= 0) (void)hipSetDevice(prev);
}

qdcb_status qdcb_plan_footprint(const qdcb_plan *p, size_t *bytes) {
  return guarded([&] {
    if (!p || !bytes) fail(QDCB_E_INVALID, "NULL argument");
    size_t b = 0;
    for (auto *x : {&p->D, &p->V, &p->Dmax, &p->Qmax, &p->Bmax, &p->panel, &p->CLd, &p->CSd,
                    &p->Gd, &p->CallL, &p->ChatL, &p->CallS, &p->ChatS, &p->Vfull, &p->W, &p->Gc,
                    &p->Q})
      b += x->bytes();
    for (auto *x : {&p->cls, &p->mu, &p->nu, &p->rs, &p->rowmapL, &p->rowmapS, &p->count,
                    &p->tasks, &p->task_bra})
      b += x->bytes();
    b += p->row_first.bytes() + p->slot_base.bytes() + p->kept.bytes() + p->pp.bytes();
    *bytes = b;
  });
}

namespace {

struct Timer {
  hipEvent_t ev[8];
  int n = 0;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    for (auto &e : ev) HIPC(hipEventCreate(&e));
  }
  ~Timer() {
    for (auto &e : ev) (void)hipEventDestroy(e);
  }
  void mark() { HIPC(hipEventRecord(ev[n++], s)); }
  double ms(int a, int b) {
    float t = 0;
    HIPC(hipEventElapsedTime(&t, ev[a], ev[b]));
    return t;
  }
};

void check_finite_host(const double *x, size_t n, const char *what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) fail(QDCB_E_INVALID, std::string("non-finite value in ") + what);
}

}  // namespace

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
    Timer tm(s);
    tm.mark();  // 0
    DensityArgs da;
    da.nrows = p.Ppad;
    da.n = n;
    da.npair_mo = p.npair_mo;
    da.ld = p.ld;
    da.cls = p.cls.p;
    da.mu = p.mu.p;
    da.nu = p.nu.p;
    da.CL = dCL;
    da.CS = dCS;
    da.NL = p.NL;
    da.NS = p.NS;
    da.rs = p.rs.p;
    da.D = p.D.p;
    da.Dmax = p.Dmax.p;
    launch_density(da, s);
    launch_tile_bounds(p.ntiles, p.Q.p, p.Dmax.p, p.Qmax.p, p.Bmax.p, s);
    HIPC(hipGetLastError());
    tm.mark();  // 1
    launch_screen_count(p.ntiles, p.Qmax.p, p.Bmax.p, p.desc.tau, p.count.p, s);
    HIPC(hipGetLastError());
    std::vector<int32_t> cnt(p.ntiles);
    HIPC(hipMemcpyAsync(cnt.data(), p.count.p, cnt.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<int64_t> base(p.ntiles);
    int64_t total = 0;
    for (int b = 0; b < p.ntiles; ++b) {
      base[b] = total;
      total += cnt[b];
    }
    HIPC(hipMemcpyAsync(p.slot_base.p, base.data(), base.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
    if ((int64_t)p.tasks.n < std::max<int64_t>(total, 1)) {
      HIPC(hipStreamSynchronize(s));
      p.tasks.alloc(ctx, (size_t)std::max<int64_t>(total, 1));
      p.task_bra.alloc(ctx, (size_t)std::max<int64_t>(total, 1));
    }
    launch_screen_fill(0, p.ntiles, p.ntiles, p.Qmax.p, p.Bmax.p, p.desc.tau, p.slot_base.p,
                       p.tasks.p, p.task_bra.p, s);
    HIPC(hipMemsetAsync(p.kept.p, 0, p.kept.bytes(), s));
    HIPC(hipGetLastError());
    tm.mark();  // 2
    // batches of consecutive bra tiles whose integral tiles fit the panel
    int nb = 0;
    double ms_eri = 0, ms_fh = 0;
    hipEvent_t e0, e1, e2;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    HIPC(hipEventCreate(&e2));
    for (int b0 = 0; b0 < p.ntiles;) {
      int b1 = b0;
      int64_t used = 0;
      while (b1 < p.ntiles && used + cnt[b1] <= p.panel_slots) used += cnt[b1++];
      EriTileArgs ea;
      ea.tasks = p.tasks.p;
      ea.task_bra = p.task_bra.p;
      ea.slot0 = base[b0];
      ea.row_first = p.row_first.p;
      ea.pp = p.pp.cview();
      ea.Q = p.Q.p;
      ea.Dmax = p.Dmax.p;
      ea.cls = p.cls.p;
      ea.tau = p.desc.tau;
      ea.panel = p.panel.p;
      ea.kept = p.kept.p;
      HIPC(hipEventRecord(e0, s));
      launch_eri_tiles(ea, used, s);
      HIPC(hipEventRecord(e1, s));
      FirstHalfArgs fa;
      fa.b0 = b0;
      fa.b1 = b1;
      fa.slot_base = p.slot_base.p;
      fa.count = p.count.p;
      fa.tasks = p.tasks.p;
      fa.slot0 = base[b0];
      fa.panel = p.panel.p;
      fa.D = p.D.p;
      fa.V = p.V.p;
      fa.ld = p.ld;
      fa.ncol_tiles = (int)(p.ld / 128);
      launch_first_half(fa, s);
      HIPC(hipGetLastError());
      HIPC(hipEventRecord(e2, s));
      HIPC(hipEventSynchronize(e2));
      float t1 = 0, t2 = 0;
      HIPC(hipEventElapsedTime(&t1, e0, e1));
      HIPC(hipEventElapsedTime(&t2, e1, e2));
      ms_eri += t1;
      ms_fh += t2;
      ++nb;
      b0 = b1;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    tm.mark();  // 3
    // second half: per column slice, both classes accumulate into Gc
    launch_build_coef_mats(p.NL, n, dCL, p.CallL.p, p.ChatL.p, s);
    if (p.NS) launch_build_coef_mats(p.NS, n, dCS, p.CallS.p, p.ChatS.p, s);
    for (int64_t c0 = 0; c0 < p.ncol; c0 += p.chunk) {
      int nc = (int)std::min<int64_t>(p.chunk, p.ncol - c0);
      for (int cls = 0; cls < (p.NS ? 2 : 1); ++cls) {
        int N = cls ? p.NS : p.NL;
        const int32_t *rowmap = cls ? p.rowmapS.p : p.rowmapL.p;
        const double *Call = cls ? p.CallS.p : p.CallL.p;
        const double *Chat = cls ? p.ChatS.p : p.ChatL.p;
        launch_unpack(N, rowmap, p.V.p, p.ld, c0, nc, p.Vfull.p, s);
        launch_dgemm_batched(0, N, 4 * n, N, 1.0, p.Vfull.p, N, (int64_t)N * N, Call, 4 * n, 0,
                             0.0, p.W.p, 4 * n, (int64_t)N * 4 * n, nc, s);
        launch_dgemm_batched(1, 4 * n, n, 4 * N, 1.0, Chat, 4 * n, 0, p.W.p, n,
                             (int64_t)N * 4 * n, cls ? 1.0 : 0.0, p.Gc.p, n,
                             (int64_t)4 * n * n, nc, s);
      }
      launch_pack(n, p.rs.p, c0, nc, p.Gc.p, dG, s);
      HIPC(hipGetLastError());
    }
    tm.mark();  // 4
    if (!dev) HIPC(hipMemcpyAsync(G, dG, nG * sizeof(double), hipMemcpyDeviceToHost, s));
    unsigned long long kept[4];
    HIPC(hipMemcpyAsync(kept, p.kept.p, sizeof(kept), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    p.have_last = true;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->ms_density = tm.ms(0, 1);
      stats->ms_screen = tm.ms(1, 2);
      stats->ms_eri = ms_eri;
      stats->ms_first_half = ms_fh;
      stats->ms_second_half = tm.ms(3, 4);
      stats->ms_total = tm.ms(0, 4);
      double ktot = 0;
      for (int c = 0; c < 4; ++c) {
        stats->kept[c] = (int64_t)kept[c];
        ktot += (double)kept[c];
      }
      stats->total[0] = p.nLL * p.nLL;
      stats->total[1] = p.nLL * p.nSS;
      stats->total[2] = p.nSS * p.nLL;
      stats->total[3] = p.nSS * p.nSS;
      stats->tiles_kept = total;
      stats->tiles_total = (int64_t)p.ntiles * p.ntiles;
      stats->flops_first_half = 2.0 * (double)p.ncol * ktot;
      double f2 = 0;
      for (int cls = 0; cls < (p.NS ? 2 : 1); ++cls) {
        double N = cls ? p.NS : p.NL;
        f2 += (8.0 * N * N * n + 32.0 * N * n * n) * (double)p.ncol;
      }
      stats->flops_second_half = f2;
      stats->flops_mfma = 2.0 * TILE * TILE * (double)p.ld * (double)total;
      stats->n_batches = nb;
    }
  });
}

qdcb_status qdcb_plan_fetch(const qdcb_plan *p, int32_t what, void *host_out, size_t bytes) {
  return guarded([&] {
    if (!p || !host_out) fail(QDCB_E_INVALID, "NULL argument");
    DeviceGuard g(p->ctx->device);
    if (what != QDCB_FETCH_DMAX && what != QDCB_FETCH_Q) fail(QDCB_E_INVALID, "unknown item");
    if (bytes < (size_t)p->P * sizeof(double)) fail(QDCB_E_INVALID, "output too small");
    if (what == QDCB_FETCH_DMAX && !p->have_last) fail(QDCB_E_INVALID, "no transform yet");
    std::vector<double> sorted(p->Ppad);
    HIPC(hipMemcpy(sorted.data(), what == QDCB_FETCH_DMAX ? p->Dmax.p : p->Q.p,
                   p->Ppad * sizeof(double), hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_out);
    for (int64_t r = 0; r < p->P; ++r) {
      int64_t idx = p->h_cls[r] == 0 ? p->h_canon[r] : p->nLL + p->h_canon[r];
      o[idx] = sorted[r];
    }
  });
}

}  // extern "C"
