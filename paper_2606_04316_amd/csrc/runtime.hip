// runtime.hip -- C ABI: context, basis and AO-integral test entry point.
//
// A basis owns the device primitive-pair (Gaussian product) data of all its
// function pairs and their Schwarz factors; both stay resident for the
// basis's lifetime and are shared by every plan built on it.
#include <map>
#include <mutex>
#include <unordered_map>

#include "runtime.h"

using namespace qdcb;

namespace qdcb {
thread_local std::string g_err;
}

namespace qdcb {

namespace {
struct TmpPool {
  std::mutex m;
  std::multimap<size_t, void *> free_blocks;  // rounded size -> block
  size_t cached = 0;
};
constexpr size_t TMP_CACHE_MAX = (size_t)1 << 30;
TmpPool &tmp_pool(int device) {
  static std::mutex m;
  static std::map<int, std::unique_ptr<TmpPool>> pools;
  std::lock_guard<std::mutex> g(m);
  auto &slot = pools[device];
  if (!slot) slot.reset(new TmpPool());
  return *slot;
}
}  // namespace

void *tmp_alloc(int device, size_t bytes, size_t *rounded) {
  size_t r = 4096;
  while (r < bytes) r <<= 1;
  *rounded = r;
  TmpPool &tp = tmp_pool(device);
  {
    std::lock_guard<std::mutex> g(tp.m);
    auto it = tp.free_blocks.find(r);
    if (it != tp.free_blocks.end()) {
      void *p = it->second;
      tp.free_blocks.erase(it);
      tp.cached -= r;
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) fail(QDCB_E_NOMEM, std::string("hipMalloc (set-up scratch): ") +
                                              hipGetErrorString(e));
  return p;
}

void tmp_release(int device, void *p, size_t rounded) {
  if (!p) return;
  TmpPool &tp = tmp_pool(device);
  {
    std::lock_guard<std::mutex> g(tp.m);
    if (tp.cached + rounded <= TMP_CACHE_MAX) {
      tp.free_blocks.emplace(rounded, p);
      tp.cached += rounded;
      return;
    }
  }
  (void)hipFree(p);
}

namespace {
struct DevCache {
  std::mutex m;
  std::multimap<size_t, void *> free_blocks;    // size -> cached block
  std::unordered_map<void *, size_t> size_of;  // every live or cached block
  size_t cached = 0;
  size_t cap = 0;
};
thread_local int t_cache_releases = 0;
DevCache &dev_cache(int device) {
  static std::mutex m;
  static std::map<int, std::unique_ptr<DevCache>> caches;
  std::lock_guard<std::mutex> g(m);
  auto &slot = caches[device];
  if (!slot) {
    slot.reset(new DevCache());
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) slot->cap = tot / 4;
  }
  return *slot;
}
size_t round_block(size_t bytes) {
  constexpr size_t MB = (size_t)1 << 20;
  if (bytes > MB) {
    // eighths of the power of two below: at most 12.5% more
    size_t top = MB;
    while (top * 2 <= bytes) top <<= 1;
    const size_t step = top / 8;
    return (bytes + step - 1) / step * step;
  }
  size_t r = 256;
  while (r < bytes) r <<= 1;
  return r;
}
}  // namespace

CacheReleases::CacheReleases() { ++t_cache_releases; }
CacheReleases::~CacheReleases() { --t_cache_releases; }

void *dev_alloc(int device, size_t bytes) {
  const size_t r = round_block(bytes);
  DevCache &dc = dev_cache(device);
  {
    std::lock_guard<std::mutex> g(dc.m);
    auto it = dc.free_blocks.lower_bound(r);
    if (it != dc.free_blocks.end() && it->first <= 2 * r) {
      void *p = it->second;
      dc.cached -= it->first;
      dc.free_blocks.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // give the cached blocks back and try once more
    std::vector<void *> blocks;
    {
      std::lock_guard<std::mutex> g(dc.m);
      for (auto &b : dc.free_blocks) {
        blocks.push_back(b.second);
        dc.size_of.erase(b.second);
      }
      dc.free_blocks.clear();
      dc.cached = 0;
    }
    for (void *b : blocks) (void)hipFree(b);
    p = nullptr;
    e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(QDCB_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> g(dc.m);
  dc.size_of[p] = r;
  return p;
}

void dev_release(int device, void *p) {
  if (!p) return;
  DevCache &dc = dev_cache(device);
  {
    std::lock_guard<std::mutex> g(dc.m);
    auto it = dc.size_of.find(p);
    const size_t sz = it != dc.size_of.end() ? it->second : 0;
    if (t_cache_releases > 0 && sz && dc.cached + sz <= dc.cap) {
      dc.free_blocks.emplace(sz, p);
      dc.cached += sz;
      return;
    }
    if (it != dc.size_of.end()) dc.size_of.erase(it);
  }
  (void)hipFree(p);
}

size_t dev_cached(int device) {
  DevCache &dc = dev_cache(device);
  std::lock_guard<std::mutex> g(dc.m);
  return dc.cached;
}

}  // namespace qdcb

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
    noalloc_init(device);
    size_t fr = 0, tot = 0;
    HIPC(hipMemGetInfo(&fr, &tot));
    auto *c = new qdcb_ctx();
    c->device = device;
    // blocks held by the allocator's cache are free for this context too
    c->budget = budget ? budget : (size_t)(0.9 * (double)(fr + dev_cached(device)));
    *out = c;
  });
}

void qdcb_ctx_destroy(qdcb_ctx *ctx) { qdcb_ctx::release_ref(ctx); }

qdcb_status qdcb_basis_create(qdcb_ctx *ctx, int32_t nfunc, const double *centers,
                              const int32_t *nprim, const double *exps, const double *coefs,
                              qdcb_basis **out) {
  return qdcb_basis_create_cart(ctx, nfunc, centers, nprim, exps, coefs, nullptr, out);
}

qdcb_status qdcb_basis_create_cart(qdcb_ctx *ctx, int32_t nfunc, const double *centers,
                                   const int32_t *nprim, const double *exps,
                                   const double *coefs, const int32_t *cart,
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
    bool any_p = false;
    for (int f = 0; cart && f < nfunc; ++f) {
      if (cart[f] < 0 || cart[f] > 19) fail(QDCB_E_INVALID, "cart codes must be in [0, 19]");
      any_p = any_p || cart[f] != 0;
    }
    DeviceGuard g(ctx->device);
    std::unique_ptr<qdcb_basis> b(new qdcb_basis());
    b->ctx = ctx;
    b->nfunc = nfunc;
    b->first = first;
    b->nprim.assign(nprim, nprim + nfunc);
    if (any_p) {
      b->cart.assign(cart, cart + nfunc);
      b->dcart.upload(ctx, b->cart);
    }
    int np = first[nfunc];
    b->cent.upload(ctx, std::vector<double>(centers, centers + 3 * nfunc));
    b->exps.upload(ctx, std::vector<double>(exps, exps + np));
    b->coefs.upload(ctx, std::vector<double>(coefs, coefs + np));
    b->dfirst.upload(ctx, first);
    b->nc.alloc(ctx, np);
    launch_norm_coefs(nfunc, b->dfirst.p, b->exps.p, b->coefs.p, b->dcart.p, b->nc.p, nullptr);
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
    DBuf<int32_t> dm(POOLED), dn(POOLED);
    dm.upload(ctx, pm);
    dn.upload(ctx, pn);
    b->dpair_first.upload(ctx, pf);
    b->pp.alloc(ctx, (size_t)pf[npairs], any_p);
    launch_pair_data(npairs, dm.p, dn.p, b->dpair_first.p, b->cent.p, b->dfirst.p, b->exps.p,
                     b->nc.p, b->dcart.p, b->cent.p, b->dfirst.p, b->exps.p, b->nc.p,
                     b->dcart.p, b->pp.view(), nullptr);
    HIPC(hipGetLastError());
    DBuf<int32_t> dcode(POOLED);
    if (any_p) {
      std::vector<int32_t> code(npairs);
      for (int64_t i = 0; i < npairs; ++i) code[i] = pair_code(b->cart[pm[i]], b->cart[pn[i]]);
      dcode.upload(ctx, code);
    }
    b->dQ.alloc(ctx, npairs);
    launch_schwarz(npairs, b->dpair_first.p, b->pp.cview(), dcode.p, b->dQ.p, nullptr);
    HIPC(hipGetLastError());
    b->Q.resize(npairs);
    HIPC(hipMemcpy(b->Q.data(), b->dQ.p, npairs * sizeof(double), hipMemcpyDeviceToHost));
    ctx->retain();
    *out = b.release();
  });
}

void qdcb_basis_destroy(qdcb_basis *b) {
  if (!b) return;
  qdcb_ctx *ctx = b->ctx;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  delete b;
  if (prev >= 0) (void)hipSetDevice(prev);
  qdcb_ctx::release_ref(ctx);
}

qdcb_status qdcb_basis_create_rkb(qdcb_ctx *ctx, const qdcb_basis *L, double *norms,
                                  qdcb_basis **out) {
  return guarded([&] {
    if (!ctx || !L || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (L->ctx->device != ctx->device) fail(QDCB_E_INVALID, "basis on another device");
    if (L->has_p()) fail(QDCB_E_UNSUPPORTED, "gradient bases are built for s functions");
    if (3LL * L->nfunc > 65535) fail(QDCB_E_INVALID, "3 nfunc must be at most 65535");
    DeviceGuard g(L->ctx->device);
    const int N = L->nfunc, np = L->first[N];
    std::vector<double> cent(3 * (size_t)N), a(np), nc(np);
    HIPC(hipMemcpy(cent.data(), L->cent.p, cent.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(a.data(), L->exps.p, np * sizeof(double), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(nc.data(), L->nc.p, np * sizeof(double), hipMemcpyDeviceToHost));
    // d/dr_K chi_mu = sum_i w_i (r_K - A_K) exp(-a_i r^2), w_i = -2 a_i nc_i; as
    // coefficients of normalized p primitives (2a/pi)^{3/4} 2 sqrt(a) (r_K - A_K) ...
    std::vector<double> gc(9 * (size_t)N), ge(3 * (size_t)np), gco(3 * (size_t)np);
    std::vector<int32_t> gn(3 * (size_t)N), gcart(3 * (size_t)N);
    std::vector<double> nrm(3 * (size_t)N);
    size_t o = 0;
    for (int mu = 0; mu < N; ++mu) {
      const int i0 = L->first[mu], i1 = L->first[mu + 1];
      // ||d_K chi_mu||^2 = sum_ij w_i w_j (pi/(a_i+a_j))^{3/2} / (2 (a_i+a_j))
      double n2 = 0.0;
      for (int i = i0; i < i1; ++i)
        for (int j = i0; j < i1; ++j) {
          const double p = a[i] + a[j];
          n2 += 4.0 * a[i] * nc[i] * a[j] * nc[j] * std::pow(PI / p, 1.5) / (2.0 * p);
        }
      for (int K = 0; K < 3; ++K) {
        const int f = 3 * mu + K;
        for (int k = 0; k < 3; ++k) gc[3 * (size_t)f + k] = cent[3 * (size_t)mu + k];
        gn[f] = i1 - i0;
        gcart[f] = K + 1;
        nrm[f] = std::sqrt(n2);
        for (int i = i0; i < i1; ++i, ++o) {
          ge[o] = a[i];
          const double pn = std::pow(2.0 * a[i] / PI, 0.75) * 2.0 * std::sqrt(a[i]);
          gco[o] = -2.0 * a[i] * nc[i] / pn;
        }
      }
    }
    const qdcb_status st = qdcb_basis_create_cart(ctx, 3 * N, gc.data(), gn.data(), ge.data(),
                                                  gco.data(), gcart.data(), out);
    if (st != QDCB_OK) fail(st, g_err);
    if (norms) std::copy(nrm.begin(), nrm.end(), norms);
  });
}

qdcb_status qdcb_rkb_small_planes(int32_t nfunc, int32_t m, const double *PS,
                                  const double *norms, double c, double *out) {
  return guarded([&] {
    if (!PS || !norms || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (nfunc < 1 || m < 1) fail(QDCB_E_INVALID, "nfunc and m must be positive");
    if (!(c > 0) || !std::isfinite(c)) fail(QDCB_E_INVALID, "c must be positive");
    const size_t N = nfunc, M = m, G = 3 * N;
    auto at = [&](int plane, size_t f, size_t a) { return PS[(plane * N + f) * M + a]; };
    const double h = 0.5 / c;  // the factor -i / 2c is applied as h * (-i)
    for (size_t mu = 0; mu < N; ++mu)
      for (size_t a = 0; a < M; ++a) {
        const double ar = at(0, mu, a), ai = at(1, mu, a);  // C^S_{mu alpha}
        const double br = at(2, mu, a), bi = at(3, mu, a);  // C^S_{mu beta}
        // sigma_K (C_alpha, C_beta): x -> (C_b, C_a); y -> (-i C_b, i C_a); z -> (C_a, -C_b)
        const double sr[3][2] = {{br, ar}, {bi, -ai}, {ar, -br}};   // real parts
        const double si[3][2] = {{bi, ai}, {-br, ar}, {ai, -bi}};   // imaginary parts
        for (int K = 0; K < 3; ++K) {
          const double w = h * norms[3 * mu + K];
          for (int u = 0; u < 2; ++u) {
            // (-i)(x + i y) = y - i x
            out[((2 * u) * G + 3 * mu + K) * M + a] = w * si[K][u];
            out[((2 * u + 1) * G + 3 * mu + K) * M + a] = -w * sr[K][u];
          }
        }
      }
  });
}

qdcb_status qdcb_rkb_small_quat(int32_t nfunc, int32_t n, const double *CS, const double *norms,
                                double c, double *out) {
  return guarded([&] {
    if (!CS || !norms || !out) fail(QDCB_E_INVALID, "NULL argument");
    if (nfunc < 1 || n < 1) fail(QDCB_E_INVALID, "nfunc and n must be positive");
    if (!(c > 0) || !std::isfinite(c)) fail(QDCB_E_INVALID, "c must be positive");
    const size_t N = nfunc, M = n, G = 3 * N;
    for (size_t mu = 0; mu < N; ++mu)
      for (size_t p = 0; p < M; ++p) {
        const double q0 = CS[(0 * N + mu) * M + p], q1 = CS[(1 * N + mu) * M + p];
        const double q2 = CS[(2 * N + mu) * M + p], q3 = CS[(3 * N + mu) * M + p];
        // e_K C for e_x = k, e_y = j, e_z = i (sigma_K = -i Q(e_K)), with
        // ki = j, kj = -i, ji = -k, jk = i, ij = k, ik = -j:
        //   k (q0 + q1 i + q2 j + q3 k) = -q3 - q2 i + q1 j + q0 k
        //   j (...)                     = -q2 + q3 i + q0 j - q1 k
        //   i (...)                     = -q1 + q0 i - q3 j + q2 k
        const double e[3][4] = {{-q3, -q2, q1, q0}, {-q2, q3, q0, -q1}, {-q1, q0, -q3, q2}};
        for (int K = 0; K < 3; ++K) {
          const double w = -0.5 / c * norms[3 * mu + K];
          for (int z = 0; z < 4; ++z) out[(z * G + 3 * mu + K) * M + p] = w * e[K][z];
        }
      }
  });
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
    const bool cart = A->has_p() || B->has_p();
    std::vector<int32_t> codes(cart ? 2 * nq : 0);
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
      if (cart) {
        // canonical pair (mu <= nu): first function mu, second nu
        const int a0 = std::min(i4[0], i4[1]), a1 = std::max(i4[0], i4[1]);
        const int b0 = std::min(i4[2], i4[3]), b1 = std::max(i4[2], i4[3]);
        codes[2 * q] = pair_code(A->cart_of(a0), A->cart_of(a1));
        codes[2 * q + 1] = pair_code(B->cart_of(b0), B->cart_of(b1));
      }
    }
    qdcb_ctx *ctx = A->ctx;
    DeviceGuard g(ctx->device);
    DBuf<int64_t> daf(POOLED), dbf(POOLED);
    DBuf<int32_t> dac(POOLED), dbc(POOLED);
    DBuf<double> dout(POOLED);
    daf.upload(ctx, af);
    dbf.upload(ctx, bf);
    dac.upload(ctx, ac);
    dbc.upload(ctx, bc);
    DBuf<int32_t> dcodes(POOLED);
    if (cart) dcodes.upload(ctx, codes);
    dout.alloc(ctx, nq);
    launch_eri_list(nq, daf.p, dbf.p, dac.p, dbc.p, dcodes.p, A->pp.cview(), B->pp.cview(),
                    dout.p, nullptr);
    HIPC(hipGetLastError());
    HIPC(hipMemcpy(out, dout.p, nq * sizeof(double), hipMemcpyDeviceToHost));
  });
}

}  // extern "C"
