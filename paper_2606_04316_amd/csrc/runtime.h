// runtime.h -- host-side objects of the qdcb runtime (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qdcb.h"
#include "kernels.h"

namespace qdcb {

extern thread_local std::string g_err;

struct Fail {
  qdcb_status st;
  std::string msg;
};

[[noreturn]] inline void fail(qdcb_status st, const std::string &m) { throw Fail{st, m}; }

inline void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(QDCB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPC(x) ::qdcb::hip_check((x), #x)

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

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device memory of contexts.  Blocks are rounded up (powers of two to 1 MiB,
// then eighths of a power of two).  dev_release returns a block with hipFree,
// or, while the calling thread is inside a CacheReleases scope, to a
// per-device cache that dev_alloc takes blocks from (the smallest cached
// block of at least the rounded size, if it is at most twice that).  hipFree synchronizes the whole device, so a plan that is
// destroyed while other plans' transforms run would otherwise wait for them
// at every buffer.  A scope may cache only blocks no stream still uses.  The
// cache keeps at most a quarter of the device's memory; it is emptied when
// hipMalloc fails.
void *dev_alloc(int device, size_t bytes);
void dev_release(int device, void *p);
size_t dev_cached(int device);  // bytes held by the cache
struct CacheReleases {
  CacheReleases();
  ~CacheReleases();
  CacheReleases(const CacheReleases &) = delete;
  CacheReleases &operator=(const CacheReleases &) = delete;
};

}  // namespace qdcb

// A context lives until it has been destroyed by its owner and every basis
// and plan created from it has been destroyed (reference count).
struct qdcb_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::atomic<int> refs{1};

  void retain() { refs.fetch_add(1); }
  static void release_ref(qdcb_ctx *c) {
    if (c && c->refs.fetch_sub(1) == 1) delete c;
  }

  void *alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (used + bytes > budget)
      qdcb::fail(QDCB_E_NOMEM, "device memory budget exceeded (" + std::to_string(used + bytes) +
                                   " > " + std::to_string(budget) + " bytes)");
    void *p = qdcb::dev_alloc(device, bytes);
    used += bytes;
    return p;
  }
  void release(void *p, size_t bytes) {
    if (!p) return;
    qdcb::dev_release(device, p);
    used -= bytes;
  }
  size_t room() const { return budget > used ? budget - used : 0; }
};

namespace qdcb {

// Device scratch of set-up work (basis and plan creation, test entries).  A
// freed block goes back to a per-device cache instead of hipFree, whose
// implicit device-wide synchronization would wait for every stream of the
// process, the transforms of other plans included.  Set-up work runs on the
// null stream, so a block is cached only after that stream has drained.
// Blocks are rounded up to a power of two (>= 4 KiB); the cache keeps at most
// 1 GiB per device and frees beyond that.  Not counted in context budgets.
void *tmp_alloc(int device, size_t bytes, size_t *rounded);
void tmp_release(int device, void *p, size_t rounded);

// Looks up the device address of the allocation-free entry points' scratch
// array on `device` (the current device); called when a context is created.
void noalloc_init(int device);

struct Pooled {};
constexpr Pooled POOLED{};

// Device buffer owned by a context (or, pooled, a set-up scratch block).
template <class T>
struct DBuf {
  qdcb_ctx *ctx = nullptr;
  T *p = nullptr;
  size_t n = 0;
  bool pooled = false;
  size_t cap_bytes = 0;  // pooled: the block's rounded size
  DBuf() = default;
  explicit DBuf(Pooled) : pooled(true) {}
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { free(); }
  void alloc(qdcb_ctx *c, size_t count) {
    free();
    ctx = c;
    n = count;
    if (pooled)
      p = count ? static_cast<T *>(tmp_alloc(c->device, count * sizeof(T), &cap_bytes)) : nullptr;
    else
      p = static_cast<T *>(c->alloc(count * sizeof(T)));
  }
  void upload(qdcb_ctx *c, const std::vector<T> &v) {
    alloc(c, v.size());
    if (!v.empty()) HIPC(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  void free() {
    if (ctx && p) {
      if (pooled) {
        (void)hipStreamSynchronize(nullptr);  // set-up kernels that read it are done
        tmp_release(ctx->device, p, cap_bytes);
      } else {
        ctx->release(p, n * sizeof(T));
      }
    }
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

struct PairStore {
  DBuf<double> p, x, y, z, e;
  DBuf<double> pa, pb;                  // Cartesian bases only (see PrimPairs)
  DBuf<double> ax, ay, az, bx, by, bz;  // likewise
  DBuf<double> E;                       // likewise, PAIR_E per primitive pair
  PairStore() = default;
  explicit PairStore(Pooled)
      : p(POOLED), x(POOLED), y(POOLED), z(POOLED), e(POOLED), pa(POOLED), pb(POOLED),
        ax(POOLED), ay(POOLED), az(POOLED), bx(POOLED), by(POOLED), bz(POOLED), E(POOLED) {}
  // cart: pa / pb and the P - A, P - B vectors (bases with p or d functions)
  void alloc(qdcb_ctx *c, size_t n, bool cart = false) {
    p.alloc(c, n);
    x.alloc(c, n);
    y.alloc(c, n);
    z.alloc(c, n);
    e.alloc(c, n);
    for (DBuf<double> *b : {&pa, &pb, &ax, &ay, &az, &bx, &by, &bz}) {
      if (cart)
        b->alloc(c, n);
      else
        b->free();
    }
    if (cart)
      E.alloc(c, n * PAIR_E);
    else
      E.free();
  }
  PrimPairs view() {
    PrimPairs v{p.p, x.p, y.p, z.p, e.p, pa.p, pb.p};
    v.ax = ax.p;
    v.ay = ay.p;
    v.az = az.p;
    v.bx = bx.p;
    v.by = by.p;
    v.bz = bz.p;
    v.E = E.p;
    return v;
  }
  PrimPairsC cview() const { return PrimPairsC(const_cast<PairStore *>(this)->view()); }
  void free() {
    for (DBuf<double> *b : {&p, &x, &y, &z, &e, &pa, &pb, &ax, &ay, &az, &bx, &by, &bz, &E})
      b->free();
  }
  size_t bytes() const {
    return p.bytes() * 5 + pa.bytes() + pb.bytes() +
           (ax.bytes() + ay.bytes() + az.bytes() + bx.bytes() + by.bytes() + bz.bytes()) +
           E.bytes();
  }
};

}  // namespace qdcb

struct qdcb_basis {
  qdcb_ctx *ctx = nullptr;
  int nfunc = 0;
  std::vector<int32_t> first;       // primitive offsets [nfunc+1]
  std::vector<int32_t> nprim;       // [nfunc]
  std::vector<int64_t> pair_first;  // canonical pairs (mu <= nu, nu-major) [npairs+1]
  std::vector<double> Q;            // host copy of the Schwarz factors
  // [nfunc] 0 = s, 1..3 = p_x, p_y, p_z, 4..9 = d_xx, d_yy, d_zz, d_xy, d_xz,
  // d_yz, 10..19 = f_xxx, f_yyy, f_zzz, f_xxy, f_xxz, f_xyy, f_yyz, f_xzz,
  // f_yzz, f_xyz (empty: all s)
  std::vector<int32_t> cart;
  int64_t npairs = 0;
  bool has_p() const { return !cart.empty(); }  // any Cartesian function (p, d or f)
  bool has_gen() const {  // a d or f function (the general integral form)
    for (int32_t c : cart)
      if (c >= 4) return true;
    return false;
  }
  bool has_f() const {
    for (int32_t c : cart)
      if (c >= 10) return true;
    return false;
  }
  int32_t cart_of(int f) const { return cart.empty() ? 0 : cart[f]; }
  qdcb::DBuf<double> cent, exps, coefs, nc;
  qdcb::DBuf<int32_t> dfirst, dcart;
  qdcb::DBuf<int64_t> dpair_first;
  qdcb::PairStore pp;
  qdcb::DBuf<double> dQ;

  static int64_t canon(int mu, int nu) {
    if (mu > nu) std::swap(mu, nu);
    return (int64_t)nu * (nu + 1) / 2 + mu;
  }
};
