// noalloc.hip -- entry points that allocate no device memory.
//
// qdcb_eri_quartets_noalloc computes the same contracted integrals as
// qdcb_eri_quartets, whose per-call device buffers (the quartet list, the
// primitive-pair ranges and codes of each quartet, and the output) are taken
// here from one file-scope device array instead of the allocator.  The array
// has a fixed size; its device address is looked up once per device when a
// context is created on that device (the library's init call), and only that
// address is used from host code.
#include <mutex>

#include "runtime.h"

namespace qdcb {

// Per-quartet staging: idx (4 int32), pair ranges (2 int64 + 2 int32), pair
// codes (2 int32), result (1 double) = 56 bytes; each region 256-byte aligned.
constexpr int64_t NOALLOC_MAX_QUARTETS = QDCB_NOALLOC_MAX_QUARTETS;
static_assert(NOALLOC_MAX_QUARTETS == 262144, "documented limit");
constexpr size_t region(size_t bytes) { return (bytes + 255) / 256 * 256; }
constexpr size_t R_IDX = 0;
constexpr size_t R_AF = R_IDX + region(16 * NOALLOC_MAX_QUARTETS);
constexpr size_t R_BF = R_AF + region(8 * NOALLOC_MAX_QUARTETS);
constexpr size_t R_AC = R_BF + region(8 * NOALLOC_MAX_QUARTETS);
constexpr size_t R_BC = R_AC + region(4 * NOALLOC_MAX_QUARTETS);
constexpr size_t R_CODES = R_BC + region(4 * NOALLOC_MAX_QUARTETS);
constexpr size_t R_OUT = R_CODES + region(8 * NOALLOC_MAX_QUARTETS);
constexpr size_t NOALLOC_BYTES = R_OUT + region(8 * NOALLOC_MAX_QUARTETS);

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
unsigned char *g_scratch[MAX_DEVICES] = {};  // device address of scratch, per device
std::mutex g_init_mu;
std::mutex g_call_mu[MAX_DEVICES];  // calls on one device take turns (one array each)
}  // namespace

// Looks up this device's copy of the array (the calling thread's current
// device must be `device`).
void noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) fail(QDCB_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_scratch[device]) return;
  void *ptr = nullptr;
  HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(QDCB_E_DEVICE, "hipGetSymbolAddress returned no address");
  g_scratch[device] = static_cast<unsigned char *>(ptr);
}

// Pair ranges and codes of each quartet from the bases' device-resident
// canonical pair offsets (pair nu (nu + 1) / 2 + mu for mu <= nu) and
// Cartesian codes (NULL: all s).
__global__ void k_quartet_ranges(int64_t nq, const int32_t *idx, const int64_t *pfA,
                                 const int64_t *pfB, const int32_t *cartA,
                                 const int32_t *cartB, int64_t *af, int64_t *bf, int32_t *ac,
                                 int32_t *bc, int32_t *codes) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int i0 = idx[4 * q], i1 = idx[4 * q + 1], i2 = idx[4 * q + 2], i3 = idx[4 * q + 3];
  const int a0 = min(i0, i1), a1 = max(i0, i1), b0 = min(i2, i3), b1 = max(i2, i3);
  const int64_t pa = (int64_t)a1 * (a1 + 1) / 2 + a0, pb = (int64_t)b1 * (b1 + 1) / 2 + b0;
  af[q] = pfA[pa];
  ac[q] = (int32_t)(pfA[pa + 1] - pfA[pa]);
  bf[q] = pfB[pb];
  bc[q] = (int32_t)(pfB[pb + 1] - pfB[pb]);
  if (codes) {
    codes[2 * q] = pair_code(cartA ? cartA[a0] : 0, cartA ? cartA[a1] : 0);
    codes[2 * q + 1] = pair_code(cartB ? cartB[b0] : 0, cartB ? cartB[b1] : 0);
  }
}

}  // namespace qdcb

using namespace qdcb;

extern "C" {

qdcb_status qdcb_eri_quartets_noalloc(const qdcb_basis *A, const qdcb_basis *B, int64_t nq,
                                      const int32_t *idx, double *out) {
  return guarded([&] {
    if (!A || !B || (nq > 0 && (!idx || !out))) fail(QDCB_E_INVALID, "NULL argument");
    if (A->ctx != B->ctx) fail(QDCB_E_INVALID, "bases belong to different contexts");
    if (nq > NOALLOC_MAX_QUARTETS)
      fail(QDCB_E_INVALID, "nq = " + std::to_string(nq) + " exceeds the allocation-free limit of " +
                               std::to_string(NOALLOC_MAX_QUARTETS) + " quartets per call");
    if (nq <= 0) return;
    for (int64_t q = 0; q < nq; ++q) {
      const int32_t *i4 = idx + 4 * q;
      if (i4[0] < 0 || i4[1] < 0 || i4[0] >= A->nfunc || i4[1] >= A->nfunc || i4[2] < 0 ||
          i4[3] < 0 || i4[2] >= B->nfunc || i4[3] >= B->nfunc)
        fail(QDCB_E_INVALID, "quartet index out of range");
    }
    const int dev = A->ctx->device;
    unsigned char *base = (dev >= 0 && dev < MAX_DEVICES) ? g_scratch[dev] : nullptr;
    if (!base) fail(QDCB_E_DEVICE, "no scratch address for this device (no context created on it)");
    std::lock_guard<std::mutex> lk(g_call_mu[dev]);
    DeviceGuard g(dev);
    int32_t *didx = reinterpret_cast<int32_t *>(base + R_IDX);
    int64_t *af = reinterpret_cast<int64_t *>(base + R_AF);
    int64_t *bf = reinterpret_cast<int64_t *>(base + R_BF);
    int32_t *ac = reinterpret_cast<int32_t *>(base + R_AC);
    int32_t *bc = reinterpret_cast<int32_t *>(base + R_BC);
    int32_t *codes = (A->has_p() || B->has_p()) ? reinterpret_cast<int32_t *>(base + R_CODES)
                                                 : nullptr;
    double *dout = reinterpret_cast<double *>(base + R_OUT);
    HIPC(hipMemcpy(didx, idx, (size_t)nq * 4 * sizeof(int32_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_quartet_ranges, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0,
                       nullptr, nq, didx, A->dpair_first.p, B->dpair_first.p,
                       A->has_p() ? A->dcart.p : nullptr, B->has_p() ? B->dcart.p : nullptr, af,
                       bf, ac, bc, codes);
    HIPC(hipGetLastError());
    launch_eri_list(nq, af, bf, ac, bc, codes, A->pp.cview(), B->pp.cview(), dout, nullptr);
    HIPC(hipGetLastError());
    HIPC(hipMemcpy(out, dout, (size_t)nq * sizeof(double), hipMemcpyDeviceToHost));
  });
}

}  // extern "C"
