// k_eri.hip -- on-the-fly AO integral tiles for the first half.
//
// For every kept (bra tile, ket tile) a 64 x 64 block of contracted s-type
// ERIs (mn|kl) is generated from the primitive-pair data (Gaussian product
// theorem, Boys F0 in erf form) and stored as panel[slot][ket j][bra m].  Each
// element is masked individually by the directed density-weighted Schwarz
// predicate of Eq. (SchwarzDen): it is computed only when
// (Q_mn * Q_kl) * Dmax_kl >= tau and is 0 otherwise, which is exactly the skip
// of that contribution.
//
// Unique mode: (mn|kl) = (kl|mn), so one computed tile of a unique pair
// (b >= k) fills both directed tiles (b <- k) and (k <- b), each masked by
// its own directed predicate; the transposed one is written column-wise
// (a minor cost next to the primitive-quartet work of each element).
//
// The Boys function comes from a Taylor table staged in LDS (no range branches
// to diverge across lanes; see common.h).
//
// Work layout: 8 wavefronts x 8 ket rows each; lane = bra row.  The primitive
// pairs of the 64 bra rows are staged in LDS once per workgroup when no row has
// more than ERI_LDS_ROWPRIMS of them, primitive-major ([t][row]) so that the
// lanes of a wavefront read consecutive words; the ket pair of a wavefront is uniform
// across its lanes, so its primitive data comes through scalar loads.  Stores
// are one 512-byte row of 64 bra values per ket row (coalesced).
#include "kernels.h"

namespace qdcb {

constexpr int ERI_LDS_ROWPRIMS = 22;  // bra primitives per row held in LDS
constexpr int ERI_LDS_PRIMS = ERI_LDS_ROWPRIMS * 64;  // 55 KB of bra primitive data
constexpr int ERI_WAVES = 8;         // wavefronts per tile, TILE / ERI_WAVES ket rows each
constexpr int ERI_THREADS = 64 * ERI_WAVES;

// out: directed tile (bt <- kt) stored [ket j][bra lane], or NULL; outT (unique
// mode): directed tile (kt <- bt), whose ket rows are bt's, stored [lane][j], or NULL.
template <bool LDS>
__device__ __forceinline__ void eri_tile_body(const EriTileArgs &a, const double *sip,
                                              const double *sx, const double *sy,
                                              const double *sz, const double *se,
                                              const double *tab, int kt, int bt,
                                              int lane, int w, double *out, double *outT,
                                              long long kept[4]) {
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  // this lane's bra primitives: LDS [t][lane] (t < count), or global [first + t]
  const int64_t bfirst = a.row_first[brow];
  const int bcount = (int)(a.row_first[brow + 1] - bfirst);
  const int64_t bbase = LDS ? lane : bfirst;
  const int64_t bstride = LDS ? TILE : 1;
  const double *bip = LDS ? sip : a.pp.ip;
  const double *bx = LDS ? sx : a.pp.x;
  const double *by = LDS ? sy : a.pp.y;
  const double *bz = LDS ? sz : a.pp.z;
  const double *be = LDS ? se : a.pp.e;
  // the ket row data of the next row and the ket primitive data of the next
  // primitive are read one iteration ahead (their loads overlap the quartets)
  int64_t krow = (int64_t)kt * TILE + w;
  double nqk = a.Q[krow], ndk = a.Dmax[krow];
  int nck = a.cls[krow];
  int64_t nkf0 = a.row_first[krow], nkf1 = a.row_first[krow + 1];
  for (int i = 0; i < TILE / ERI_WAVES; ++i) {
    const int j = w + ERI_WAVES * i;
    const double qk = nqk, dk = ndk;
    const int ck = nck;
    const int64_t kf0 = nkf0, kf1 = nkf1;
    if (i + 1 < TILE / ERI_WAVES) {
      krow += ERI_WAVES;
      nqk = a.Q[krow];
      ndk = a.Dmax[krow];
      nck = a.cls[krow];
      nkf0 = a.row_first[krow];
      nkf1 = a.row_first[krow + 1];
    }
    double v = 0.0;
    const bool keep_bk = out && (qb * qk) * dk >= a.tau;    // (bra row <- ket row)
    const bool keep_kb = outT && (qk * qb) * db >= a.tau;   // (ket row <- bra row)
    if (keep_bk || keep_kb) {
      double pip = 0.0, px = 0.0, py = 0.0, pz = 0.0, pe = 0.0;
      if (kf0 < kf1) {
        pip = a.pp.ip[kf0];
        px = a.pp.x[kf0];
        py = a.pp.y[kf0];
        pz = a.pp.z[kf0];
        pe = a.pp.e[kf0];
      }
      for (int64_t k = kf0; k < kf1; ++k) {
        const double iq = pip, qx = px, qy = py, qz = pz, ek = pe;
        if (k + 1 < kf1) {
          pip = a.pp.ip[k + 1];
          px = a.pp.x[k + 1];
          py = a.pp.y[k + 1];
          pz = a.pp.z[k + 1];
          pe = a.pp.e[k + 1];
        }
        double s = 0.0;
        for (int t = 0; t < bcount; ++t) {
          const int64_t b = bbase + t * bstride;
          s += be[b] * coulomb_kernel_tab<BOYS_LD>(tab, bip[b], bx[b], by[b], bz[b], iq, qx, qy, qz);
        }
        v += ek * s;
      }
      if (cb >= 0 && ck >= 0) {
        if (keep_bk) kept[cb * 2 + ck] += 1;
        if (keep_kb) kept[ck * 2 + cb] += 1;
      }
    }
    if (out) out[j * TILE + lane] = keep_bk ? v : 0.0;
    // transposed tile: its bra rows are kt's rows (j), its ket rows bt's (lane)
    if (outT) outT[lane * TILE + j] = keep_kb ? v : 0.0;
  }
}

__global__ void __launch_bounds__(ERI_THREADS) k_eri_tiles(EriTileArgs a) {
  __shared__ double sip[ERI_LDS_PRIMS], sx[ERI_LDS_PRIMS], sy[ERI_LDS_PRIMS],
      sz[ERI_LDS_PRIMS], se[ERI_LDS_PRIMS];
  __shared__ __attribute__((aligned(16))) double tab[BOYS_N * BOYS_LD];
  __shared__ int s_maxcnt;
  if (a.overflow && *a.overflow) return;  // uniform: the panel cannot hold the tiles
  if (a.d_total && (int64_t)blockIdx.x >= min(*a.d_total, a.cap)) return;  // uniform exit
  const int64_t slot = a.slot0 + blockIdx.x;
  const int kt = a.tasks[slot];
  const int bt = a.task_bra[slot];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *out, *outT = nullptr;
  if (a.uslot_bk) {
    const int32_t s1 = a.uslot_bk[slot], s2 = a.uslot_kb[slot];
    out = s1 >= 0 ? a.panel + (int64_t)s1 * TILE * TILE : nullptr;
    outT = s2 >= 0 ? a.panel + (int64_t)s2 * TILE * TILE : nullptr;
  } else {
    out = a.panel + (int64_t)blockIdx.x * TILE * TILE;
  }
  long long kept[4] = {0, 0, 0, 0};
  for (int t = threadIdx.x; t < BOYS_N * 8; t += ERI_THREADS)
    tab[(t >> 3) * BOYS_LD + (t & 7)] = a.boys[t];
  // largest primitive count of the tile's bra rows
  if (threadIdx.x < 64) {
    const int64_t r = (int64_t)bt * TILE + threadIdx.x;
    int c = (int)(a.row_first[r + 1] - a.row_first[r]);
    for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
    if (threadIdx.x == 0) s_maxcnt = c;
  }
  __syncthreads();
  if (s_maxcnt <= ERI_LDS_ROWPRIMS) {
    // primitive t of bra row m at [t][m]: a wavefront's reads of one t are
    // consecutive doubles (no bank conflicts)
    for (int e = threadIdx.x; e < s_maxcnt * TILE; e += ERI_THREADS) {
      const int t = e / TILE, m = e % TILE;
      const int64_t r = (int64_t)bt * TILE + m;
      const int64_t f = a.row_first[r];
      if (f + t < a.row_first[r + 1]) {
        sip[e] = a.pp.ip[f + t];
        sx[e] = a.pp.x[f + t];
        sy[e] = a.pp.y[f + t];
        sz[e] = a.pp.z[f + t];
        se[e] = a.pp.e[f + t];
      }
    }
    __syncthreads();
    eri_tile_body<true>(a, sip, sx, sy, sz, se, tab, kt, bt, lane, w, out, outT, kept);
  } else {
    __syncthreads();
    eri_tile_body<false>(a, nullptr, nullptr, nullptr, nullptr, nullptr, tab, kt, bt, lane,
                         w, out, outT, kept);
  }
  if (a.kept) {
    for (int c = 0; c < 4; ++c) {
      long long t = wave_sum_ll(kept[c]);
      if (lane == 0 && t) atomicAdd(a.kept + c, (unsigned long long)t);
    }
  }
}

void launch_eri_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_eri_tiles, dim3((unsigned)nslots), dim3(ERI_THREADS), 0, s, a);
}

}  // namespace qdcb
