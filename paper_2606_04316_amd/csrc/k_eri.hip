// k_eri.hip -- on-the-fly AO integral tiles for the first half.
//
// For every kept (bra tile, ket tile) a 64 x 64 block of contracted s-type
// ERIs (mn|kl) is generated from the primitive-pair data (Gaussian product
// theorem, Boys F0 from a Taylor table) and stored as panel[slot][ket j][bra m].  Each
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
// Work layout: 8 wavefronts x 8 ket rows each; lane = bra row.  The first
// ERI_LDS_ROWPRIMS primitive pairs of each of the 64 bra rows are staged in LDS
// once per tile, primitive-major ([t][row]) so that the lanes of a wavefront
// read consecutive words; deeper rows read the rest from global memory.  The
// ket pair of a wavefront is uniform
// across its lanes, so its primitive data comes through scalar loads.  Stores
// are one 512-byte row of 64 bra values per ket row (coalesced).
//
// Gauge tiles (Eq. gaugeInt): the same loops with six accumulators per element,
// B_KL = ((mn| r_K r_L / r^3 |kl) - delta_KL (mn|kl)) / 2 for (K, L) = xx, xy,
// xz, yy, yz, zz, from F0, F1 and F2 of one Taylor table (see gauge_kernel_tab).
//
// Cartesian tiles (bases with p functions, k_eri_tiles_cart*): the same
// layout and masks; each primitive quartet is evaluated in McMurchie-Davidson
// form (Hermite expansion of each pair, derivatives of the Boys kernel up to
// fourth order, common.h) with F_0 .. F_4 from one Taylor table; bra
// primitives are read from global memory (no LDS staging).  General tiles
// (bases with d or f functions, k_eri_tiles_gen*; gauge tiles of every
// Cartesian basis, k_eri_gauge_tiles_gen*): lane = bra row and the same
// masks, the pairs' Hermite coefficients from the pair data and the Hermite
// integrals factorized by direction (common.h); each kernel instantiated for
// the largest Hermite orders of the plan's bases, and the general Coulomb
// tiles in workgroups of four wavefronts x 16 ket rows.
//
// Schedules: one workgroup per tile in list order (k_eri_tiles), or a
// persistent grid of a few workgroups per compute unit that pull tiles from a
// device queue ordered by decreasing primitive-quartet count
// (k_eri_tiles_queue, longest first, so that tiles of uneven contraction depth
// do not leave a long tail).
#include "kernels.h"

namespace qdcb {

constexpr int ERI_LDS_ROWPRIMS = 22;  // bra primitives per row held in LDS
constexpr int ERI_LDS_PRIMS = ERI_LDS_ROWPRIMS * 64;  // 55 KB of bra primitive data
constexpr int ERI_WAVES = 8;         // wavefronts per tile, TILE / ERI_WAVES ket rows each
constexpr int ERI_THREADS = 64 * ERI_WAVES;

// LDS of an integral workgroup: the first ERI_LDS_ROWPRIMS primitive pairs of
// each bra row, primitive-major ([t][row]), the Boys table, and the largest
// primitive count of the current tile's bra rows
struct EriLds {
  double sip[ERI_LDS_PRIMS], sx[ERI_LDS_PRIMS], sy[ERI_LDS_PRIMS], sz[ERI_LDS_PRIMS],
      se[ERI_LDS_PRIMS];
  __attribute__((aligned(16))) double tab[BOYS_N * BOYS_LD];
  int maxcnt;
};

// out: directed tile (bt <- kt) stored [ket j][bra lane], or NULL; outT (unique
// mode): directed tile (kt <- bt), whose ket rows are bt's, stored [lane][j], or NULL.
__device__ __forceinline__ void eri_tile_body(const EriTileArgs &a, const EriLds &L, int kt,
                                              int bt, int lane, int w, double *out,
                                              double *outT, long long kept[4]) {
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  // this lane's bra primitives: t < nl from LDS [t][lane], the rest (rows of
  // deep contractions) from global memory [first + t]; the sum runs over t in
  // order either way
  const int64_t bfirst = a.row_first[brow];
  const int bcount = (int)(a.row_first[brow + 1] - bfirst);
  const int nl = min(bcount, ERI_LDS_ROWPRIMS);
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
        for (int t = 0; t < nl; ++t) {
          const int b = t * TILE + lane;
          s += L.se[b] * coulomb_kernel_tab<BOYS_LD>(L.tab, L.sip[b], L.sx[b], L.sy[b], L.sz[b],
                                                     iq, qx, qy, qz);
        }
        for (int t = nl; t < bcount; ++t) {
          const int64_t b = bfirst + t;
          s += a.pp.e[b] * coulomb_kernel_tab<BOYS_LD>(L.tab, a.pp.ip[b], a.pp.x[b], a.pp.y[b],
                                                       a.pp.z[b], iq, qx, qy, qz);
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

// The gauge kernel of one primitive quartet without its charge factors: with
// g_m = (2 / sqrt(pi)) sqrt(rho) F_m(T), T = rho R^2, R = P - Q,
//   B_KL = ga delta_KL + gb R_K R_L,  ga = (g1 - g0) / 2,  gb = rho (g1 - g2),
// or with ga = (g1 + g0) / 2 the Breit tiles (Gaunt's (mn|kl) delta_KL added)
// when diag = +1/2 instead of -1/2.
// Near field (T < 36): F0, F1, F2 from one table of F_k(T_i), k = 0 .. 9, by
// their Taylor series F_m(T_i + d) = sum_k F_{m+k}(T_i) (-d)^k / k! (k <= 7,
// nested).  Far field: F0 = (1/2) sqrt(pi / T) (erf = 1) and the upward
// recursion F_{m+1} = ((2m + 1) F_m - exp(-T)) / (2T), exact there.
__device__ __forceinline__ void gauge_kernel_tab(const double *tab, double ip, double px,
                                                 double py, double pz, double iq, double qx,
                                                 double qy, double qz, double diag, double &ga,
                                                 double &gb, double &dx, double &dy, double &dz) {
  const double t = ip + iq;  // 1/rho
  const double sr = rsqrt_pos(t);
  dx = px - qx;
  dy = py - qy;
  dz = pz - qz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double rho = sr * sr;
  const double T = r2 * rho;
  double g0, g1, g2;
  if (T < BOYS_TMAX) {
    const int i = (int)fma(T, 8.0, 0.5);
    const double nd = fma(0.125, (double)i, -T);  // -(T - T_i)
    const double *c = tab + BOYS_LD * i;
    g0 = c[7];
    g1 = c[8];
    g2 = c[9];
#pragma unroll
    for (int k = 7; k >= 1; --k) {
      const double h = nd * (1.0 / k);
      g0 = fma(g0, h, c[k - 1]);
      g1 = fma(g1, h, c[k]);
      g2 = fma(g2, h, c[k + 1]);
    }
    g0 *= sr;
    g1 *= sr;
    g2 *= sr;
  } else {
    g0 = rsqrt(r2);
    const double e = TWO_OVER_SQRTPI * sr * exp(-T);
    const double h = 0.5 / T;
    g1 = (g0 - e) * h;
    g2 = fma(3.0, g1, -e) * h;
  }
  ga = fma(0.5, g1, diag * g0);
  gb = rho * (g1 - g2);
}

// Gauge counterpart of eri_tile_body: six tiles per slot (stride TILE^2).
__device__ __forceinline__ void eri_gauge_tile_body(const EriTileArgs &a, const EriLds &L, int kt,
                                                    int bt, int lane, int w, double *out,
                                                    double *outT, long long kept[4]) {
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  const int64_t bfirst = a.row_first[brow];
  const int bcount = (int)(a.row_first[brow + 1] - bfirst);
  const int nl = min(bcount, ERI_LDS_ROWPRIMS);
  for (int i = 0; i < TILE / ERI_WAVES; ++i) {
    const int j = w + ERI_WAVES * i;
    const int64_t krow = (int64_t)kt * TILE + j;
    const double qk = a.Q[krow], dk = a.Dmax[krow];
    const int ck = a.cls[krow];
    const int64_t kf0 = a.row_first[krow], kf1 = a.row_first[krow + 1];
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool keep_bk = out && (qb * qk) * dk >= a.tau;
    const bool keep_kb = outT && (qk * qb) * db >= a.tau;
    if (keep_bk || keep_kb) {
      for (int64_t k = kf0; k < kf1; ++k) {
        const double iq = a.pp.ip[k], qx = a.pp.x[k], qy = a.pp.y[k], qz = a.pp.z[k];
        const double ek = a.pp.e[k];
        double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        auto add = [&](double eb, double ip, double px, double py, double pz) {
          double ga, gb, dx, dy, dz;
          gauge_kernel_tab(L.tab, ip, px, py, pz, iq, qx, qy, qz, a.gauge_diag, ga, gb, dx, dy,
                           dz);
          const double ea = eb * ga, ebb = eb * gb;
          const double bx = ebb * dx, by = ebb * dy, bz = ebb * dz;
          s[0] += fma(bx, dx, ea);
          s[1] = fma(bx, dy, s[1]);
          s[2] = fma(bx, dz, s[2]);
          s[3] += fma(by, dy, ea);
          s[4] = fma(by, dz, s[4]);
          s[5] += fma(bz, dz, ea);
        };
        for (int t = 0; t < nl; ++t) {
          const int b = t * TILE + lane;
          add(L.se[b], L.sip[b], L.sx[b], L.sy[b], L.sz[b]);
        }
        for (int t = nl; t < bcount; ++t) {
          const int64_t b = bfirst + t;
          add(a.pp.e[b], a.pp.ip[b], a.pp.x[b], a.pp.y[b], a.pp.z[b]);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = fma(ek, s[c], v[c]);
      }
      if (cb >= 0 && ck >= 0) {
        if (keep_bk) kept[cb * 2 + ck] += 1;
        if (keep_kb) kept[ck * 2 + cb] += 1;
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (out) out[c * TILE * TILE + j * TILE + lane] = keep_bk ? v[c] : 0.0;
      if (outT) outT[c * TILE * TILE + lane * TILE + j] = keep_kb ? v[c] : 0.0;
    }
  }
}

template <bool GAUGE>
__device__ __forceinline__ void eri_stage_table(const EriTileArgs &a, EriLds &L) {
  if constexpr (GAUGE) {
    for (int t = threadIdx.x; t < BOYS_N * BOYS_LD; t += ERI_THREADS) L.tab[t] = a.boys3[t];
  } else {
    for (int t = threadIdx.x; t < BOYS_N * 8; t += ERI_THREADS)
      L.tab[(t >> 3) * BOYS_LD + (t & 7)] = a.boys[t];
  }
}

// One tile: task `slot` of the lists, written to its panel slot(s).  Opens
// with a barrier-separated staging phase, so consecutive calls of one
// workgroup may reuse the LDS (the table must have been staged before).
template <bool GAUGE>
__device__ __forceinline__ void eri_one_tile(const EriTileArgs &a, EriLds &L, int64_t slot,
                                             long long kept[4]) {
  constexpr int64_t SLOT = (GAUGE ? 6 : 1) * TILE * TILE;  // doubles per panel slot
  const int kt = a.tasks[slot];
  const int bt = a.task_bra[slot];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *out, *outT = nullptr;
  if (a.uslot_bk) {
    const int32_t s1 = a.uslot_bk[slot], s2 = a.uslot_kb[slot];
    out = s1 >= 0 ? a.panel + (int64_t)s1 * SLOT : nullptr;
    outT = s2 >= 0 ? a.panel + (int64_t)s2 * SLOT : nullptr;
  } else {
    out = a.panel + (slot - a.slot0) * SLOT;
  }
  // largest primitive count of the tile's bra rows
  if (threadIdx.x < 64) {
    const int64_t r = (int64_t)bt * TILE + threadIdx.x;
    int c = (int)(a.row_first[r + 1] - a.row_first[r]);
    for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
    if (threadIdx.x == 0) L.maxcnt = c;
  }
  __syncthreads();
  const int nstage = min(L.maxcnt, ERI_LDS_ROWPRIMS);
  // primitive t of bra row m at [t][m]: a wavefront's reads of one t are
  // consecutive doubles (no bank conflicts)
  for (int e = threadIdx.x; e < nstage * TILE; e += ERI_THREADS) {
    const int t = e / TILE, m = e % TILE;
    const int64_t r = (int64_t)bt * TILE + m;
    const int64_t f = a.row_first[r];
    if (f + t < a.row_first[r + 1]) {
      L.sip[e] = a.pp.ip[f + t];
      L.sx[e] = a.pp.x[f + t];
      L.sy[e] = a.pp.y[f + t];
      L.sz[e] = a.pp.z[f + t];
      L.se[e] = a.pp.e[f + t];
    }
  }
  __syncthreads();
  if constexpr (GAUGE)
    eri_gauge_tile_body(a, L, kt, bt, lane, w, out, outT, kept);
  else
    eri_tile_body(a, L, kt, bt, lane, w, out, outT, kept);
}

__device__ __forceinline__ void eri_count(const EriTileArgs &a, const long long kept[4]) {
  if (!a.kept) return;
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < 4; ++c) {
    long long t = wave_sum_ll(kept[c]);
    if (lane == 0 && t) atomicAdd(a.kept + c, (unsigned long long)t);
  }
}

// One workgroup per tile, in list order.
template <bool GAUGE>
__global__ void __launch_bounds__(ERI_THREADS) k_eri_tiles(EriTileArgs a) {
  __shared__ EriLds L;
  if (a.overflow && *a.overflow) return;  // uniform: the panel cannot hold the tiles
  if (a.d_total && (int64_t)blockIdx.x >= min(*a.d_total, a.cap)) return;  // uniform exit
  long long kept[4] = {0, 0, 0, 0};
  eri_stage_table<GAUGE>(a, L);
  eri_one_tile<GAUGE>(a, L, a.slot0 + blockIdx.x, kept);
  eri_count(a, kept);
}

// Persistent: a fixed grid whose workgroups take tasks order[i] from a queue
// (counter *qctr, zero at launch) until the list is exhausted; every
// workgroup's last fetch returns an index past the end, so all of them exit.
// The Boys table is staged once per workgroup.  Which workgroup computes a
// tile does not change its values.
template <bool GAUGE>
__global__ void __launch_bounds__(ERI_THREADS) k_eri_tiles_queue(EriTileArgs a,
                                                                 const int32_t *order,
                                                                 unsigned long long *qctr,
                                                                 int64_t n_host) {
  __shared__ EriLds L;
  __shared__ int64_t s_next;
  if (a.overflow && *a.overflow) return;  // uniform
  const int64_t n = a.d_total ? min(*a.d_total, a.cap) : n_host;
  long long kept[4] = {0, 0, 0, 0};
  eri_stage_table<GAUGE>(a, L);
  for (;;) {
    __syncthreads();  // the previous tile's LDS reads (and s_next's) are done
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(qctr, 1ull);
    __syncthreads();
    const int64_t i = s_next;
    if (i >= n) break;  // uniform
    eri_one_tile<GAUGE>(a, L, order[i], kept);
  }
  eri_count(a, kept);
}

// ---- Cartesian (s/p) tiles

// Directions of one (bra row, ket row) pair of a Cartesian tile: a, b of the
// bra functions (lane), c, d of the ket functions (wavefront-uniform); an
// absent direction (s function) has a zero Hermite coefficient, so its index
// only needs to be valid (0).  The Kronecker deltas between the directions
// are fixed for the pair, so they are formed once, outside the primitive
// loops.
struct CartDirs {
  int a, b, c;            // ket: c = the direction of a one-p ket (either function)
  int d;                  // second ket direction (two-p kets)
  bool ha, hb;            // bra functions of p type
  double dab, dac, dad, dbc, dbd, dcd;
};

// g_n = (2/sqrt(pi)) sqrt(rho) F_n(T), n < NG: near field from the table
// tab[BOYS_LDC i + k] = (2/sqrt(pi)) F_k(T_i) by the Taylor series
// F_m(T_i + d) = sum_k F_{m+k}(T_i) (-d)^k / k! (k <= 7, nested); far field
// (T >= 36) from 1/R and the upward recursion.
template <int NG, int LD = BOYS_LDC>
__device__ __forceinline__ void boys_g_tab_n(const double *tab, double T, double r2, double sr,
                                             double g[NG]) {
  static_assert(NG + 7 <= LD, "eight Taylor terms per order");
  if (T < BOYS_TMAX) {
    const int i = (int)fma(T, 8.0, 0.5);
    const double nd = fma(0.125, (double)i, -T);
    const double *c = tab + LD * i;
#pragma unroll
    for (int m = 0; m < NG; ++m) g[m] = c[m + 7];
#pragma unroll
    for (int k = 7; k >= 1; --k) {
      const double h = nd * (1.0 / k);
#pragma unroll
      for (int m = 0; m < NG; ++m) g[m] = fma(g[m], h, c[m + k - 1]);
    }
#pragma unroll
    for (int m = 0; m < NG; ++m) g[m] *= sr;
  } else {
    g[0] = rsqrt(r2);
    const double e = TWO_OVER_SQRTPI * sr * exp(-T);
    const double h = 0.5 / T;
#pragma unroll
    for (int m = 0; m + 1 < NG; ++m) g[m + 1] = fma(2.0 * m + 1.0, g[m], -e) * h;
  }
}

__device__ __forceinline__ double sel3(int i, double x, double y, double z) {
  return i == 0 ? x : (i == 1 ? y : z);
}

// Contracted value of one (bra row, ket row) pair of a Cartesian tile.  KT is
// the ket's number of p functions (0, 1, 2); the bra side is branch-free
// (its absent terms have zero coefficients).  With W_u the bra-contracted
// Hermite integral sum_t h_t R_{t+u} for the ket Hermite index u:
//   KT = 0: h0 W_0;  KT = 1: h0 W_0 - h1 W_c;
//   KT = 2: h0 W_0 - h1 W_c - h2 W_d + h3 W_cd  (ket coefficients h).
// Read-only view of pair data in the constant address space: the pair data
// are not written while an integral kernel runs, so wavefront-uniform reads
// through it become scalar loads.
typedef const __attribute__((address_space(4))) double *cdptr;
__device__ __forceinline__ cdptr as_const(const double *p) { return (cdptr)p; }

// Contracted value of one (bra row, ket row) pair of a Cartesian tile.  KT is
// the ket's number of p functions (0, 1, 2); the bra side is branch-free
// (its absent terms have zero coefficients).  With W_u the bra-contracted
// Hermite integral sum_t h_t R_{t+u} for the ket Hermite index u:
//   KT = 0: h0 W_0;  KT = 1: h0 W_0 - h1 W_c;
//   KT = 2: h0 W_0 - h1 W_c - h2 W_d + h3 W_cd  (ket coefficients h).
// Loop order: the lane's bra primitive outside (held in registers), the
// wavefront-uniform ket primitives inside (scalar loads).
template <int KT>
__device__ __forceinline__ double cart_row_pair(const EriTileArgs &A, const double *tab,
                                                int64_t kf0, int64_t kf1, int64_t b0, int64_t b1,
                                                const CartDirs &r, int kcode) {
  constexpr int NG = 3 + KT;  // G_0 .. G_{2 + KT}
  const int kc = code_f(kcode) - 1;
  const cdptr kip = as_const(A.pp.ip), kx = as_const(A.pp.x), ky = as_const(A.pp.y),
              kz = as_const(A.pp.z), ke = as_const(A.pp.e), kpa = as_const(A.pp.pa),
              kpb = as_const(A.pp.pb);
  double v = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    const double ip = A.pp.ip[b], px = A.pp.x[b], py = A.pp.y[b], pz = A.pp.z[b];
    // bra Hermite coefficients (zero for absent functions)
    const double half = 0.5 * ip;
    const double fa = r.ha ? A.pp.pa[b] : 1.0, fb = r.hb ? A.pp.pb[b] : 1.0;
    const double h0 = fma(fa, fb, r.dab * half);
    const double h1 = r.ha ? fb * half : 0.0;
    const double h2 = r.hb ? fa * half : 0.0;
    const double h3 = (r.ha && r.hb) ? half * half : 0.0;
    double s = 0.0;
    for (int64_t k = kf0; k < kf1; ++k) {
      const double iq = kip[k];
      // ket Hermite coefficients
      double k0 = 1.0, k1 = 0.0, k2 = 0.0, k3 = 0.0;
      if constexpr (KT == 1) {
        k0 = kc >= 0 ? kpa[k] : kpb[k];
        k1 = 0.5 * iq;
      } else if constexpr (KT == 2) {
        const double hq = 0.5 * iq, qa = kpa[k], qb = kpb[k];
        k0 = fma(qa, qb, r.dcd * hq);
        k1 = qb * hq;
        k2 = qa * hq;
        k3 = hq * hq;
      }
      const double X0 = px - kx[k], X1 = py - ky[k], X2 = pz - kz[k];
      const double sr = rsqrt_pos(ip + iq);
      const double rho = sr * sr;
      const double r2 = X0 * X0 + X1 * X1 + X2 * X2;
      double g[NG];
      boys_g_tab_n<NG>(tab, r2 * rho, r2, sr, g);
      const double m2r = -2.0 * rho;
      const double G1 = g[1] * m2r, G2 = g[2] * (m2r * m2r);
      const double xa = sel3(r.a, X0, X1, X2), xb = sel3(r.b, X0, X1, X2);
      // W_0 = h0 R_0 + h1 R_a + h2 R_b + h3 R_ab
      const double w0 = h0 * g[0] + (h1 * xa + h2 * xb) * G1 + h3 * fma(xa * xb, G2, r.dab * G1);
      double val = k0 * w0;
      if constexpr (KT >= 1) {
        const double G3 = g[3] * (m2r * m2r * m2r);
        const double xc = sel3(r.c, X0, X1, X2);
        // W_c = h0 R_c + h1 R_ac + h2 R_bc + h3 R_abc
        const double wc = h0 * xc * G1 + h1 * fma(xa * xc, G2, r.dac * G1) +
                          h2 * fma(xb * xc, G2, r.dbc * G1) +
                          h3 * fma(r.dab * xc + r.dac * xb + r.dbc * xa, G2, xa * xb * xc * G3);
        val -= k1 * wc;
        if constexpr (KT == 2) {
          const double G4 = g[4] * ((m2r * m2r) * (m2r * m2r));
          const double xd = sel3(r.d, X0, X1, X2);
          const double wd = h0 * xd * G1 + h1 * fma(xa * xd, G2, r.dad * G1) +
                            h2 * fma(xb * xd, G2, r.dbd * G1) +
                            h3 * fma(r.dab * xd + r.dad * xb + r.dbd * xa, G2, xa * xb * xd * G3);
          // W_cd = h0 R_cd + h1 R_acd + h2 R_bcd + h3 R_abcd
          const double rcd = fma(xc * xd, G2, r.dcd * G1);
          const double racd = fma(r.dac * xd + r.dad * xc + r.dcd * xa, G2, xa * xc * xd * G3);
          const double rbcd = fma(r.dbc * xd + r.dbd * xc + r.dcd * xb, G2, xb * xc * xd * G3);
          const double d2 = r.dab * r.dcd + r.dac * r.dbd + r.dad * r.dbc;
          const double d1 = r.dab * xc * xd + r.dac * xb * xd + r.dad * xb * xc +
                            r.dbc * xa * xd + r.dbd * xa * xc + r.dcd * xa * xb;
          const double rabcd = d2 * G2 + d1 * G3 + (xa * xb) * (xc * xd) * G4;
          const double wcd = h0 * rcd + h1 * racd + h2 * rbcd + h3 * rabcd;
          val = fma(-k2, wd, fma(k3, wcd, val));
        }
      }
      s = fma(ke[k], val, s);
    }
    v = fma(A.pp.e[b], s, v);
  }
  return v;
}

__device__ __forceinline__ void eri_cart_tile_body(const EriTileArgs &a, const double *tab,
                                                   int kt, int bt, int lane, int w, double *out,
                                                   double *outT, long long kept[4]) {
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  const int bcode = a.code[brow];
  const int64_t bfirst = a.row_first[brow];
  const int64_t blast = a.row_first[brow + 1];
  const int ba = code_f(bcode) - 1, bb = code_g(bcode) - 1;
  for (int i = 0; i < TILE / ERI_WAVES; ++i) {
    const int j = w + ERI_WAVES * i;
    const int64_t krow = (int64_t)kt * TILE + j;
    const double qk = a.Q[krow], dk = a.Dmax[krow];
    const int ck = a.cls[krow];
    const int kcode = __builtin_amdgcn_readfirstlane(a.code[krow]);
    const int64_t kf0 = a.row_first[krow], kf1 = a.row_first[krow + 1];
    double v = 0.0;
    const bool keep_bk = out && (qb * qk) * dk >= a.tau;
    const bool keep_kb = outT && (qk * qb) * db >= a.tau;
    if (keep_bk || keep_kb) {
      const int kc = code_f(kcode) - 1, kd = code_g(kcode) - 1;
      const int kt_p = (kc >= 0) + (kd >= 0);
      CartDirs r;
      r.ha = ba >= 0;
      r.hb = bb >= 0;
      r.a = max(ba, 0);
      r.b = max(bb, 0);
      r.c = kc >= 0 ? kc : max(kd, 0);  // one-p kets: their direction
      r.d = max(kd, 0);
      auto del = [](int x, int y) { return (x >= 0 && x == y) ? 1.0 : 0.0; };
      r.dab = del(ba, bb);
      r.dcd = del(kc, kd);
      const int c1 = kt_p == 1 ? r.c : kc;  // the first ket direction
      r.dac = del(ba, c1);
      r.dbc = del(bb, c1);
      r.dad = del(ba, kd);
      r.dbd = del(bb, kd);
      if (kt_p == 0)
        v = cart_row_pair<0>(a, tab, kf0, kf1, bfirst, blast, r, kcode);
      else if (kt_p == 1)
        v = cart_row_pair<1>(a, tab, kf0, kf1, bfirst, blast, r, kcode);
      else
        v = cart_row_pair<2>(a, tab, kf0, kf1, bfirst, blast, r, kcode);
      if (cb >= 0 && ck >= 0) {
        if (keep_bk) kept[cb * 2 + ck] += 1;
        if (keep_kb) kept[ck * 2 + cb] += 1;
      }
    }
    if (out) out[j * TILE + lane] = keep_bk ? v : 0.0;
    if (outT) outT[lane * TILE + j] = keep_kb ? v : 0.0;
  }
}

__device__ __forceinline__ void eri_cart_one_tile(const EriTileArgs &a, const double *tab,
                                                  int64_t slot, long long kept[4]) {
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
    out = a.panel + (slot - a.slot0) * TILE * TILE;
  }
  eri_cart_tile_body(a, tab, kt, bt, lane, w, out, outT, kept);
}

__global__ void __launch_bounds__(ERI_THREADS) k_eri_tiles_cart(EriTileArgs a) {
  __shared__ double tab[BOYS_N * BOYS_LDC];
  if (a.overflow && *a.overflow) return;  // uniform
  if (a.d_total && (int64_t)blockIdx.x >= min(*a.d_total, a.cap)) return;  // uniform
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDC; t += ERI_THREADS) tab[t] = a.boysc[t];
  __syncthreads();
  long long kept[4] = {0, 0, 0, 0};
  eri_cart_one_tile(a, tab, a.slot0 + blockIdx.x, kept);
  eri_count(a, kept);
}

// Persistent variant; same queue protocol as k_eri_tiles_queue.
__global__ void __launch_bounds__(ERI_THREADS) k_eri_tiles_queue_cart(EriTileArgs a,
                                                                      const int32_t *order,
                                                                      unsigned long long *qctr,
                                                                      int64_t n_host) {
  __shared__ double tab[BOYS_N * BOYS_LDC];
  __shared__ int64_t s_next;
  if (a.overflow && *a.overflow) return;  // uniform
  const int64_t n = a.d_total ? min(*a.d_total, a.cap) : n_host;
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDC; t += ERI_THREADS) tab[t] = a.boysc[t];
  long long kept[4] = {0, 0, 0, 0};
  for (;;) {
    __syncthreads();  // table staged; the previous s_next read by every thread
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(qctr, 1ull);
    __syncthreads();
    const int64_t i = s_next;
    if (i >= n) break;  // uniform
    eri_cart_one_tile(a, tab, order[i], kept);
  }
  eri_count(a, kept);
}

// ---- general (s .. f) tiles: bases with d or f functions

// Workgroups of four wavefronts (each 16 ket rows of the tile): the general
// form holds more registers than the s and p kernels, and smaller workgroups
// let three of them share a compute unit when the registers allow it (the
// d-sized kernel; the f-sized one is held to two).
constexpr int GEN_WAVES = 4;
constexpr int GEN_THREADS = 64 * GEN_WAVES;
template <int TMAX>
constexpr int gen_blocks() {  // workgroups per compute unit the registers are sized for
  return TMAX <= 4 ? 3 : 2;
}

// Contracted value of one (bra row, ket row) pair of a general tile (codes
// pair_code(cf, cg)), in the factorized McMurchie-Davidson form of common.h,
// with TB, TK bounding the Hermite orders of the tile's bra pairs and of the
// ket pair.  The pairs' Hermite coefficients come with the pair data (made
// with it, for the pair's codes).  The lane's bra primitive outside (its
// coefficients held in registers), the wavefront-uniform ket primitives
// inside (scalar loads).
template <int TB, int TK>
__device__ __forceinline__ double gen_row_pair(const EriTileArgs &A, const double *tab,
                                               int64_t kf0, int64_t kf1, int64_t b0, int64_t b1,
                                               int bcode, int kcode) {
  constexpr int TS = TB + TK;
  const cdptr kip = as_const(A.pp.ip), kx = as_const(A.pp.x), ky = as_const(A.pp.y),
              kz = as_const(A.pp.z), ke = as_const(A.pp.e), kE = as_const(A.pp.E);
  double v = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    const double ip = A.pp.ip[b], px = A.pp.x[b], py = A.pp.y[b], pz = A.pp.z[b];
    // the pair's Hermite coefficients (pair data, t <= TB)
    double Ebx[TB + 1], Eby[TB + 1], Ebz[TB + 1];
    const double *Eb = A.pp.E + PAIR_E * b;
#pragma unroll
    for (int t = 0; t <= TB; ++t) {
      Ebx[t] = Eb[t];
      Eby[t] = Eb[7 + t];
      Ebz[t] = Eb[14 + t];
    }
    double s = 0.0;
    for (int64_t k = kf0; k < kf1; ++k) {
      const double iq = kip[k];
      const double X0 = px - kx[k], X1 = py - ky[k], X2 = pz - kz[k];
      const double sr = rsqrt_pos(ip + iq);
      const double rho = sr * sr;
      const double r2 = X0 * X0 + X1 * X1 + X2 * X2;
      double G[TS + 1];
      boys_g_tab_n<TS + 1, BOYS_LDG>(tab, r2 * rho, r2, sr, G);
      const double m2r = -2.0 * rho;
      double f = m2r;
#pragma unroll
      for (int n = 1; n <= TS; ++n) {
        G[n] *= f;
        f *= m2r;
      }
      double Ek[TK + 1], Px[TS + 1], Py[TS + 1], Pz[TS + 1];
      const int64_t ko = PAIR_E * k;
#pragma unroll
      for (int t = 0; t <= TK; ++t) Ek[t] = kE[ko + t];
      herm_dir<TB, TK>(Ebx, Ek, X0, Px);
#pragma unroll
      for (int t = 0; t <= TK; ++t) Ek[t] = kE[ko + 7 + t];
      herm_dir<TB, TK>(Eby, Ek, X1, Py);
#pragma unroll
      for (int t = 0; t <= TK; ++t) Ek[t] = kE[ko + 14 + t];
      herm_dir<TB, TK>(Ebz, Ek, X2, Pz);
      s = fma(ke[k], herm_sum<TS>(Px, Py, Pz, G), s);
    }
    v = fma(A.pp.e[b], s, v);
  }
  return v;
}

// TMAX: the largest Hermite order bound of the launch (4 when neither basis
// has an f function: the f-sized forms, and their registers, stay out of the
// kernel)
template <int TB, int TMAX>
__device__ __forceinline__ double gen_row_pair_k(const EriTileArgs &A, const double *tab,
                                                 int64_t kf0, int64_t kf1, int64_t b0,
                                                 int64_t b1, int bcode, int kcode, int tk) {
  if (tk == 2) return gen_row_pair<TB, 2>(A, tab, kf0, kf1, b0, b1, bcode, kcode);
  if (TMAX == 4 || tk == 4) return gen_row_pair<TB, 4>(A, tab, kf0, kf1, b0, b1, bcode, kcode);
  return gen_row_pair<TB, TMAX>(A, tab, kf0, kf1, b0, b1, bcode, kcode);
}

template <int TMAX>
__device__ __forceinline__ void eri_gen_one_tile(const EriTileArgs &a, const double *tab,
                                                 int64_t slot, long long kept[4]) {
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
    out = a.panel + (slot - a.slot0) * TILE * TILE;
  }
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  const int bcode = a.code[brow];
  const int64_t bfirst = a.row_first[brow], blast = a.row_first[brow + 1];
  // the Hermite order bound of the tile's bra pairs (uniform)
  int tb = gen_bucket(bcode);
  for (int o = 32; o > 0; o >>= 1) tb = max(tb, __shfl_xor(tb, o, 64));
  tb = __builtin_amdgcn_readfirstlane(tb);
  for (int i = 0; i < TILE / GEN_WAVES; ++i) {
    const int j = w + GEN_WAVES * i;
    const int64_t krow = (int64_t)kt * TILE + j;
    const double qk = a.Q[krow], dk = a.Dmax[krow];
    const int ck = a.cls[krow];
    const int kcode = __builtin_amdgcn_readfirstlane(a.code[krow]);
    const int64_t kf0 = a.row_first[krow], kf1 = a.row_first[krow + 1];
    double v = 0.0;
    const bool keep_bk = out && (qb * qk) * dk >= a.tau;
    const bool keep_kb = outT && (qk * qb) * db >= a.tau;
    if (keep_bk || keep_kb) {
      const int tk = gen_bucket(kcode);
      if (tb == 2)
        v = gen_row_pair_k<2, TMAX>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, tk);
      else if (TMAX == 4 || tb == 4)
        v = gen_row_pair_k<4, TMAX>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, tk);
      else
        v = gen_row_pair_k<TMAX, TMAX>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, tk);
      if (cb >= 0 && ck >= 0) {
        if (keep_bk) kept[cb * 2 + ck] += 1;
        if (keep_kb) kept[ck * 2 + cb] += 1;
      }
    }
    if (out) out[j * TILE + lane] = keep_bk ? v : 0.0;
    if (outT) outT[lane * TILE + j] = keep_kb ? v : 0.0;
  }
}

template <int TMAX>
__global__ void __launch_bounds__(GEN_THREADS, gen_blocks<TMAX>()) k_eri_tiles_gen(EriTileArgs a) {
  __shared__ double tab[BOYS_N * BOYS_LDG];
  if (a.overflow && *a.overflow) return;  // uniform
  if (a.d_total && (int64_t)blockIdx.x >= min(*a.d_total, a.cap)) return;  // uniform
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDG; t += GEN_THREADS) tab[t] = a.boysg[t];
  __syncthreads();
  long long kept[4] = {0, 0, 0, 0};
  eri_gen_one_tile<TMAX>(a, tab, a.slot0 + blockIdx.x, kept);
  eri_count(a, kept);
}

// Persistent variant; same queue protocol as k_eri_tiles_queue.
template <int TMAX>
__global__ void __launch_bounds__(GEN_THREADS, gen_blocks<TMAX>()) k_eri_tiles_queue_gen(EriTileArgs a,
                                                                     const int32_t *order,
                                                                     unsigned long long *qctr,
                                                                     int64_t n_host) {
  __shared__ double tab[BOYS_N * BOYS_LDG];
  __shared__ int64_t s_next;
  if (a.overflow && *a.overflow) return;  // uniform
  const int64_t n = a.d_total ? min(*a.d_total, a.cap) : n_host;
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDG; t += GEN_THREADS) tab[t] = a.boysg[t];
  long long kept[4] = {0, 0, 0, 0};
  for (;;) {
    __syncthreads();  // table staged; the previous s_next read by every thread
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(qctr, 1ull);
    __syncthreads();
    const int64_t i = s_next;
    if (i >= n) break;  // uniform
    eri_gen_one_tile<TMAX>(a, tab, order[i], kept);
  }
  eri_count(a, kept);
}

// ---- gauge (or Breit) tiles over Cartesian bases (p, d, f): six components
// (xx, xy, xz, yy, yz, zz) of A delta_KL + B X_K X_L in the general form
// (common.h, herm_dir3), T bounding the Hermite orders of the tile's bra
// pairs and of the ket pair.
template <int T>
__device__ __forceinline__ void gauge_gen_row_pair(const EriTileArgs &A, const double *tab,
                                                   int64_t kf0, int64_t kf1, int64_t b0,
                                                   int64_t b1, int bcode, int kcode,
                                                   double v[6]) {
  constexpr int TS = 2 * T;
  const double diag = A.gauge_diag;
  const cdptr kip = as_const(A.pp.ip), kx = as_const(A.pp.x), ky = as_const(A.pp.y),
              kz = as_const(A.pp.z), ke = as_const(A.pp.e), kE = as_const(A.pp.E);
#pragma unroll
  for (int c = 0; c < 6; ++c) v[c] = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    const double ip = A.pp.ip[b], px = A.pp.x[b], py = A.pp.y[b], pz = A.pp.z[b];
    const double eb = A.pp.e[b];
    double Ebx[T + 1], Eby[T + 1], Ebz[T + 1];
    const double *Eb = A.pp.E + PAIR_E * b;
#pragma unroll
    for (int t = 0; t <= T; ++t) {
      Ebx[t] = Eb[t];
      Eby[t] = Eb[7 + t];
      Ebz[t] = Eb[14 + t];
    }
    for (int64_t k = kf0; k < kf1; ++k) {
      const double iq = kip[k];
      const double X0 = px - kx[k], X1 = py - ky[k], X2 = pz - kz[k];
      const double sr = rsqrt_pos(ip + iq);
      const double rho = sr * sr;
      const double r2 = X0 * X0 + X1 * X1 + X2 * X2;
      double g[TS + 3];
      boys_g_tab_n<TS + 3, BOYS_LDG>(tab, r2 * rho, r2, sr, g);
      double DA[TS + 1], DB[TS + 1];
      const double m2r = -2.0 * rho;
      double f = 1.0;
#pragma unroll
      for (int n = 0; n <= TS; ++n) {
        DA[n] = f * fma(0.5, g[n + 1], diag * g[n]);
        DB[n] = f * rho * (g[n + 1] - g[n + 2]);
        f *= m2r;
      }
      double Ek[T + 1];
      double P0x[TS + 1], P1x[TS + 1], P2x[TS + 1];
      double P0y[TS + 1], P1y[TS + 1], P2y[TS + 1];
      double P0z[TS + 1], P1z[TS + 1], P2z[TS + 1];
      const int64_t ko = PAIR_E * k;
#pragma unroll
      for (int t = 0; t <= T; ++t) Ek[t] = kE[ko + t];
      herm_dir3<T, T>(Ebx, Ek, X0, P0x, P1x, P2x);
#pragma unroll
      for (int t = 0; t <= T; ++t) Ek[t] = kE[ko + 7 + t];
      herm_dir3<T, T>(Eby, Ek, X1, P0y, P1y, P2y);
#pragma unroll
      for (int t = 0; t <= T; ++t) Ek[t] = kE[ko + 14 + t];
      herm_dir3<T, T>(Ebz, Ek, X2, P0z, P1z, P2z);
      const double w = eb * ke[k];
      const double sa = herm_sum<TS>(P0x, P0y, P0z, DA);
      v[0] = fma(w, herm_sum<TS>(P2x, P0y, P0z, DB) + sa, v[0]);
      v[1] = fma(w, herm_sum<TS>(P1x, P1y, P0z, DB), v[1]);
      v[2] = fma(w, herm_sum<TS>(P1x, P0y, P1z, DB), v[2]);
      v[3] = fma(w, herm_sum<TS>(P0x, P2y, P0z, DB) + sa, v[3]);
      v[4] = fma(w, herm_sum<TS>(P0x, P1y, P1z, DB), v[4]);
      v[5] = fma(w, herm_sum<TS>(P0x, P0y, P2z, DB) + sa, v[5]);
    }
  }
}

// the d- and f-sized forms in functions of their own: their register
// pressure (and spills) stays out of the p-sized form's code
template <int T>
__device__ __attribute__((noinline)) void gauge_gen_row_pair_call(const EriTileArgs &A,
                                                                  const double *tab,
                                                                  int64_t kf0, int64_t kf1,
                                                                  int64_t b0, int64_t b1,
                                                                  int bcode, int kcode,
                                                                  double v[6]) {
  gauge_gen_row_pair<T>(A, tab, kf0, kf1, b0, b1, bcode, kcode, v);
}

// TMAX: the largest Hermite order bound of the launch (2 for s and p bases, 4
// with d and no f functions, else 6): the larger forms, and their registers,
// stay out of kernels that never run them
template <int TMAX>
__device__ __forceinline__ void eri_gauge_gen_one_tile(const EriTileArgs &a, const double *tab,
                                                       int64_t slot, long long kept[4]) {
  const int kt = a.tasks[slot];
  const int bt = a.task_bra[slot];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *out, *outT = nullptr;
  constexpr int64_t SL = 6 * (int64_t)TILE * TILE;
  if (a.uslot_bk) {
    const int32_t s1 = a.uslot_bk[slot], s2 = a.uslot_kb[slot];
    out = s1 >= 0 ? a.panel + (int64_t)s1 * SL : nullptr;
    outT = s2 >= 0 ? a.panel + (int64_t)s2 * SL : nullptr;
  } else {
    out = a.panel + (slot - a.slot0) * SL;
  }
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const double db = a.Dmax[brow];
  const int cb = a.cls[brow];
  const int bcode = a.code[brow];
  const int64_t bfirst = a.row_first[brow], blast = a.row_first[brow + 1];
  int tb = gen_bucket(bcode);
  for (int o = 32; o > 0; o >>= 1) tb = max(tb, __shfl_xor(tb, o, 64));
  tb = __builtin_amdgcn_readfirstlane(tb);
  for (int i = 0; i < TILE / ERI_WAVES; ++i) {
    const int j = w + ERI_WAVES * i;
    const int64_t krow = (int64_t)kt * TILE + j;
    const double qk = a.Q[krow], dk = a.Dmax[krow];
    const int ck = a.cls[krow];
    const int kcode = __builtin_amdgcn_readfirstlane(a.code[krow]);
    const int64_t kf0 = a.row_first[krow], kf1 = a.row_first[krow + 1];
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool keep_bk = out && (qb * qk) * dk >= a.tau;
    const bool keep_kb = outT && (qk * qb) * db >= a.tau;
    if (keep_bk || keep_kb) {
      const int t = max(tb, gen_bucket(kcode));
      if (TMAX == 2 || t == 2)
        gauge_gen_row_pair<2>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, v);
      else if (TMAX == 4 || t == 4)
        gauge_gen_row_pair_call<4>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, v);
      else
        gauge_gen_row_pair_call<6>(a, tab, kf0, kf1, bfirst, blast, bcode, kcode, v);
      if (cb >= 0 && ck >= 0) {
        if (keep_bk) kept[cb * 2 + ck] += 1;
        if (keep_kb) kept[ck * 2 + cb] += 1;
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (out) out[c * TILE * TILE + j * TILE + lane] = keep_bk ? v[c] : 0.0;
      if (outT) outT[c * TILE * TILE + lane * TILE + j] = keep_kb ? v[c] : 0.0;
    }
  }
}

template <int TMAX>
__global__ void __launch_bounds__(ERI_THREADS) k_eri_gauge_tiles_gen(EriTileArgs a) {
  __shared__ double tab[BOYS_N * BOYS_LDG];
  if (a.overflow && *a.overflow) return;  // uniform
  if (a.d_total && (int64_t)blockIdx.x >= min(*a.d_total, a.cap)) return;  // uniform
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDG; t += ERI_THREADS) tab[t] = a.boysg[t];
  __syncthreads();
  long long kept[4] = {0, 0, 0, 0};
  eri_gauge_gen_one_tile<TMAX>(a, tab, a.slot0 + blockIdx.x, kept);
  eri_count(a, kept);
}

// Persistent variant; same queue protocol as k_eri_tiles_queue.
template <int TMAX>
__global__ void __launch_bounds__(ERI_THREADS) k_eri_gauge_tiles_queue_gen(
    EriTileArgs a, const int32_t *order, unsigned long long *qctr, int64_t n_host) {
  __shared__ double tab[BOYS_N * BOYS_LDG];
  __shared__ int64_t s_next;
  if (a.overflow && *a.overflow) return;  // uniform
  const int64_t n = a.d_total ? min(*a.d_total, a.cap) : n_host;
  for (int t = threadIdx.x; t < BOYS_N * BOYS_LDG; t += ERI_THREADS) tab[t] = a.boysg[t];
  long long kept[4] = {0, 0, 0, 0};
  for (;;) {
    __syncthreads();  // table staged; the previous s_next read by every thread
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(qctr, 1ull);
    __syncthreads();
    const int64_t i = s_next;
    if (i >= n) break;  // uniform
    eri_gauge_gen_one_tile<TMAX>(a, tab, order[i], kept);
  }
  eri_count(a, kept);
}

void launch_eri_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s) {
  if (nslots <= 0) return;
  if (a.boysg && a.gen_tmax <= 4)
    hipLaunchKernelGGL(k_eri_tiles_gen<4>, dim3((unsigned)nslots), dim3(GEN_THREADS), 0, s, a);
  else if (a.boysg)
    hipLaunchKernelGGL(k_eri_tiles_gen<6>, dim3((unsigned)nslots), dim3(GEN_THREADS), 0, s, a);
  else if (a.code)
    hipLaunchKernelGGL(k_eri_tiles_cart, dim3((unsigned)nslots), dim3(ERI_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL(k_eri_tiles<false>, dim3((unsigned)nslots), dim3(ERI_THREADS), 0, s, a);
}

void launch_eri_tiles_queue(const EriTileArgs &a, const int32_t *order, unsigned long long *qctr,
                            int64_t n_host, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  // the d-sized general kernel's smaller workgroups: three per compute unit
  // where the others run two (nblocks is sized for two)
  const int gblocks = nblocks / 2 * gen_blocks<4>() + nblocks % 2;
  if (a.boysg && a.gen_tmax <= 4)
    hipLaunchKernelGGL(k_eri_tiles_queue_gen<4>, dim3((unsigned)gblocks), dim3(GEN_THREADS), 0,
                       s, a, order, qctr, n_host);
  else if (a.boysg)
    hipLaunchKernelGGL(k_eri_tiles_queue_gen<6>, dim3((unsigned)nblocks), dim3(GEN_THREADS), 0,
                       s, a, order, qctr, n_host);
  else if (a.code)
    hipLaunchKernelGGL(k_eri_tiles_queue_cart, dim3((unsigned)nblocks), dim3(ERI_THREADS), 0, s,
                       a, order, qctr, n_host);
  else
    hipLaunchKernelGGL(k_eri_tiles_queue<false>, dim3((unsigned)nblocks), dim3(ERI_THREADS), 0,
                       s, a, order, qctr, n_host);
}

void launch_eri_gauge_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s) {
  if (nslots <= 0) return;
  if (a.code && a.gen_tmax <= 2)  // Cartesian bases: the general form
    hipLaunchKernelGGL(k_eri_gauge_tiles_gen<2>, dim3((unsigned)nslots), dim3(ERI_THREADS), 0,
                       s, a);
  else if (a.code && a.gen_tmax <= 4)
    hipLaunchKernelGGL(k_eri_gauge_tiles_gen<4>, dim3((unsigned)nslots), dim3(ERI_THREADS), 0,
                       s, a);
  else if (a.code)
    hipLaunchKernelGGL(k_eri_gauge_tiles_gen<6>, dim3((unsigned)nslots), dim3(ERI_THREADS), 0,
                       s, a);
  else
    hipLaunchKernelGGL(k_eri_tiles<true>, dim3((unsigned)nslots), dim3(ERI_THREADS), 0, s, a);
}

void launch_eri_gauge_tiles_queue(const EriTileArgs &a, const int32_t *order,
                                  unsigned long long *qctr, int64_t n_host, int nblocks,
                                  hipStream_t s) {
  if (nblocks <= 0) return;
  if (a.code && a.gen_tmax <= 2)
    hipLaunchKernelGGL(k_eri_gauge_tiles_queue_gen<2>, dim3((unsigned)nblocks),
                       dim3(ERI_THREADS), 0, s, a, order, qctr, n_host);
  else if (a.code && a.gen_tmax <= 4)
    hipLaunchKernelGGL(k_eri_gauge_tiles_queue_gen<4>, dim3((unsigned)nblocks),
                       dim3(ERI_THREADS), 0, s, a, order, qctr, n_host);
  else if (a.code)
    hipLaunchKernelGGL(k_eri_gauge_tiles_queue_gen<6>, dim3((unsigned)nblocks),
                       dim3(ERI_THREADS), 0, s, a, order, qctr, n_host);
  else
    hipLaunchKernelGGL(k_eri_tiles_queue<true>, dim3((unsigned)nblocks), dim3(ERI_THREADS), 0,
                       s, a, order, qctr, n_host);
}

}  // namespace qdcb
