// k_gemm.hip -- the first-half contraction (FP64 MFMA; FP32 / BF16 tiers).
//
// k_first_half: the first-half integral-density contraction of Eq.
// (firsthalf), V[mn][col] = sum over kept ket tiles of I[mn][kl] D~[kl][col],
// a block-sparse GEMM whose A blocks are the masked integral tiles and whose
// B rows are the symmetrized quaternion pair densities.  Each workgroup
// accumulates its V block over the kept ket tiles in registers, so V is
// written once and no atomics are used (the result is deterministic).
//
// FP64 path: v_mfma_f64_16x16x4f64, lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element i of lane l is D[l/16 + 4*i][l%16].
#include <climits>
#include <type_traits>

#include "kernels.h"

namespace qdcb {

#define MFMA_F64(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

// First half: one workgroup owns a pair of consecutive 64-row bra tiles (128
// rows, similar Schwarz factors, hence nearly identical ket lists) and a
// 128-column slice.  The two ordered ket-tile lists are merged on the fly;
// a ket tile kept for only one of the two bra tiles leaves the other half's
// staging rows stale and that half's wavefronts skip its MFMAs.  Four
// wavefronts hold 64 x 64 accumulator blocks (16 MFMA tiles each).
//
// Staging: steps of KH ket rows.  Each step's integral rows (2 x 64 bra
// values per ket row) and density rows (128 columns per ket row) go straight
// from global memory into LDS with 16-byte direct loads (one 1 KB row per
// wavefront instruction, no registers), double-buffered: the loads of step
// t+1 are issued right after the barrier that opens step t and complete while
// step t's MFMAs run.
//
// Workgroup order: the chip's 8 XCDs take workgroups round-robin and each
// has its own L2.  With at least 8 column slices, XCD x gets the slices
// x, x+8, ... and walks bra-tile pairs in order with its slices fastest, so
// the workgroups resident on one XCD share integral tiles (same bra pair,
// other slices) and density rows (neighbouring bra pairs, same slices).
constexpr int FH_COLS = 128;        // columns per workgroup
constexpr int FH_ROWS = 2 * TILE;   // bra rows per workgroup
constexpr int FH_KH = 16;           // ket rows staged per step
constexpr int AS_LD = FH_ROWS + 2;  // LDS row strides in doubles (padded against bank
constexpr int BS_LD = FH_COLS + 2;  // conflicts; 1040 B keeps rows 16-byte aligned)
constexpr int N_XCD = 8;

typedef __attribute__((address_space(3))) void *lds_ptr;

__device__ __forceinline__ void load_row_lds(const double *src, double *lds_row) {
  __builtin_amdgcn_global_load_lds(src, (lds_ptr)lds_row, 16, 0, 0);
}

__device__ __forceinline__ void wait_loads() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt unchanged (max)
}

// Reduced-precision tiers (k_first_half_lp): V += the tier's contributions.
//   FP32: v_mfma_f32_16x16x4f32, lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   BF16: v_mfma_f32_16x16x16bf16_1k, lane l supplies A[l%16][4(l/16)..+3] and
//         B[4(l/16)..+3][l%16];
// both accumulate D[4(l/16)+i][l%16] in FP32.  Block scaling: the integral
// tile (b, k) is multiplied by 2^-eI with 2^eI above the Cauchy-Schwarz bound
// Qmax_b Qmax_k of its elements and the density rows of ket tile k by 2^-eD
// with 2^eD above 2 max Dmax (the symmetrized density is a sum of two terms),
// so every rounded operand is at most 1 in magnitude.  The density rows come
// from an FP32 copy made with those scales (k_density_lo); each task's
// products go to a scaled FP32 partial that is multiplied back by the exact
// 2^(eI+eD) into the FP32 running sum, and V (FP64) receives the sum once.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// One step's FP64 MFMAs from staged buffers A (KH x AS_LD) and B (KH x BS_LD).
template <int KH>
__device__ __forceinline__ void fh_mfma(const double *Ac, const double *Bc, int wr, int wc, int lr,
                                        int lk, dbl4 (&acc)[4][4]) {
#pragma unroll
  for (int kk = 0; kk < KH / 4; ++kk) {
    const int j = kk * 4 + lk;
    double av[4], bv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = Ac[j * AS_LD + wr * 64 + r * 16 + lr];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = Bc[j * BS_LD + wc * 64 + c * 16 + lr];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
  }
}

// Gauge panel slot of the symmetric pair (K, L): xx, xy, xz, yy, yz, zz.
__device__ __forceinline__ int gauge_sym_index(int K, int L) {
  const int lo = K < L ? K : L, hi = K < L ? L : K;
  return lo * 3 - lo * (lo + 1) / 2 + hi;
}

// TENSOR (gauge term, FP64): workgroup (bp, ct, K = blockIdx.y) accumulates
// V^K over the kept ket tiles and, per ket tile, over L = x, y, z: each task
// is three runs of TILE / KH steps, the L-th reading panel tile (K, L) of the
// slot and the density rows' L-th column block.
template <int KH, int PREC, bool TENSOR = false>
__global__ void __launch_bounds__(256) k_first_half(FirstHalfArgs a, int nbp, int nct, int ncx,
                                                    int64_t ldK, int accumulate) {
  static_assert(PREC == PREC_F64, "the reduced tiers run in k_first_half_lp");
  constexpr int NS_MAX = TILE / KH;                      // steps per task and L run
  constexpr int NSTEP = (TENSOR ? 3 : 1) * NS_MAX;        // staged steps of a full task
  constexpr int64_t SLOT = (TENSOR ? 6 : 1) * TILE * TILE;  // doubles per panel slot
  // two staging buffers as distinct objects, so that the compiler can tell
  // the loads into one from the reads of the other
  __shared__ __attribute__((aligned(16))) double As0[KH * AS_LD], As1[KH * AS_LD];
  __shared__ __attribute__((aligned(16))) double Bs0[KH * BS_LD], Bs1[KH * BS_LD];
  if (a.overflow && *a.overflow) return;  // uniform: the task lists did not fit
  int bp, ct;
  if (ncx > 0) {  // XCD-aware order (see above)
    const int L = blockIdx.x, x = L % N_XCD, loc = L / N_XCD;
    bp = loc / ncx;
    ct = x + N_XCD * (loc % ncx);
    if (ct >= nct) return;  // uniform: ragged column slices
  } else {
    bp = blockIdx.x % nbp;
    ct = blockIdx.x / nbp;
  }
  const int bt0 = a.b0 + 2 * bp;
  const bool two = bt0 + 1 < a.b1;
  // panel slot bases and list starts of the two bra tiles
  const int64_t s0 = a.slot_base[bt0], s1 = two ? a.slot_base[bt0 + 1] : 0;
  const int64_t l0 = s0 + (a.toff ? a.toff[bt0] : 0);
  const int64_t l1 = two ? s1 + (a.toff ? a.toff[bt0 + 1] : 0) : 0;
  const int n0 = a.count[bt0], n1 = two ? a.count[bt0 + 1] : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;  // wave's 64-row half (bra tile) and 64-column half
  const int64_t c0 = (int64_t)ct * FH_COLS;
  const int lr = lane & 15, lk = lane >> 4;
  const int Kt = TENSOR ? (int)blockIdx.y : 0;
  struct {
    dbl4 acc[4][4];
  } f;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) f.acc[r][c] = (dbl4){0, 0, 0, 0};
  const int64_t vc0 = (TENSOR ? Kt * ldK : 0) + c0;  // this workgroup's first V column
  if (TENSOR && accumulate && (wr == 0 || two)) {
    // adding to V: the accumulators start from it (loaded before the loop,
    // where registers are free, instead of read-modify-writes at the end)
    const int64_t row0 = (int64_t)(bt0 + wr) * TILE;
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c)
        for (int i = 0; i < 4; ++i) {
          const int lr_ = r * 16 + lk + 4 * i;
          const int64_t row = row0 + (a.perm ? a.perm[row0 + lr_] : lr_);
          f.acc[r][c][i] = a.V[row * a.ld + vc0 + wc * 64 + c * 16 + lr];
        }
  }
  // bra tile bounds of the pair (step skipping)
  const double qm0 = a.sthr ? a.Qmax[bt0] : 0.0, qm1 = a.sthr && two ? a.Qmax[bt0 + 1] : 0.0;
  const double tq = a.tau * (1.0 - 1e-12);
  int i0 = 0, i1 = 0;
  // step state: current task's ket tile and tiles, sub-step h within the task;
  // ns = steps per L run of the task (the longer of the two bra tiles' needs),
  // ns0 / ns1 = each bra tile's own (0 when it does not keep the task)
  const double *P0 = nullptr, *P1 = nullptr;
  int kt = 0, h = NSTEP, nst = NSTEP, ns = NS_MAX, ns0 = NS_MAX, ns1 = NS_MAX;
  // step bounds of the two list heads, loaded during the task before theirs
  // (off the path between a barrier and the next step's loads)
  double th0[NS_MAX - 1], th1[NS_MAX - 1];
  int th_k0 = -1, th_k1 = -1;
  bool has0 = false, has1 = false;
  // heads of the two ordered lists, read one task ahead so that the list
  // reads are off the path between a barrier and the next step's loads
  // (with their panel ranks when the lists are tier sub-lists)
  int nk0 = n0 > 0 ? a.tasks[l0] : INT_MAX;
  int nk1 = n1 > 0 ? a.tasks[l1] : INT_MAX;
  int nr0 = n0 > 0 && a.rank ? a.rank[l0] : 0;
  int nr1 = n1 > 0 && a.rank ? a.rank[l1] : 0;
  // advance to the next step; false when the merged lists are exhausted
  auto load_th = [&](int k, double (&th)[NS_MAX - 1]) {
#pragma unroll
    for (int st = 1; st < NS_MAX; ++st) th[st - 1] = a.sthr[(int64_t)k * NS_MAX + st];
  };
  auto advance = [&]() -> bool {
    if (++h < nst) {
      if (a.sthr && h == 1) {  // the heads are known by now: their step bounds
        th_k0 = __builtin_amdgcn_readfirstlane(nk0);
        th_k1 = __builtin_amdgcn_readfirstlane(nk1);
        if (th_k0 != INT_MAX) load_th(th_k0, th0);
        if (th_k1 != INT_MAX) load_th(th_k1, th1);
      }
      return true;
    }
    const int k0 = __builtin_amdgcn_readfirstlane(nk0), k1 = __builtin_amdgcn_readfirstlane(nk1);
    if (k0 == INT_MAX && k1 == INT_MAX) return false;
    kt = k0 < k1 ? k0 : k1;
    has0 = k0 == kt;
    has1 = k1 == kt;
    if (has0) {
      const int64_t r0 = a.rank ? __builtin_amdgcn_readfirstlane(nr0) : i0;
      P0 = a.panel + (s0 + r0 - a.slot0) * SLOT;
      ++i0;
      nk0 = i0 < n0 ? a.tasks[l0 + i0] : INT_MAX;
      if (a.rank && i0 < n0) nr0 = a.rank[l0 + i0];
    } else {
      P0 = nullptr;
    }
    if (has1) {
      const int64_t r1 = a.rank ? __builtin_amdgcn_readfirstlane(nr1) : i1;
      P1 = a.panel + (s1 + r1 - a.slot0) * SLOT;
      ++i1;
      nk1 = i1 < n1 ? a.tasks[l1 + i1] : INT_MAX;
      if (a.rank && i1 < n1) nr1 = a.rank[l1 + i1];
    } else {
      P1 = nullptr;
    }
    if (a.sthr) {
      // steps whose largest ket bound passes against the bra tile's largest Q
      // (a prefix: the bounds decrease with the step; step 0 holds the ket
      // tile's largest bound, which every kept task passes)
      double th[NS_MAX - 1];
      if (kt == th_k0) {
#pragma unroll
        for (int st = 0; st < NS_MAX - 1; ++st) th[st] = th0[st];
      } else if (kt == th_k1) {
#pragma unroll
        for (int st = 0; st < NS_MAX - 1; ++st) th[st] = th1[st];
      } else {
        load_th(kt, th);  // the first task, or one that followed a one-step task
      }
      th_k0 = th_k1 = -1;
      int need0 = 1, need1 = 1;
#pragma unroll
      for (int st = 1; st < NS_MAX; ++st) {
        if (qm0 * th[st - 1] >= tq) need0 = st + 1;
        if (qm1 * th[st - 1] >= tq) need1 = st + 1;
      }
      ns0 = has0 ? need0 : 0;
      ns1 = has1 ? need1 : 0;
      ns = ns0 > ns1 ? ns0 : ns1;
      nst = (TENSOR ? 3 : 1) * ns;
    }
    h = 0;
    return true;
  };
  // direct loads of the current step: wave w stages rows w, w+4, ... of the
  // integral slice (lanes 0-31: tile of bra tile bt0, lanes 32-63: of bt0+1)
  // and of the density slice
  auto issue = [&](double *A, double *B) {
    int hh = h;
    int64_t poff = 0, doff = 0;
    if constexpr (TENSOR) {
      const int Lc = h / ns;
      hh = h - Lc * ns;
      poff = (int64_t)gauge_sym_index(Kt, Lc) * (TILE * TILE);
      doff = Lc * ldK;
    }
    const double *P = lane < 32 ? P0 : P1;
#pragma unroll
    for (int q = 0; q < KH / 4; ++q) {
      const int jj = w + 4 * q;
      if (P) load_row_lds(P + poff + (hh * KH + jj) * TILE + 2 * (lane & 31), A + jj * AS_LD);
    }
    // density rows (stored in the tiles' row order)
    const double *Dr = a.D + ((int64_t)kt * TILE + hh * KH) * a.ld + doff + c0 + 2 * lane;
#pragma unroll
    for (int q = 0; q < KH / 4; ++q) {
      const int r = w + 4 * q;
      load_row_lds(Dr + r * a.ld, B + r * BS_LD);
    }
  };
  // what the MFMAs of a staged step need, taken when the step is issued
  auto desc = [&]() -> int {
    // this wave's bra tile: active while the step is within its own need
    const int hh = TENSOR ? h % ns : h;
    const int own = wr == 0 ? ns0 : ns1;
    return (wr == 0 ? has0 : has1) && hh < own;
  };
  // one staged step: MFMAs when this wave's bra tile keeps the task
  auto run = [&](const double *A, const double *B, int act) {
    if (!act) return;
    fh_mfma<KH>(A, B, wr, wc, lr, lk, f.acc);
  };

  // steps alternate between the two buffers: even steps in 0, odd in 1
  bool more = advance();
  int nxt = desc();
  if (more) issue(As0, Bs0);
  while (more) {
    wait_loads();
    __syncthreads();  // even step staged by every wave; buffer 1's readers are done
    int cur = nxt;
    more = advance();
    if (more) {
      nxt = desc();
      issue(As1, Bs1);
    }
    run(As0, Bs0, cur);
    if (!more) break;
    wait_loads();
    __syncthreads();  // odd step staged; buffer 0's readers are done
    cur = nxt;
    more = advance();
    if (more) {
      nxt = desc();
      issue(As0, Bs0);
    }
    run(As1, Bs1, cur);
  }
  if (wr == 1 && !two) return;
  const int64_t row0 = (int64_t)(bt0 + wr) * TILE;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lr_ = r * 16 + lk + 4 * i;
        const int64_t row = row0 + (a.perm ? a.perm[row0 + lr_] : lr_);
        a.V[row * a.ld + vc0 + wc * 64 + c * 16 + lr] = f.acc[r][c][i];
      }
}

// ---------------------------------------------------------------------------
// Reduced tiers.  Same workgroup and list structure as k_first_half, over the
// tier's sub-lists.  The integral tiles of these entries were rounded once,
// in their own panel slots, after they were made (k_panel_lo): FP32 tiles
// [ket j][bra m] (16 KB) and BF16 tiles in groups of four ket rows
// ([j / 4][m][j % 4], 8 KB), both already scaled by 2^-eI.  A step stages 8
// (FP32) or 4 KB (BF16) of integrals and 8 KB of scaled FP32 densities, and
// three steps are in flight, the loads of step t + 2 issued when step t
// starts (a reduced-precision step is too short to cover the latency of
// loads issued one step ahead).  The list reads go through the scalar cache,
// so the vector memory counter holds only the staging loads: LP_LOADS per
// wave and step.
//
// LDS row strides (4-byte words): FP32 integral and density rows 144 (rows
// j and j + 1, read by lane groups lk and lk + 1, start 16 banks apart); BF16
// integral blocks 288 (blocks lk and lk + 1 start 32 banks apart) and BF16
// density rows 132 (rows 4 lk + t of lane groups lk and lk + 1 start 16
// banks apart).
constexpr int A32_LD = FH_COLS + 16;       // FP32 integral row (floats)
constexpr int A16_LD = 2 * (FH_COLS + 16);  // BF16 block of four ket rows (words)
template <int TIER> constexpr int lp_bl_ld() { return TIER == PREC_F32 ? FH_COLS + 16 : FH_COLS + 4; }
template <int TIER> constexpr int lp_a_words() {
  return TIER == PREC_F32 ? FH_KH * A32_LD : (FH_KH / 4) * A16_LD;
}
template <int TIER> constexpr int lp_loads() { return TIER == PREC_F32 ? 8 : 5; }

typedef const __attribute__((address_space(4))) int32_t *ci32p;
typedef const __attribute__((address_space(4))) int64_t *ci64p;
typedef const __attribute__((address_space(4))) double *cdblp;

// One step of a reduced tier into the per-task partial: A (the step's
// rounded integral rows, layout above), B (KH rows of scaled FP32 densities).
template <int TIER>
__device__ __forceinline__ void lp_mfma(const float *Ac, const float *Bc, int wr, int wc, int lr,
                                        int lk, flt4 (&part)[4][4]) {
  constexpr int KH = FH_KH, BL = lp_bl_ld<TIER>();
  if constexpr (TIER == PREC_F32) {
#pragma unroll
    for (int kk = 0; kk < KH / 4; ++kk) {
      const int j = kk * 4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = Ac[j * A32_LD + wr * 64 + r * 16 + lr];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bc[j * BL + wc * 64 + c * 16 + lr];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          part[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv[c], part[r][c], 0, 0, 0);
    }
  } else {
    static_assert(KH == 16, "one BF16 MFMA step of 16 ket rows");
    bf16x4 av[4], bv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      av[r] = *reinterpret_cast<const bf16x4 *>(Ac + lk * A16_LD + 2 * (wr * 64 + r * 16 + lr));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = 4 * lk + t;
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c][t] = (__bf16)Bc[j * BL + wc * 64 + c * 16 + lr];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        part[r][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[r], bv[c], part[r][c], 0, 0, 0);
  }
}

// Task descriptor of a reduced-tier list entry (k_tier_split): the steps its
// bra tile needs (1..4), and the block-scale exponents eI, eD.
__device__ __forceinline__ int lp_steps(int d) { return d & 7; }
__device__ __forceinline__ int lp_eI(int d) { return ((d >> 3) & 2047) - 1024; }
__device__ __forceinline__ int lp_eD(int d) { return ((d >> 14) & 2047) - 1024; }

template <int TIER>
__global__ void __launch_bounds__(256, 2) k_first_half_lp(FirstHalfArgs a, int nbp, int nct,
                                                          int ncx) {
  constexpr int KH = FH_KH, BL = lp_bl_ld<TIER>(), AW = lp_a_words<TIER>();
  constexpr int64_t SLOT = TILE * TILE;
  // three staging buffers as distinct objects (so that the compiler can tell
  // the loads into one from the reads of another)
  __shared__ __attribute__((aligned(16))) float A0[AW], A1[AW], A2[AW];
  __shared__ __attribute__((aligned(16))) float B0[KH * BL], B1[KH * BL], B2[KH * BL];
  if (a.overflow && *a.overflow) return;  // uniform: the task lists did not fit
  int bp, ct;
  if (ncx > 0) {  // XCD-aware order (as k_first_half)
    const int L = blockIdx.x, x = L % N_XCD, loc = L / N_XCD;
    bp = loc / ncx;
    ct = x + N_XCD * (loc % ncx);
    if (ct >= nct) return;  // uniform: ragged column slices
  } else {
    bp = blockIdx.x % nbp;
    ct = blockIdx.x / nbp;
  }
  const ci32p tasks = (ci32p)a.tasks, rank = (ci32p)a.rank, tdesc = (ci32p)a.tdesc;
  const ci32p count = (ci32p)a.count, toff = (ci32p)a.toff;
  const ci64p slot_base = (ci64p)a.slot_base;
  const int bt0 = a.b0 + 2 * bp;
  const bool two = bt0 + 1 < a.b1;
  const int64_t s0 = slot_base[bt0], s1 = two ? slot_base[bt0 + 1] : 0;
  const int64_t l0 = s0 + toff[bt0], l1 = two ? s1 + toff[bt0 + 1] : 0;
  const int n0 = count[bt0], n1 = two ? count[bt0 + 1] : 0;
  if (n0 + n1 == 0) return;  // uniform: nothing to add in this tier
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;
  const int64_t c0 = (int64_t)ct * FH_COLS;
  const int lr = lane & 15, lk = lane >> 4;
  flt4 acc[4][4], part[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) acc[r][c] = part[r][c] = (flt4){0, 0, 0, 0};
  // merged walk over the two lists (heads read one task ahead)
  int i0 = 0, i1 = 0;
  int nk0 = n0 > 0 ? tasks[l0] : INT_MAX, nk1 = n1 > 0 ? tasks[l1] : INT_MAX;
  int nr0 = n0 > 0 ? rank[l0] : 0, nr1 = n1 > 0 ? rank[l1] : 0;
  int nd0 = n0 > 0 ? tdesc[l0] : 0, nd1 = n1 > 0 ? tdesc[l1] : 0;
  const double *P0 = nullptr, *P1 = nullptr;
  int kt = 0, h = 0, nst = 0, ns0 = 0, ns1 = 0, d0 = 0, d1 = 0;
  auto advance = [&]() -> bool {
    if (++h < nst) return true;
    if (nk0 == INT_MAX && nk1 == INT_MAX) return false;
    kt = nk0 < nk1 ? nk0 : nk1;
    const bool has0 = nk0 == kt, has1 = nk1 == kt;
    P0 = P1 = nullptr;
    ns0 = ns1 = 0;
    if (has0) {
      P0 = a.panel + (s0 + nr0 - a.slot0) * SLOT;
      d0 = nd0;
      ns0 = lp_steps(d0);
      ++i0;
      nk0 = i0 < n0 ? tasks[l0 + i0] : INT_MAX;
      nr0 = i0 < n0 ? rank[l0 + i0] : 0;
      nd0 = i0 < n0 ? tdesc[l0 + i0] : 0;
    }
    if (has1) {
      P1 = a.panel + (s1 + nr1 - a.slot0) * SLOT;
      d1 = nd1;
      ns1 = lp_steps(d1);
      ++i1;
      nk1 = i1 < n1 ? tasks[l1 + i1] : INT_MAX;
      nr1 = i1 < n1 ? rank[l1 + i1] : 0;
      nd1 = i1 < n1 ? tdesc[l1 + i1] : 0;
    }
    nst = ns0 > ns1 ? ns0 : ns1;
    h = 0;
    return true;
  };
  // the current step's loads into stage st (a lane group whose tile does not
  // keep the task reads the other tile's rows, unused).  FP32: wave w stages
  // integral rows w, w+4, ... (lanes 0-15 bra tile bt0, 16-31 bt0+1);
  // BF16: wave w stages the block of ket rows 4w..4w+3 (lanes 0-31 bt0, 32-63
  // bt0+1).  Density rows w, w+4, ... (lanes 0-31, 16 bytes each).
  auto issue = [&](float *A, float *B) {
    if constexpr (TIER == PREC_F32) {
      const float *P = reinterpret_cast<const float *>(lane < 16 ? (P0 ? P0 : P1)
                                                                 : (P1 ? P1 : P0));
#pragma unroll
      for (int q = 0; q < KH / 4; ++q) {
        const int jj = w + 4 * q;
        if (lane < 32)
          __builtin_amdgcn_global_load_lds(P + (h * KH + jj) * TILE + 4 * (lane & 15),
                                           (lds_ptr)(A + jj * A32_LD), 16, 0, 0);
      }
    } else {
      const __bf16 *P = reinterpret_cast<const __bf16 *>(lane < 32 ? (P0 ? P0 : P1)
                                                                    : (P1 ? P1 : P0));
      __builtin_amdgcn_global_load_lds(P + ((h * KH) / 4 + w) * (4 * TILE) + 8 * (lane & 31),
                                       (lds_ptr)(A + w * A16_LD), 16, 0, 0);
    }
    const float *Dr = a.Dlo + ((int64_t)kt * TILE + h * KH) * a.ld + c0 + 4 * lane;
#pragma unroll
    for (int q = 0; q < KH / 4; ++q) {
      const int r = w + 4 * q;
      if (lane < 32)
        __builtin_amdgcn_global_load_lds(Dr + r * a.ld, (lds_ptr)(B + r * BL), 16, 0, 0);
    }
  };
  struct StepDesc {
    bool act, last;
    int eI, eD;
  };
  auto desc = [&]() -> StepDesc {
    const int own = wr == 0 ? ns0 : ns1, d = wr == 0 ? d0 : d1;
    return StepDesc{h < own, h == own - 1, lp_eI(d), lp_eD(d)};
  };
  auto run = [&](const float *A, const float *B, StepDesc d) {
    if (!d.act) return;
    lp_mfma<TIER>(A, B, wr, wc, lr, lk, part);
    if (!d.last) return;
    const float sc = ldexpf(1.0f, d.eI + d.eD);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[r][c] += part[r][c] * sc;
        part[r][c] = (flt4){0, 0, 0, 0};
      }
  };
  // three stages: step t in buffer t % 3.  Before step t runs, its loads
  // (every wave's) are complete while step t + 1's may still be in flight;
  // then step t + 2 is staged into the buffer step t - 1 was read from.  The
  // barrier carries no memory fence: a fence would wait for every staging
  // load, including step t + 1's.
  bool more0 = advance();
  StepDesc da = desc();
  if (more0) issue(A0, B0);
  bool more1 = more0 && advance();
  StepDesc db = desc();
  if (more1) issue(A1, B1);
  auto step = [&](const float *Ar, const float *Br, float *Ai, float *Bi) {
    if (more1)  // vmcnt(LP_LOADS): the next step's loads may be pending
      __builtin_amdgcn_s_waitcnt(0x0F70 | lp_loads<TIER>());
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    const bool more2 = more1 && advance();
    const StepDesc dc = desc();
    if (more2) issue(Ai, Bi);
    run(Ar, Br, da);
    da = db;
    db = dc;
    more0 = more1;
    more1 = more2;
  };
  while (more0) {
    step(A0, B0, A2, B2);
    if (!more0) break;
    step(A1, B1, A0, B0);
    if (!more0) break;
    step(A2, B2, A1, B1);
  }
  if (wr == 1 && !two) return;
  const int64_t row0 = (int64_t)(bt0 + wr) * TILE;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lr_ = r * 16 + 4 * lk + i;
        const int64_t row = row0 + (a.perm ? a.perm[row0 + lr_] : lr_);
        a.V[row * a.ld + c0 + wc * 64 + c * 16 + lr] += (double)acc[r][c][i];
      }
}

// Rounding of the reduced-tier integral tiles, in place, after they are
// made: workgroup (b - b0, y) takes entries y, y + gridDim.y, ... of the
// FP32 and BF16 sub-lists of bra tile b, reads the entry's whole FP64 tile,
// and writes its scaled copy x 2^-eI into the start of the same slot (FP32
// [j][m]; BF16 [j / 4][m][j % 4]).  Every value is read before any is written
// (loads complete, then a barrier); slots of different entries are disjoint.
__global__ void __launch_bounds__(256) k_panel_lo(PanelLoArgs a) {
  if (a.overflow && *a.overflow) return;  // uniform: the task lists did not fit
  constexpr int64_t SLOT = TILE * TILE;
  const int b = a.b0 + blockIdx.x, t = threadIdx.x;
  const int n32 = a.tcount[a.ntiles + b], n16 = a.tcount[2 * a.ntiles + b];
  const int64_t sb = a.slot_base[b];
  for (int e = blockIdx.y; e < n32 + n16; e += gridDim.y) {
    const bool bf = e >= n32;  // uniform
    const int64_t l = sb + (bf ? a.toff[2 * a.ntiles + b] + (e - n32) : a.toff[a.ntiles + b] + e);
    double *T = a.panel + (sb + a.rank[l] - a.slot0) * SLOT;
    const double sI = ldexp(1.0, -lp_eI(a.tdesc[l]));
    double v[16];
    if (!bf) {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = T[t + 256 * i];
      wait_loads();
      __syncthreads();
      float *F = reinterpret_cast<float *>(T);
#pragma unroll
      for (int i = 0; i < 16; ++i) F[t + 256 * i] = (float)(v[i] * sI);
    } else {
      const int m = t & 63, q = t >> 6;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * i + r] = T[(4 * (q + 4 * i) + r) * TILE + m];
      wait_loads();
      __syncthreads();
      bf16x4 *H = reinterpret_cast<bf16x4 *>(T);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bf16x4 x;
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (__bf16)(float)(v[4 * i + r] * sI);
        H[(q + 4 * i) * TILE + m] = x;
      }
    }
    // slots of different entries are disjoint: no barrier before the next
  }
}

// The reduced tiers' density operand: Dlo[r][c] = D~[r][c] 2^-eD (rounded to
// FP32), eD = scale_exp(2 Dtmax[tile of r]), over rows [0, rows) of stride ld
// (a multiple of 4).
__global__ void __launch_bounds__(256) k_density_lo(int64_t rows, int64_t ld, const double *D,
                                                    const double *Dtmax, float *Dlo) {
  const int64_t n4 = rows * ld / 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = 4 * i, r = e / ld;
    const double sc = ldexp(1.0, -scale_exp(2.0 * Dtmax[r / TILE]));
    const double2 x = *reinterpret_cast<const double2 *>(D + e);
    const double2 y = *reinterpret_cast<const double2 *>(D + e + 2);
    *reinterpret_cast<float4 *>(Dlo + e) =
        make_float4((float)(x.x * sc), (float)(x.y * sc), (float)(y.x * sc), (float)(y.y * sc));
  }
}

void launch_density_lo(int64_t rows, int64_t ld, const double *D, const double *Dtmax, float *Dlo,
                       hipStream_t s) {
  const int64_t n4 = rows * ld / 4;
  if (n4 <= 0) return;
  const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_density_lo, dim3((unsigned)blocks), dim3(256), 0, s, rows, ld, D, Dtmax,
                     Dlo);
}

void launch_panel_lo(const PanelLoArgs &a, hipStream_t s) {
  if (a.b1 <= a.b0) return;
  // 8 workgroups per bra tile share its entries (at most 32768 tiles)
  hipLaunchKernelGGL(k_panel_lo, dim3((unsigned)(a.b1 - a.b0), 8), dim3(256), 0, s, a);
}

void launch_first_half(const FirstHalfArgs &a, hipStream_t s) {
  if (a.b1 <= a.b0 || a.ncol_tiles <= 0) return;
  const int nbp = (a.b1 - a.b0 + 1) / 2, nct = a.ncol_tiles;
  const int ncx = !a.plain_order && nct >= N_XCD ? (nct + N_XCD - 1) / N_XCD : 0;
  // at most 32768 bra pairs x (ncol / 128 + 8) slices: well inside the grid limit
  const int64_t grid = ncx ? (int64_t)N_XCD * ncx * nbp : (int64_t)nbp * nct;
  hipLaunchKernelGGL((k_first_half<FH_KH, PREC_F64>), dim3((unsigned)grid), dim3(256), 0, s, a,
                     nbp, nct, ncx, (int64_t)0, 0);
}

void launch_first_half_gauge(const FirstHalfArgs &a, int64_t ldK, int accumulate,
                             hipStream_t s) {
  if (a.b1 <= a.b0 || a.ncol_tiles <= 0) return;
  const int nbp = (a.b1 - a.b0 + 1) / 2, nct = a.ncol_tiles;
  const int ncx = !a.plain_order && nct >= N_XCD ? (nct + N_XCD - 1) / N_XCD : 0;
  const int64_t grid = ncx ? (int64_t)N_XCD * ncx * nbp : (int64_t)nbp * nct;
  hipLaunchKernelGGL((k_first_half<FH_KH, PREC_F64, true>), dim3((unsigned)grid, 3), dim3(256),
                     0, s, a, nbp, nct, ncx, ldK, accumulate);
}

void launch_first_half_lp(const FirstHalfArgs &a, int tier, hipStream_t s) {
  if (a.b1 <= a.b0 || a.ncol_tiles <= 0) return;
  const int nbp = (a.b1 - a.b0 + 1) / 2, nct = a.ncol_tiles;
  const int ncx = !a.plain_order && nct >= N_XCD ? (nct + N_XCD - 1) / N_XCD : 0;
  const int64_t grid = ncx ? (int64_t)N_XCD * ncx * nbp : (int64_t)nbp * nct;
  if (tier == 2)
    hipLaunchKernelGGL(k_first_half_lp<PREC_BF16>, dim3((unsigned)grid), dim3(256), 0, s, a, nbp,
                       nct, ncx);
  else
    hipLaunchKernelGGL(k_first_half_lp<PREC_F32>, dim3((unsigned)grid), dim3(256), 0, s, a, nbp,
                       nct, ncx);
}

}  // namespace qdcb
