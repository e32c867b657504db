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

// Precision of a first-half launch: FP64 (stores V) or a reduced tier (adds
// to V).  The reduced tiers read the same FP64 staging buffers and round each
// operand as it is loaded for the MFMA:
//   FP32: v_mfma_f32_16x16x4f32, lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   BF16: v_mfma_f32_16x16x16bf16_1k, lane l supplies A[l%16][4(l/16)..+3] and
//         B[4(l/16)..+3][l%16];
// both accumulate D[4(l/16)+i][l%16] in FP32.  Block scaling: the integral
// tile (b, k) is multiplied by 2^-eI with 2^eI above the Cauchy-Schwarz bound
// Qmax_b Qmax_k of its elements and the density rows of ket tile k by 2^-eD
// with 2^eD above 2 max Dmax (the symmetrized density is a sum of two terms),
// so every rounded operand is at most 1 in magnitude; each task's products
// go to a scaled FP32 partial that is multiplied back by the exact
// 2^(eI+eD) into the FP32 running sum, and V (FP64) receives the sum once.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int scale_exp(double bound) {
  int e = 0;
  (void)frexp(bound, &e);  // bound < 2^e
  return bound > 0.0 ? e : 0;
}

template <int PREC>
struct FhAcc {
  typedef typename std::conditional<PREC == PREC_F64, dbl4, flt4>::type V;
  V acc[4][4];
  V part[PREC == PREC_F64 ? 1 : 4][PREC == PREC_F64 ? 1 : 4];
};

// One step's MFMAs from staged FP64 buffers A (KH x AS_LD) and B (KH x BS_LD).
template <int KH, int PREC>
__device__ __forceinline__ void fh_mfma(const double *Ac, const double *Bc, int wr, int wc, int lr,
                                        int lk, double sI, double sD, FhAcc<PREC> &f) {
  if constexpr (PREC == PREC_F64) {
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
        for (int c = 0; c < 4; ++c)
          f.acc[r][c] = MFMA_F64(av[r], bv[c], f.acc[r][c]);
    }
  } else if constexpr (PREC == PREC_F32) {
#pragma unroll
    for (int kk = 0; kk < KH / 4; ++kk) {
      const int j = kk * 4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = (float)(Ac[j * AS_LD + wr * 64 + r * 16 + lr] * sI);
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = (float)(Bc[j * BS_LD + wc * 64 + c * 16 + lr] * sD);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          f.part[r][c] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv[c], f.part[r][c], 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < KH / 16; ++kk) {
      bf16x4 av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = kk * 16 + 4 * lk + t;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          av[r][t] = (__bf16)(float)(Ac[j * AS_LD + wr * 64 + r * 16 + lr] * sI);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          bv[c][t] = (__bf16)(float)(Bc[j * BS_LD + wc * 64 + c * 16 + lr] * sD);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          f.part[r][c] =
              __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[r], bv[c], f.part[r][c], 0, 0, 0);
    }
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
  if (PREC != PREC_F64 && n0 + n1 == 0) return;  // uniform: nothing to add in this tier
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;  // wave's 64-row half (bra tile) and 64-column half
  const int64_t c0 = (int64_t)ct * FH_COLS;
  const int lr = lane & 15, lk = lane >> 4;
  const int Kt = TENSOR ? (int)blockIdx.y : 0;
  FhAcc<PREC> f;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) f.acc[r][c] = (typename FhAcc<PREC>::V){0, 0, 0, 0};
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
  if constexpr (PREC != PREC_F64)
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) f.part[r][c] = (typename FhAcc<PREC>::V){0, 0, 0, 0};
  // bra tile bound of this wave's half (block scales of the reduced tiers)
  const double qbw = PREC != PREC_F64 ? a.Qmax[bt0 + (two ? wr : 0)] : 0.0;
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
  int eI = 0, eD = 0;  // block-scale exponents of the current task (this wave's half)
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
    if (PREC != PREC_F64) {
      eI = scale_exp(qbw * a.Qmax[kt]);
      eD = scale_exp(2.0 * a.Dtmax[kt]);
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
  struct StepDesc {
    bool act, last;
    int eI, eD;
  };
  auto desc = [&]() -> StepDesc {
    // this wave's bra tile: active while the step is within its own need
    const int hh = TENSOR ? h % ns : h;
    const int own = wr == 0 ? ns0 : ns1;
    return StepDesc{(wr == 0 ? has0 : has1) && hh < own, hh == own - 1, eI, eD};
  };
  // one staged step: MFMAs when this wave's bra tile keeps the task; at the
  // task's last step the reduced tiers fold the scaled partial into the sum
  auto run = [&](const double *A, const double *B, const StepDesc &d) {
    if (!d.act) return;
    fh_mfma<KH, PREC>(A, B, wr, wc, lr, lk, ldexp(1.0, -d.eI), ldexp(1.0, -d.eD), f);
    if constexpr (PREC != PREC_F64) {
      if (!d.last) return;
      const float sc = ldexpf(1.0f, d.eI + d.eD);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          f.acc[r][c] += f.part[r][c] * sc;
          f.part[r][c] = (typename FhAcc<PREC>::V){0, 0, 0, 0};
        }
    }
  };

  // steps alternate between the two buffers: even steps in 0, odd in 1
  bool more = advance();
  StepDesc nxt = desc();
  if (more) issue(As0, Bs0);
  while (more) {
    wait_loads();
    __syncthreads();  // even step staged by every wave; buffer 1's readers are done
    StepDesc cur = nxt;
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
        if constexpr (PREC == PREC_F64) {
          const int lr_ = r * 16 + lk + 4 * i;
          const int64_t row = row0 + (a.perm ? a.perm[row0 + lr_] : lr_);
          a.V[row * a.ld + vc0 + wc * 64 + c * 16 + lr] = f.acc[r][c][i];
        } else {
          const int lr_ = r * 16 + 4 * lk + i;
          const int64_t row = row0 + (a.perm ? a.perm[row0 + lr_] : lr_);
          a.V[row * a.ld + c0 + wc * 64 + c * 16 + lr] += (double)f.acc[r][c][i];
        }
      }
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
    hipLaunchKernelGGL((k_first_half<FH_KH, PREC_BF16>), dim3((unsigned)grid), dim3(256), 0, s,
                       a, nbp, nct, ncx, (int64_t)0, 0);
  else
    hipLaunchKernelGGL((k_first_half<FH_KH, PREC_F32>), dim3((unsigned)grid), dim3(256), 0, s,
                       a, nbp, nct, ncx, (int64_t)0, 0);
}

}  // namespace qdcb
