// k_gemm.hip -- FP64 MFMA contractions.
//
// k_first_half: the first-half integral-density contraction of Eq.
// (firsthalf), V[mn][col] = sum over kept ket tiles of I[mn][kl] D~[kl][col],
// a block-sparse GEMM whose A blocks are the masked integral tiles and whose
// B rows are the symmetrized quaternion pair densities.  Each workgroup
// accumulates its V block over the kept ket tiles in registers, so V is
// written once and no atomics are used (the result is deterministic).
//
// k_dgemm_batched: plain batched GEMM for the second-half quarter
// transforms (Sec. 2.4.2).
//
// Both use v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element i of lane l is D[l/16 + 4*i][l%16].
#include <climits>

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

// One step's MFMAs from staged buffers A (KH x AS_LD) and B (KH x BS_LD).
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

template <int KH>
__global__ void __launch_bounds__(256) k_first_half(FirstHalfArgs a, int nbp, int nct, int ncx) {
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
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;  // wave's 64-row half (bra tile) and 64-column half
  const int64_t c0 = (int64_t)ct * FH_COLS;
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 acc[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};

  const int64_t s0 = a.slot_base[bt0], s1 = two ? a.slot_base[bt0 + 1] : 0;
  const int n0 = a.count[bt0], n1 = two ? a.count[bt0 + 1] : 0;
  int i0 = 0, i1 = 0;
  // step state: current task's ket tile and tiles, sub-step h within the task
  const double *P0 = nullptr, *P1 = nullptr;
  int kt = 0, h = TILE / KH;
  bool has0 = false, has1 = false;
  // heads of the two ordered lists, read one task ahead so that the list
  // reads are off the path between a barrier and the next step's loads
  int nk0 = n0 > 0 ? a.tasks[s0] : INT_MAX;
  int nk1 = n1 > 0 ? a.tasks[s1] : INT_MAX;
  // advance to the next step; false when the merged lists are exhausted
  auto advance = [&]() -> bool {
    if (++h < TILE / KH) return true;
    const int k0 = __builtin_amdgcn_readfirstlane(nk0), k1 = __builtin_amdgcn_readfirstlane(nk1);
    if (k0 == INT_MAX && k1 == INT_MAX) return false;
    kt = k0 < k1 ? k0 : k1;
    has0 = k0 == kt;
    has1 = k1 == kt;
    P0 = has0 ? a.panel + (s0 + i0 - a.slot0) * (TILE * TILE) : nullptr;
    P1 = has1 ? a.panel + (s1 + i1 - a.slot0) * (TILE * TILE) : nullptr;
    if (has0) {
      ++i0;
      nk0 = i0 < n0 ? a.tasks[s0 + i0] : INT_MAX;
    }
    if (has1) {
      ++i1;
      nk1 = i1 < n1 ? a.tasks[s1 + i1] : INT_MAX;
    }
    h = 0;
    return true;
  };
  // direct loads of the current step: wave w stages rows w, w+4, ... of the
  // integral slice (lanes 0-31: tile of bra tile bt0, lanes 32-63: of bt0+1)
  // and of the density slice
  auto issue = [&](double *A, double *B) {
    const double *P = lane < 32 ? P0 : P1;
#pragma unroll
    for (int q = 0; q < KH / 4; ++q) {
      const int jj = w + 4 * q;
      if (P) load_row_lds(P + (h * KH + jj) * TILE + 2 * (lane & 31), A + jj * AS_LD);
    }
    const double *Dr = a.D + ((int64_t)kt * TILE + h * KH) * a.ld + c0 + 2 * lane;
#pragma unroll
    for (int q = 0; q < KH / 4; ++q) {
      const int r = w + 4 * q;
      load_row_lds(Dr + r * a.ld, B + r * BS_LD);
    }
  };

  // steps alternate between the two buffers: even steps in 0, odd in 1
  bool more = advance();
  bool act = wr == 0 ? has0 : has1;  // uniform per wavefront
  if (more) issue(As0, Bs0);
  while (more) {
    wait_loads();
    __syncthreads();  // even step staged by every wave; buffer 1's readers are done
    bool act_cur = act;
    more = advance();
    if (more) {
      act = wr == 0 ? has0 : has1;
      issue(As1, Bs1);
    }
    if (act_cur) fh_mfma<KH>(As0, Bs0, wr, wc, lr, lk, acc);
    if (!more) break;
    wait_loads();
    __syncthreads();  // odd step staged; buffer 0's readers are done
    act_cur = act;
    more = advance();
    if (more) {
      act = wr == 0 ? has0 : has1;
      issue(As0, Bs0);
    }
    if (act_cur) fh_mfma<KH>(As1, Bs1, wr, wc, lr, lk, acc);
  }
  if (wr == 1 && !two) return;
  const int64_t row0 = (int64_t)(bt0 + wr) * TILE;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + r * 16 + lk + 4 * i;
        a.V[row * a.ld + c0 + wc * 64 + c * 16 + lr] = acc[r][c][i];
      }
}

void launch_first_half(const FirstHalfArgs &a, hipStream_t s) {
  if (a.b1 <= a.b0 || a.ncol_tiles <= 0) return;
  const int nbp = (a.b1 - a.b0 + 1) / 2, nct = a.ncol_tiles;
  const int ncx = nct >= N_XCD ? (nct + N_XCD - 1) / N_XCD : 0;
  // at most 32768 bra pairs x (ncol / 128 + 8) slices: well inside the grid limit
  const int64_t grid = ncx ? (int64_t)N_XCD * ncx * nbp : (int64_t)nbp * nct;
  hipLaunchKernelGGL(k_first_half<FH_KH>, dim3((unsigned)grid), dim3(256), 0, s, a, nbp, nct, ncx);
}

// ---------------------------------------------------------------------------
// batched GEMM (64 x 64 tile, K step 16, four 32 x 32 wave tiles)
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

__global__ void __launch_bounds__(256) k_dgemm_batched(int transA, int M, int N, int K,
                                                       double alpha, const double *A,
                                                       int64_t lda, int64_t sA, const double *B,
                                                       int64_t ldb, int64_t sB, double beta,
                                                       double *C, int64_t ldc, int64_t sC) {
  __shared__ double As[GB_K][GB_M + 2];
  __shared__ double Bs[GB_K][GB_N + 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.x * GB_M, n0 = blockIdx.y * GB_N;
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += GB_K) {
    if (!transA) {  // A[m][k]: thread -> (m = tid/4, 4 consecutive k)
      int m = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + m, gk = k0 + kq + i;
        As[kq + i][m] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : 0.0;
      }
    } else {  // A[k][m]: thread -> (k = tid/16, 4 consecutive m)
      int k = tid >> 4, mq = (tid & 15) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + mq + i, gk = k0 + k;
        As[k][mq + i] = (gm < M && gk < K) ? A[(int64_t)gk * lda + gm] : 0.0;
      }
    }
    {
      int k = tid >> 4, nq = (tid & 15) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gn = n0 + nq + i, gk = k0 + k;
        Bs[k][nq + i] = (gn < N && gk < K) ? B[(int64_t)gk * ldb + gn] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GB_K / 4; ++kk) {
      int k = kk * 4 + lk;
      double av[2], bv[2];
      for (int r = 0; r < 2; ++r) av[r] = As[k][wr + r * 16 + lr];
      for (int c = 0; c < 2; ++c) bv[c] = Bs[k][wc + c * 16 + lr];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + wr + r * 16 + lk + 4 * i, gn = n0 + wc + c * 16 + lr;
        if (gm < M && gn < N) {
          double *p = C + (int64_t)gm * ldc + gn;
          double v = alpha * acc[r][c][i];
          *p = beta == 0.0 ? v : v + beta * *p;
        }
      }
}

void launch_dgemm_batched(int transA, int M, int N, int K, double alpha, const double *A,
                          int64_t lda, int64_t strideA, const double *B, int64_t ldb,
                          int64_t strideB, double beta, double *C, int64_t ldc, int64_t strideC,
                          int batch, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  dim3 grid((M + GB_M - 1) / GB_M, (N + GB_N - 1) / GB_N, batch);
  hipLaunchKernelGGL(k_dgemm_batched, grid, dim3(256), 0, s, transA, M, N, K, alpha, A, lda,
                     strideA, B, ldb, strideB, beta, C, ldc, strideC);
}

}  // namespace qdcb
