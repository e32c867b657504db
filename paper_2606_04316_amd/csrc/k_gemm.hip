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
// a ket tile kept for only one of the two bra tiles contributes zeros to the
// other half and that half's wavefronts skip its MFMAs.  Four wavefronts hold
// 64 x 64 accumulator blocks (16 MFMA tiles each).  Per staged step of 32 ket
// rows the workgroup reads 32 KB of integral tile and 32 KB of density slice
// for 2 x 128 x 128 x 32 flops.
constexpr int FH_COLS = 128;       // columns per workgroup
constexpr int FH_ROWS = 2 * TILE;  // bra rows per workgroup
constexpr int FH_KH = 32;          // ket rows staged per step
constexpr int AS_LD = FH_ROWS + 2; // LDS row strides (padded against bank conflicts)
constexpr int BS_LD = FH_COLS + 2;

__global__ void __launch_bounds__(256) k_first_half(FirstHalfArgs a) {
  __shared__ double As[FH_KH * AS_LD];
  __shared__ double Bs[FH_KH * BS_LD];
  if (a.overflow && *a.overflow) return;  // uniform: the task lists did not fit
  // bra-tile pairs vary fastest: workgroups in flight share the column slice
  // and, through the ordered ket lists of neighbouring bra tiles, density rows
  const int bt0 = a.b0 + 2 * blockIdx.x;
  const bool two = bt0 + 1 < a.b1;
  const int ct = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;  // wave's 64-row half (bra tile) and 64-column half
  const int64_t c0 = (int64_t)ct * FH_COLS;
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 acc[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};

  const int64_t s0 = a.slot_base[bt0], s1 = two ? a.slot_base[bt0 + 1] : 0;
  const int n0 = a.count[bt0], n1 = two ? a.count[bt0 + 1] : 0;
  int i0 = 0, i1 = 0;
  while (i0 < n0 || i1 < n1) {
    const int k0 = i0 < n0 ? a.tasks[s0 + i0] : INT_MAX;
    const int k1 = i1 < n1 ? a.tasks[s1 + i1] : INT_MAX;
    const int kt = k0 < k1 ? k0 : k1;
    const bool has0 = k0 == kt, has1 = k1 == kt;
    const double *P0 = has0 ? a.panel + (s0 + i0 - a.slot0) * (TILE * TILE) : nullptr;
    const double *P1 = has1 ? a.panel + (s1 + i1 - a.slot0) * (TILE * TILE) : nullptr;
    i0 += has0;
    i1 += has1;
    const bool active = wr == 0 ? has0 : has1;  // uniform per wavefront
    for (int h = 0; h < TILE / FH_KH; ++h) {
      // integral slice: ket rows j of this step x 128 bra rows (two tiles)
#pragma unroll
      for (int i = 0; i < (FH_KH * FH_ROWS / 2) / 256; ++i) {
        const int e = tid + 256 * i;  // double2 index
        const int jj = e / (FH_ROWS / 2), m2 = e % (FH_ROWS / 2);
        const int half = m2 >= TILE / 2;
        const double *P = half ? P1 : P0;
        double2 v = make_double2(0.0, 0.0);
        if (P) v = reinterpret_cast<const double2 *>(P + (h * FH_KH + jj) * TILE)[m2 - half * (TILE / 2)];
        *reinterpret_cast<double2 *>(As + jj * AS_LD + 2 * m2) = v;
      }
      const int64_t krow0 = (int64_t)kt * TILE + h * FH_KH;
#pragma unroll
      for (int i = 0; i < (FH_KH * FH_COLS / 2) / 256; ++i) {
        const int e = tid + 256 * i;
        const int r = e / (FH_COLS / 2), c2 = e % (FH_COLS / 2);
        const double2 v = reinterpret_cast<const double2 *>(a.D + (krow0 + r) * a.ld + c0)[c2];
        *reinterpret_cast<double2 *>(Bs + r * BS_LD + 2 * c2) = v;
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int kk = 0; kk < FH_KH / 4; ++kk) {
          const int j = kk * 4 + lk;
          double av[4], bv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) av[r] = As[j * AS_LD + wr * 64 + r * 16 + lr];
#pragma unroll
          for (int c = 0; c < 4; ++c) bv[c] = Bs[j * BS_LD + wc * 64 + c * 16 + lr];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
        }
      }
      __syncthreads();
    }
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
  hipLaunchKernelGGL(k_first_half, dim3((a.b1 - a.b0 + 1) / 2, a.ncol_tiles), dim3(256), 0, s, a);
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
