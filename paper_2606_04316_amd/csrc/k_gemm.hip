// k_gemm.hip -- FP64 MFMA contractions.
//
// k_first_half: the first-half integral-density contraction of Eq.
// (firsthalf), V[mn][col] = sum over kept ket tiles of I[mn][kl] D~[kl][col],
// a block-sparse GEMM whose A blocks are the masked integral tiles and whose
// B rows are the symmetrized quaternion pair densities.  One workgroup owns a
// 64-row bra tile and a 128-column slice and accumulates over that bra
// tile's kept ket tiles in registers, so V is written once and no atomics are
// used (the result is deterministic).
//
// k_dgemm_batched: plain batched GEMM for the second-half quarter
// transforms (Sec. 2.4.2).
//
// Both use v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element i of lane l is D[l/16 + 4*i][l%16].
#include "kernels.h"

namespace qdcb {

#define MFMA_F64(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

constexpr int FH_COLS = 128;  // columns per workgroup
constexpr int FH_KH = 32;     // ket rows staged per step
constexpr int AS_LD = 64;     // LDS row stride of the integral slice [j][m]
constexpr int BS_LD = 128;    // LDS row stride of the density slice [j][col]

__global__ void __launch_bounds__(256) k_first_half(FirstHalfArgs a) {
  __shared__ double As[FH_KH * AS_LD];
  __shared__ double Bs[FH_KH * BS_LD];
  // bra tiles vary fastest: workgroups in flight share the column slice and,
  // through the ordered ket lists of neighbouring bra tiles, the density rows
  const int bt = a.b0 + blockIdx.x;
  const int ct = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t c0 = (int64_t)ct * FH_COLS;
  dbl4 acc[4][2];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};

  const int64_t s0 = a.slot_base[bt];
  const int ntask = a.count[bt];
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = 0; t < ntask; ++t) {
    const int64_t slot = s0 + t;
    const int kt = a.tasks[slot];
    const double *P = a.panel + (slot - a.slot0) * (TILE * TILE);
    for (int h = 0; h < TILE / FH_KH; ++h) {
      // stage integral rows j in [h*32, h*32+32) (x 64 bra) and density rows
      {
        const double2 *src = reinterpret_cast<const double2 *>(P + h * FH_KH * TILE);
        double2 *dst = reinterpret_cast<double2 *>(As);
#pragma unroll
        for (int i = 0; i < (FH_KH * TILE / 2) / 256; ++i) dst[tid + 256 * i] = src[tid + 256 * i];
      }
      {
        const int64_t krow0 = (int64_t)kt * TILE + h * FH_KH;
#pragma unroll
        for (int i = 0; i < (FH_KH * FH_COLS / 2) / 256; ++i) {
          int e = tid + 256 * i;         // double2 index
          int r = e / (FH_COLS / 2), c2 = e % (FH_COLS / 2);
          const double2 *src =
              reinterpret_cast<const double2 *>(a.D + (krow0 + r) * a.ld + c0) + c2;
          reinterpret_cast<double2 *>(Bs + r * BS_LD)[c2] = *src;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < FH_KH / 4; ++kk) {
        const int j = kk * 4 + lk;
        double av[4], bv[2];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = As[j * AS_LD + r * 16 + lr];
#pragma unroll
        for (int c = 0; c < 2; ++c) bv[c] = Bs[j * BS_LD + w * 32 + c * 16 + lr];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
      }
      __syncthreads();
    }
  }
  const int64_t row0 = (int64_t)bt * TILE;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int64_t row = row0 + r * 16 + lk + 4 * i;
        a.V[row * a.ld + c0 + w * 32 + c * 16 + lr] = acc[r][c][i];
      }
}

void launch_first_half(const FirstHalfArgs &a, hipStream_t s) {
  if (a.b1 <= a.b0 || a.ncol_tiles <= 0) return;
  hipLaunchKernelGGL(k_first_half, dim3(a.b1 - a.b0, a.ncol_tiles), dim3(256), 0, s, a);
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
