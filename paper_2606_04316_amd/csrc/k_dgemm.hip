// k_dgemm.hip -- batched FP64 MFMA GEMM for the second-half quarter
// transforms (Sec. 2.4.2).
//
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element i of lane l is D[l/16 + 4*i][l%16].
#include "kernels.h"

namespace qdcb {

#define MFMA_F64(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

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
