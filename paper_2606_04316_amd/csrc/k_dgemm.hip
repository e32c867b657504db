// k_dgemm.hip -- FP64 MFMA GEMMs for the second-half quarter transforms
// (Sec. 2.4.2): the gathered first quarter (k_gather_gemm) and a plain
// batched GEMM (k_dgemm_batched).
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
                                                       double *C, int64_t ldc, int64_t sC,
                                                       int tri_n) {
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
  // triangle (tri_n > 0, a multiple of 16): row m is (x, p) = (m / tri_n,
  // m % tri_n) and column n is q; 16 x 16 blocks whose every p exceeds every
  // q are neither computed nor stored
  unsigned skip = 0;
  if (tri_n > 0)
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        if ((m0 + wr + r * 16) % tri_n >= n0 + wc + c * 16 + 16) skip |= 1u << (r * 2 + c);
  dbl4 acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += GB_K) {
    // staging: lane l of each wave takes column l of its k rows, so that the
    // 64 lanes of a wave write 64 consecutive doubles of one LDS row (no bank
    // conflicts) and read consecutive m (op(A) = A^T) and n columns
    const int col = tid & 63, kr = tid >> 6;
#pragma unroll
    for (int i = 0; i < GB_K / 4; ++i) {
      const int k = kr + 4 * i, gk = k0 + k;
      const int gm = m0 + col, gn = n0 + col;
      As[k][col] = (gm < M && gk < K)
                       ? (transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk])
                       : 0.0;
      Bs[k][col] = (gn < N && gk < K) ? B[(int64_t)gk * ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GB_K / 4; ++kk) {
      int k = kk * 4 + lk;
      double av[2], bv[2];
      for (int r = 0; r < 2; ++r) av[r] = As[k][wr + r * 16 + lr];
      for (int c = 0; c < 2; ++c) bv[c] = Bs[k][wc + c * 16 + lr];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
          if (!(skip >> (r * 2 + c) & 1u)) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + wr + r * 16 + lk + 4 * i, gn = n0 + wc + c * 16 + lr;
        if (gm < M && gn < N && !(skip >> (r * 2 + c) & 1u)) {
          double *p = C + (int64_t)gm * ldc + gn;
          double v = alpha * acc[r][c][i];
          *p = beta == 0.0 ? v : v + beta * *p;
        }
      }
}

void launch_dgemm_batched(int transA, int M, int N, int K, double alpha, const double *A,
                          int64_t lda, int64_t strideA, const double *B, int64_t ldb,
                          int64_t strideB, double beta, double *C, int64_t ldc, int64_t strideC,
                          int batch, hipStream_t s, int tri_n) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  dim3 grid((M + GB_M - 1) / GB_M, (N + GB_N - 1) / GB_N, batch);
  hipLaunchKernelGGL(k_dgemm_batched, grid, dim3(256), 0, s, transA, M, N, K, alpha, A, lda,
                     strideA, B, ldb, strideB, beta, C, ldc, strideC, tri_n);
}

// ---------------------------------------------------------------------------
// Gathered GEMM.  Workgroup: 128 slice columns (c) x 128 output columns (j)
// of one batch, four wavefronts of 64 x 64.  Steps of 16 k rows; each row of
// the A^T tile (128 consecutive V columns of row rowmap[b, k]) and of the B
// tile (128 consecutive B columns) is one wavefront instruction of 16-byte
// direct global->LDS loads, double-buffered so that the loads of step t+1
// run under step t's MFMAs.  Rows k >= K are zero-filled; lanes past the V
// row or past J load nothing (they only feed outputs that are not stored).
// Two workgroups per compute unit (the register budget is held to that).
//
// Workgroup order: the chip's 8 XCDs take workgroups round-robin; workgroup
// L runs on XCD L % 8, whose consecutive workgroups cover the tiles of one
// sharing group (the tiles that read the same A or B tile), so that the
// shared tile is fetched into that XCD's L2 once.
constexpr int GG_KH = 16;
constexpr int GG_LD = 130;  // LDS row stride (doubles): 16-byte rows, padded

typedef __attribute__((address_space(3))) void *gg_lds_ptr;

__device__ __forceinline__ void gg_mfma(const double *A, const double *B, int wr, int wc, int lr,
                                        int lk, unsigned skip, dbl4 (&acc)[4][4]) {
#pragma unroll
  for (int kk = 0; kk < GG_KH / 4; ++kk) {
    const int j = kk * 4 + lk;
    double av[4], bv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = A[j * GG_LD + wr * 64 + r * 16 + lr];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = B[j * GG_LD + wc * 64 + c * 16 + lr];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (!(skip >> (r * 4 + c) & 1u)) acc[r][c] = MFMA_F64(av[r], bv[c], acc[r][c]);
  }
}

constexpr int GG_XCD = 8;

__global__ void __launch_bounds__(256, 2) k_gather_gemm(GatherGemmArgs a, int nct, int njt) {
  __shared__ __attribute__((aligned(16))) double As0[GG_KH * GG_LD], As1[GG_KH * GG_LD];
  __shared__ __attribute__((aligned(16))) double Bs0[GG_KH * GG_LD], Bs1[GG_KH * GG_LD];
  int ct, jt, b;
  {
    const int L = blockIdx.x, loc = L / GG_XCD;
    const int inner = a.share_b ? nct : njt;  // tiles of one sharing group
    const int64_t g = (int64_t)GG_XCD * (loc / inner) + L % GG_XCD;
    const int t = loc % inner;
    if (a.share_b) {  // group (jt, b)
      if (g >= (int64_t)njt * a.nb) return;  // uniform: ragged last groups
      ct = t;
      jt = (int)(g % njt);
      b = (int)(g / njt);
    } else {  // group (ct, b)
      if (g >= (int64_t)nct * a.nb) return;
      jt = t;
      ct = (int)(g % nct);
      b = (int)(g / nct);
    }
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;
  const int lr = lane & 15, lk = lane >> 4;
  // triangle: skip[r][c] for this wave's 16 x 16 blocks (p of every row above
  // q of every column); a workgroup whose blocks are all skipped exits
  unsigned skip = 0;
  if (a.tri_n > 0) {
    const int qw = jt * 128 + wc * 64;
    for (int r = 0; r < 4; ++r) {
      // first p of block r (a 16-row block never spans two x: 16 divides tri_n)
      const int pr = (int)(((int64_t)ct * 128 + wr * 64 + r * 16) % a.tri_n);
      for (int c = 0; c < 4; ++c)
        if (pr >= qw + c * 16 + 16) skip |= 1u << (r * 4 + c);
    }
    const int pg = (int)(((int64_t)ct * 128) % a.tri_n);
    if (pg + 128 <= a.tri_n && pg >= jt * 128 + 128) return;  // uniform: every p > every q
  }
  const int64_t c0 = (int64_t)ct * 128 + 2 * lane;  // this lane's two columns
  const int j0 = jt * 128 + 2 * lane;
  const bool c_ok = a.col0 + c0 + 1 < a.ld;
  const bool j_ok = j0 + 1 < a.J;
  dbl4 acc[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) acc[r][c] = (dbl4){0.0, 0.0, 0.0, 0.0};
  const int nsteps = (a.K + GG_KH - 1) / GG_KH;
  // V rows of this wave's k rows, read one step ahead of their loads so that
  // the only memory waits are the ones at the step barriers
  int nrow[GG_KH / 4];
  auto fetch_rows = [&](int t) {
#pragma unroll
    for (int q = 0; q < GG_KH / 4; ++q) {
      const int k = t * GG_KH + w + 4 * q;
      nrow[q] = k >= a.K ? 0 : a.rowmap ? a.rowmap[(int64_t)b * a.sb + (int64_t)k * a.sk] : k;
    }
  };
  auto issue = [&](int t, double *A, double *B) {
#pragma unroll
    for (int q = 0; q < GG_KH / 4; ++q) {
      const int kk = w + 4 * q, k = t * GG_KH + kk;
      if (k < a.K) {
        const int64_t row = __builtin_amdgcn_readfirstlane(nrow[q]);
        if (c_ok)
          __builtin_amdgcn_global_load_lds(a.V + row * a.ld + a.col0 + c0,
                                           (gg_lds_ptr)(A + kk * GG_LD), 16, 0, 0);
        if (j_ok)
          __builtin_amdgcn_global_load_lds(a.B + (int64_t)b * a.sbB + (int64_t)k * a.ldb + j0,
                                           (gg_lds_ptr)(B + kk * GG_LD), 16, 0, 0);
      } else {
        *reinterpret_cast<double2 *>(A + kk * GG_LD + 2 * lane) = make_double2(0.0, 0.0);
        *reinterpret_cast<double2 *>(B + kk * GG_LD + 2 * lane) = make_double2(0.0, 0.0);
      }
    }
  };
  auto mfma = [&](const double *A, const double *B) { gg_mfma(A, B, wr, wc, lr, lk, skip, acc); };
  fetch_rows(0);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  bool more = nsteps > 0;
  if (more) issue(0, As0, Bs0);
  fetch_rows(1);
  int t = 0;  // step staged in the buffer about to be read
  while (more) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // this wave's loads of step t done
    __syncthreads();                     // ... and every wave's; buffer 1 free
    more = t + 1 < nsteps;
    if (more) {
      issue(t + 1, As1, Bs1);
      fetch_rows(t + 2);
    }
    mfma(As0, Bs0);
    ++t;
    if (more) {
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
      more = t + 1 < nsteps;
      if (more) {
        issue(t + 1, As0, Bs0);
        fetch_rows(t + 2);
      }
      mfma(As1, Bs1);
      ++t;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t cc = (int64_t)ct * 128 + wr * 64 + r * 16 + lk + 4 * i;
        const int jj = jt * 128 + wc * 64 + c * 16 + lr;
        if (cc < a.nc && jj < a.J && !(skip >> (r * 4 + c) & 1u)) {
          double *o = a.C + cc * a.ldc_c + (int64_t)b * a.ldc_b + jj;
          *o = a.accumulate ? *o + acc[r][c][i] : acc[r][c][i];
        }
      }
}

void launch_gather_gemm(const GatherGemmArgs &a, hipStream_t s) {
  if (a.nc <= 0 || a.J <= 0 || a.nb <= 0) return;
  const int nct = (a.nc + 127) / 128, njt = (a.J + 127) / 128;
  const int inner = a.share_b ? nct : njt;
  const int64_t groups = (int64_t)(a.share_b ? njt : nct) * a.nb;
  // at most (65532 / 128) x 32 x 2^16 tiles: inside the grid limit
  const int64_t grid = (int64_t)GG_XCD * inner * ((groups + GG_XCD - 1) / GG_XCD);
  hipLaunchKernelGGL(k_gather_gemm, dim3((unsigned)grid), dim3(256), 0, s, a, nct, njt);
}

}  // namespace qdcb
