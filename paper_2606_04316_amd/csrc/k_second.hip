// k_second.hip -- second-half helpers (Sec. 2.4.2, Eq. secondhalf).
//
// The half-transformed V[mn][(rs, y)] is real and symmetric in (m, n) for
// every column, so G_{pq} = sum_mn conj(C_mp) V_mn C_nq is done per column as
// two real GEMMs on quaternion planes:
//   W[m][(z, q)]  = sum_n V[m][n] C_z[n][q]                 (4 planes at once)
//   G[(x, p)][q]  = sum_(m, z) Chat[(m, z)][(x, p)] W[(m, z)][q]
// where Chat holds the signed components of conj(C_mp) that multiply W_z in
// component x of the quaternion product.  These kernels build Chat, unpack V
// column slices into dense matrices and scatter the result into G.
#include "kernels.h"

namespace qdcb {

__global__ void k_build_coef_mats(int N, int n, const double *C, double *Call, double *Chat) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * n) return;
  int mu = (int)(t / n), p = (int)(t % n);
  double a0 = C[((int64_t)0 * N + mu) * n + p];
  double a1 = C[((int64_t)1 * N + mu) * n + p];
  double a2 = C[((int64_t)2 * N + mu) * n + p];
  double a3 = C[((int64_t)3 * N + mu) * n + p];
  Call[(int64_t)mu * 4 * n + 0 * n + p] = a0;
  Call[(int64_t)mu * 4 * n + 1 * n + p] = a1;
  Call[(int64_t)mu * 4 * n + 2 * n + p] = a2;
  Call[(int64_t)mu * 4 * n + 3 * n + p] = a3;
  // [conj(a) w]_x = sum_z coef[x][z] w_z
  const double coef[4][4] = {{a0, a1, a2, a3},
                             {-a1, a0, a3, -a2},
                             {-a2, -a3, a0, a1},
                             {-a3, a2, -a1, a0}};
  for (int z = 0; z < 4; ++z)
    for (int x = 0; x < 4; ++x)
      Chat[((int64_t)mu * 4 + z) * 4 * n + x * n + p] = coef[x][z];
}

void launch_build_coef_mats(int N, int n, const double *C, double *Call, double *Chat,
                            hipStream_t s) {
  int64_t tot = (int64_t)N * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_build_coef_mats, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N,
                     n, C, Call, Chat);
}

// LDS transpose: 64 (nu) x 64 (columns) per workgroup, fixed mu.
__global__ void __launch_bounds__(256) k_unpack(int N, const int32_t *rowmap, const double *V,
                                                int64_t ld, int64_t c0, int nc, double *Vfull) {
  __shared__ double tile[64][65];
  const int nu0 = blockIdx.x * 64, mu = blockIdx.y, cb = blockIdx.z * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    int nl = e >> 6, cl = e & 63;
    int nu = nu0 + nl, c = cb + cl;
    double v = 0.0;
    if (nu < N && c < nc) v = V[(int64_t)rowmap[(int64_t)mu * N + nu] * ld + c0 + c];
    tile[nl][cl] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    int cl = e >> 6, nl = e & 63;
    int nu = nu0 + nl, c = cb + cl;
    if (nu < N && c < nc) Vfull[((int64_t)c * N + mu) * N + nu] = tile[nl][cl];
  }
}

void launch_unpack(int N, const int32_t *rowmap, const double *V, int64_t ld, int64_t c0, int nc,
                   double *Vfull, hipStream_t s) {
  if (N <= 0 || nc <= 0) return;
  dim3 grid((N + 63) / 64, N, (nc + 63) / 64);
  hipLaunchKernelGGL(k_unpack, grid, dim3(256), 0, s, N, rowmap, V, ld, c0, nc, Vfull);
}

// One thread per (MO pair r <= s of the chunk, p, q): 16 contiguous outputs.
__global__ void k_pack(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc,
                       double *G) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nidx = nc / 4;
  if (t >= nidx * n * n) return;
  int q = (int)(t % n);
  int p = (int)((t / n) % n);
  int64_t il = t / ((int64_t)n * n);
  int64_t idx = c0 / 4 + il;
  int rsv = rs[idx];
  int r = rsv & 0xffff, s = rsv >> 16;
  double v[4][4];
  for (int y = 0; y < 4; ++y)
    for (int x = 0; x < 4; ++x)
      v[x][y] = Gc[((il * 4 + y) * 4 * n + (int64_t)x * n + p) * n + q];
  double *o = G + ((((int64_t)p * n + q) * n + r) * n + s) * 16;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; y += 2)
      reinterpret_cast<double2 *>(o + x * 4 + y)[0] = make_double2(v[x][y], v[x][y + 1]);
  if (r != s) {
    double *m = G + ((((int64_t)p * n + q) * n + s) * n + r) * 16;
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; y += 2)
        reinterpret_cast<double2 *>(m + x * 4 + y)[0] =
            make_double2(y == 0 ? v[x][0] : -v[x][y], -v[x][y + 1]);
  }
}

void launch_pack(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc, double *G,
                 hipStream_t s) {
  int64_t tot = (int64_t)(nc / 4) * n * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rs, c0, nc,
                     Gc, G);
}

}  // namespace qdcb
