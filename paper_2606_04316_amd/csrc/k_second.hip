// k_second.hip -- second-half helpers (Sec. 2.4.2, Eq. secondhalf).
//
// The half-transformed V[mn][(rs, y)] is a real N_A x N_B matrix for every
// column, so G_pq = sum_mn a_mp V_mn b_nq (a, b quaternion coefficient rows)
// is done per column as two real GEMMs on quaternion planes:
//   W[m][(z, q)]  = sum_n V[m][n] b_z[n][q]                 (4 planes at once)
//   G[(x, p)][q]  = sum_(m, z) Chat[(m, z)][(x, p)] W[(m, z)][q]
// where Chat holds the left-multiplication matrix of a_mp.  Coulomb uses
// a = conj(C), b = C; the Gaunt chains use a = conj(C^L) e_K, b = C^S and
// a = conj(C^S) e_K, b = C^L (Eq. GauntInt).  The first product reads the
// rows of V directly (k_dgemm.hip, gathered GEMM); these kernels build Chat
// and scatter the result into G.
#include "kernels.h"

namespace qdcb {

__global__ void k_build_coef_mats(int N, int n, const double *C, int unit, double *Call,
                                  double *Chat) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * n) return;
  int mu = (int)(t / n), p = (int)(t % n);
  double c[4];
  for (int z = 0; z < 4; ++z) {
    c[z] = C[((int64_t)z * N + mu) * n + p];
    Call[(int64_t)mu * 4 * n + z * n + p] = c[z];
  }
  // a = conj(c) * e
  double a0 = c[0], a1 = -c[1], a2 = -c[2], a3 = -c[3];
  double q0 = a0, q1 = a1, q2 = a2, q3 = a3;
  if (unit == 2) {  // * i
    q0 = -a1; q1 = a0; q2 = a3; q3 = -a2;
  } else if (unit == 1) {  // * j
    q0 = -a2; q1 = -a3; q2 = a0; q3 = a1;
  } else if (unit == 0) {  // * k
    q0 = -a3; q1 = a2; q2 = -a1; q3 = a0;
  }
  // left multiplication: (q w)_x = sum_z L[x][z] w_z
  const double L[4][4] = {{q0, -q1, -q2, -q3},
                          {q1, q0, -q3, q2},
                          {q2, q3, q0, -q1},
                          {q3, -q2, q1, q0}};
  for (int z = 0; z < 4; ++z)
    for (int x = 0; x < 4; ++x) Chat[((int64_t)mu * 4 + z) * 4 * n + x * n + p] = L[x][z];
}

void launch_build_coef_mats(int N, int n, const double *C, int unit, double *Call,
                            double *Chat, hipStream_t s) {
  int64_t tot = (int64_t)N * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_build_coef_mats, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N,
                     n, C, unit, Call, Chat);
}

// G_pq^x of slice column il * 4 + y (s_0 = +1, s_1,2,3 = -1).
//   Coulomb (mirror = +1): Gc holds G_pq for p <= q; for p > q the bra-pair
//     rule G_pq^x = s_x G_qp^x (the symmetric V of an unordered pair).
//   Gaunt (mirror = -1): Gc holds T_pq, the term of the bra density
//     conj(C^L_mu p) e_K C^S_nu q, for every (p, q).  The other term,
//     conj(C^S_nu p) e_K C^L_mu q, is minus the conjugate of the first one at
//     (q, p), so G_pq^x = T_pq^x - s_x T_qp^x.
__device__ __forceinline__ double gc_entry(const double *Gc, int n, int64_t il, int y, int x,
                                           int p, int q, double mirror) {
  const double *P = Gc + (il * 4 + y) * 4 * n * (int64_t)n + (int64_t)x * n * n;
  const double sx = x == 0 ? 1.0 : -1.0;
  if (mirror > 0) return p <= q ? P[(int64_t)p * n + q] : sx * P[(int64_t)q * n + p];
  return P[(int64_t)p * n + q] - sx * P[(int64_t)q * n + p];
}

// One thread per (MO pair r <= s of the slice, p, q): 16 contiguous outputs.
__global__ void k_pack(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc,
                       double *G, double mirror, int accumulate) {
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
    for (int x = 0; x < 4; ++x) v[x][y] = gc_entry(Gc, n, il, y, x, p, q, mirror);
  double *o = G + ((((int64_t)p * n + q) * n + r) * n + s) * 16;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; y += 2) {
      double2 *d = reinterpret_cast<double2 *>(o + x * 4 + y);
      double2 w = make_double2(v[x][y], v[x][y + 1]);
      if (accumulate) {
        double2 old = d[0];
        w.x += old.x;
        w.y += old.y;
      }
      d[0] = w;
    }
  if (r != s) {
    double *m = G + ((((int64_t)p * n + q) * n + s) * n + r) * 16;
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; y += 2) {
        double2 *d = reinterpret_cast<double2 *>(m + x * 4 + y);
        // s_y = +1 for y = 0, -1 otherwise
        double2 w = make_double2(mirror * (y == 0 ? v[x][0] : -v[x][y]), -mirror * v[x][y + 1]);
        if (accumulate) {
          double2 old = d[0];
          w.x += old.x;
          w.y += old.y;
        }
        d[0] = w;
      }
  }
}

// General two-spinor mode (planes alpha re, alpha im, beta re, beta im).
__global__ void k_build_spinor_mats(int N, int n, const double *C, int K, double *Call,
                                    double *Chat) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * n) return;
  int mu = (int)(t / n), p = (int)(t % n);
  double c[4];
  for (int z = 0; z < 4; ++z) c[z] = C[((int64_t)z * N + mu) * n + p];
  double *o = Call + (int64_t)mu * 4 * n + p;
  if (K < 0) {
    for (int z = 0; z < 4; ++z) o[z * n] = c[z];
    // re: sum_tau c_re W_re + c_im W_im;  im: sum_tau c_re W_im - c_im W_re
    const double L[4][4] = {{c[0], c[1], c[2], c[3]},
                            {-c[1], c[0], -c[3], c[2]},
                            {0.0, 0.0, 0.0, 0.0},
                            {0.0, 0.0, 0.0, 0.0}};
    for (int z = 0; z < 4; ++z)
      for (int x = 0; x < 4; ++x) Chat[((int64_t)mu * 4 + z) * 4 * n + x * n + p] = L[x][z];
    return;
  }
  // -sigma_K c: sigma_x (b, a); sigma_y (-i b, i a); sigma_z (a, -b)
  double s[4];
  if (K == 0) {
    s[0] = c[2]; s[1] = c[3]; s[2] = c[0]; s[3] = c[1];
  } else if (K == 1) {
    s[0] = c[3]; s[1] = -c[2]; s[2] = -c[1]; s[3] = c[0];
  } else {
    s[0] = c[0]; s[1] = c[1]; s[2] = -c[2]; s[3] = -c[3];
  }
  for (int z = 0; z < 4; ++z) o[z * n] = -s[z];
}

void launch_build_spinor_mats(int N, int n, const double *C, int K, double *Call, double *Chat,
                              hipStream_t s) {
  int64_t tot = (int64_t)N * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_build_spinor_mats, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     N, n, C, K, Call, Chat);
}

// One thread per (spinor pair of the slice, p, q).
__global__ void k_pack_spinor(int n, const int32_t *rs, int nspair, int64_t c0, int nc,
                              const double *Gc, double *G, int accumulate) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npl = nc / 2;  // spinor pairs of the slice
  if (t >= npl * n * n) return;
  int q = (int)(t % n);
  int p = (int)((t / n) % n);
  int64_t jl = t / ((int64_t)n * n);  // pair within the slice
  int64_t i = c0 / 2 + jl;            // global spinor pair
  if (i >= nspair) return;            // empty half of the last group
  const int rsv = rs[i];
  const int c = rsv & 0xffff, d = rsv >> 16;
  // planes x = 0 (re), 1 (im) of the columns of V re (2 jl) and V im (2 jl + 1)
  const double *A = Gc + (2 * jl) * 4 * (int64_t)n * n;
  const double *B = A + 4 * (int64_t)n * n;
  const int64_t pq = (int64_t)p * n + q;
  const double ar = A[pq], ai = A[(int64_t)n * n + pq];
  const double br = B[pq], bi = B[(int64_t)n * n + pq];
  double *o = G + ((pq * n + c) * n + d) * 2;
  double2 v = make_double2(ar - bi, ai + br);
  if (accumulate) {
    const double2 old = *reinterpret_cast<double2 *>(o);
    v.x += old.x;
    v.y += old.y;
  }
  *reinterpret_cast<double2 *>(o) = v;
  if (c != d) {
    double *m = G + ((pq * n + d) * n + c) * 2;
    double2 w = make_double2(ar + bi, ai - br);
    if (accumulate) {
      const double2 old = *reinterpret_cast<double2 *>(m);
      w.x += old.x;
      w.y += old.y;
    }
    *reinterpret_cast<double2 *>(m) = w;
  }
}

void launch_pack_spinor(int n, const int32_t *rs, int nspair, int64_t c0, int nc,
                        const double *Gc, double *G, int accumulate, hipStream_t s) {
  int64_t tot = (int64_t)(nc / 2) * n * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_pack_spinor, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rs,
                     nspair, c0, nc, Gc, G, accumulate);
}

// Block output: one thread per (MO pair r <= s of the slice, p, q) writes
// B[i][p][q][0][x][y] = G_pqrs^xy and B[i][p][q][1][x][y] = G_pqsr^xy (the same
// entry when r = s), i the pair's index in the block (first pair b_i0).
__global__ void k_pack_block(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc,
                             double *B, int64_t b_i0, double mirror, int accumulate) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nidx = nc / 4;
  if (t >= nidx * n * n) return;
  int q = (int)(t % n);
  int p = (int)((t / n) % n);
  int64_t il = t / ((int64_t)n * n);
  const int rsv = rs[c0 / 4 + il];
  const bool diag = (rsv & 0xffff) == (rsv >> 16);
  int64_t i = c0 / 4 + il - b_i0;
  double *o = B + ((i * n + p) * n + q) * 32;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) {
      const double v = gc_entry(Gc, n, il, y, x, p, q, mirror);
      // s_y = +1 for y = 0, -1 otherwise
      const double m = diag ? v : mirror * (y == 0 ? v : -v);
      o[x * 4 + y] = accumulate ? o[x * 4 + y] + v : v;
      o[16 + x * 4 + y] = accumulate ? o[16 + x * 4 + y] + m : m;
    }
}

void launch_pack_block(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc,
                       double *B, int64_t b_i0, double mirror, int accumulate, hipStream_t s) {
  int64_t tot = (int64_t)(nc / 4) * n * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_pack_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rs,
                     c0, nc, Gc, B, b_i0, mirror, accumulate);
}

void launch_pack(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc, double *G,
                 double mirror, int accumulate, hipStream_t s) {
  int64_t tot = (int64_t)(nc / 4) * n * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rs, c0, nc,
                     Gc, G, mirror, accumulate);
}

}  // namespace qdcb
