// k_density.hip -- quaternion MO-pair densities and their infinity-norm bound.
//
// Coulomb classes (LL, SS rows).  For an AO pair (ka, la) and MO pair r <= s
// the quaternion pair density is D^{rs}_{ka la} = conj(C_ka r) C_la s, the
// Kramers-paired form of Eqs. (Den) and (QuaternionScatter): its four real
// components are the four Pauli-scalar densities of the Kramers block.  The AO
// integral is symmetric in ka <-> la, so the first half contracts with
//   D~ = D_{ka la} + D_{la ka}   (ka != la),   D_{ka ka}   (ka = la).
// Dmax_{ka la} is the largest |component| of D over all ordered MO pairs
// (r, t), the ||D~||_inf of Eq. (SchwarzDen); the r <= s loop covers it
// because conj(D^{rt}_{ka la}) = D^{tr}_{la ka}.
//
// Gaunt class (LS rows, ka in L, la in S).  The density of the Gaunt term
// -alpha_1.alpha_2/r12 (Eqs. breit, GauntInt) for Pauli component K is
//   D^{K,rs}_{ka la} = conj(C^L_ka r) e_K C^S_la s + conj(C^S_la r) e_K C^L_ka s,
// e_x = k, e_y = j, e_z = i (sigma_K = -i Q(e_K)).  D^{K,sr} = -conj(D^{K,rs}),
// so r <= s again covers every ordered pair for Dmax.
//
// One workgroup per pair row; the coefficient rows are staged in LDS, threads
// stride over MO pairs and write 32 contiguous bytes each; a block reduction
// forms Dmax.  Bound-only launches compute Dmax over a range of MO pairs (all of
// them for the AO-driven transform, one batch for the MO-driven one) without
// writing D; write launches fill the columns of MO pairs [i0, i1).
#include "kernels.h"

namespace qdcb {

constexpr int DENS_THREADS = 256;
constexpr int MAX_N = 512;

__device__ __forceinline__ void qmul4(const double a[4], const double b[4], double r[4]) {
  r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// conj(c) * e_K for K = 0 (x: e = k), 1 (y: e = j), 2 (z: e = i)
__device__ __forceinline__ void conj_times_unit(const double c[4], int K, double r[4]) {
  const double a0 = c[0], a1 = -c[1], a2 = -c[2], a3 = -c[3];
  if (K == 2) {  // q * i = (-q1, q0, q3, -q2)
    r[0] = -a1; r[1] = a0; r[2] = a3; r[3] = -a2;
  } else if (K == 1) {  // q * j = (-q2, -q3, q0, q1)
    r[0] = -a2; r[1] = -a3; r[2] = a0; r[3] = a1;
  } else {  // q * k = (-q3, q2, -q1, q0)
    r[0] = -a3; r[1] = a2; r[2] = -a1; r[3] = a0;
  }
}

__device__ __forceinline__ double block_max(double mx, double *red) {
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < DENS_THREADS / 64; ++w) m = fmax(m, red[w]);
  return m;
}

__global__ void __launch_bounds__(DENS_THREADS) k_density(DensityArgs a) {
  __shared__ double ck[4][MAX_N];
  __shared__ double cl[4][MAX_N];
  __shared__ double red[DENS_THREADS / 64];
  const int64_t row = blockIdx.x;
  const int cls = a.cls[row];
  const int n = a.n;
  const int i0 = a.i0, i1 = a.i1;
  double *Drow = a.D + row * a.ld;
  if (cls < 0) {  // padding row: zero density, zero bound
    if (!a.bound_only)
      for (int c = threadIdx.x; c < 4 * (i1 - i0); c += DENS_THREADS) Drow[c] = 0.0;
    else if (threadIdx.x == 0)
      a.Dmax[row] = 0.0;
    return;
  }
  const double *C = cls == 0 ? a.CL : a.CS;
  const int N = cls == 0 ? a.NL : a.NS;
  const int ka = a.mu[row], la = a.nu[row];
  for (int t = threadIdx.x; t < 4 * n; t += DENS_THREADS) {
    int z = t / n, r = t % n;
    ck[z][r] = C[((int64_t)z * N + ka) * n + r];
    cl[z][r] = C[((int64_t)z * N + la) * n + r];
  }
  __syncthreads();
  const bool offdiag = ka != la;
  double mx = 0.0;
  for (int idx = i0 + threadIdx.x; idx < i1; idx += DENS_THREADS) {
    int rs = a.rs[idx];
    int r = rs & 0xffff, s = rs >> 16;
    double d0, d1, d2, d3;
    qconjmul(ck[0][r], ck[1][r], ck[2][r], ck[3][r], cl[0][s], cl[1][s], cl[2][s], cl[3][s],
             d0, d1, d2, d3);
    mx = fmax(mx, fmax(fmax(fabs(d0), fabs(d1)), fmax(fabs(d2), fabs(d3))));
    if (offdiag) {
      double e0, e1, e2, e3;
      qconjmul(cl[0][r], cl[1][r], cl[2][r], cl[3][r], ck[0][s], ck[1][s], ck[2][s], ck[3][s],
               e0, e1, e2, e3);
      mx = fmax(mx, fmax(fmax(fabs(e0), fabs(e1)), fmax(fabs(e2), fabs(e3))));
      d0 += e0;
      d1 += e1;
      d2 += e2;
      d3 += e3;
    }
    if (!a.bound_only) {
      double2 *dst = reinterpret_cast<double2 *>(Drow + 4 * (idx - i0));
      dst[0] = make_double2(d0, d1);
      dst[1] = make_double2(d2, d3);
    }
  }
  if (a.bound_only) {
    double m = block_max(mx, red);
    if (threadIdx.x == 0) a.Dmax[row] = m;
  }
}

__global__ void __launch_bounds__(DENS_THREADS) k_density_gaunt(DensityArgs a) {
  __shared__ double ck[4][MAX_N];  // C^L row ka
  __shared__ double cl[4][MAX_N];  // C^S row la
  __shared__ double red[DENS_THREADS / 64];
  const int64_t row = blockIdx.x;
  const int cls = a.cls[row];
  const int n = a.n;
  const int i0 = a.i0, i1 = a.i1;
  double *Drow = a.D + row * a.ld;
  if (cls < 0) {
    if (!a.bound_only) {
      for (int K = 0; K < 3; ++K)
        for (int c = threadIdx.x; c < 4 * (i1 - i0); c += DENS_THREADS)
          Drow[K * a.ldK + c] = 0.0;
    } else if (threadIdx.x == 0) {
      a.Dmax[row] = 0.0;
    }
    return;
  }
  const int ka = a.mu[row], la = a.nu[row];
  for (int t = threadIdx.x; t < 4 * n; t += DENS_THREADS) {
    int z = t / n, r = t % n;
    ck[z][r] = a.CL[((int64_t)z * a.NL + ka) * n + r];
    cl[z][r] = a.CS[((int64_t)z * a.NS + la) * n + r];
  }
  __syncthreads();
  double mx = 0.0;
  for (int idx = i0 + threadIdx.x; idx < i1; idx += DENS_THREADS) {
    int rs = a.rs[idx];
    int r = rs & 0xffff, s = rs >> 16;
    const double lr[4] = {ck[0][r], ck[1][r], ck[2][r], ck[3][r]};
    const double sr[4] = {cl[0][r], cl[1][r], cl[2][r], cl[3][r]};
    const double ls[4] = {ck[0][s], ck[1][s], ck[2][s], ck[3][s]};
    const double ss[4] = {cl[0][s], cl[1][s], cl[2][s], cl[3][s]};
    for (int K = 0; K < 3; ++K) {
      double u[4], v[4], d1[4], d2[4];
      conj_times_unit(lr, K, u);
      qmul4(u, ss, d1);
      conj_times_unit(sr, K, v);
      qmul4(v, ls, d2);
      double d0 = d1[0] + d2[0], dd1 = d1[1] + d2[1], dd2 = d1[2] + d2[2], dd3 = d1[3] + d2[3];
      mx = fmax(mx, fmax(fmax(fabs(d0), fabs(dd1)), fmax(fabs(dd2), fabs(dd3))));
      if (!a.bound_only) {
        double2 *dst = reinterpret_cast<double2 *>(Drow + K * a.ldK + 4 * (idx - i0));
        dst[0] = make_double2(d0, dd1);
        dst[1] = make_double2(dd2, dd3);
      }
    }
  }
  if (a.bound_only) {
    double m = block_max(mx, red);
    if (threadIdx.x == 0) a.Dmax[row] = m;
  }
}

// ---------------------------------------------------------------------------
// General (Kramers-unrestricted) two-spinor MOs, Eqs. (Den), (QuaternionScatter):
// the Pauli-scalar density of spinor pair (c, d) on the AO pair (ka, la) is
//   D^{cd}_{ka la} = sum_tau conj(c_{ka tau c}) c_{la tau d}  (complex),
// symmetrized over ka <-> la like the quaternion density; D^{dc}_{la ka} =
// conj(D^{cd}_{ka la}), so pairs c <= d with both orderings cover Dmax, the
// largest |re| or |im| part over all ordered pairs.  Gaunt (LS rows): the
// sigma_K-weighted density of both L-S orderings,
//   P^{K,cd} = c^L(ka, c)^dagger sigma_K c^S(la, d) + c^S(la, c)^dagger sigma_K c^L(ka, d),
// with P^{K,dc} = conj(P^{K,cd}).
struct Cx {
  double re, im;
};
__device__ __forceinline__ Cx cmul_conj(double ar, double ai, double br, double bi) {
  return {ar * br + ai * bi, ar * bi - ai * br};  // conj(a) b
}

// c^dagger sigma_K d for two-spinors c = (ca, cb), d = (da, db)
__device__ __forceinline__ Cx sigma_form(int K, const double c[4], const double d[4]) {
  const Cx aa = cmul_conj(c[0], c[1], d[0], d[1]), ab = cmul_conj(c[0], c[1], d[2], d[3]);
  const Cx ba = cmul_conj(c[2], c[3], d[0], d[1]), bb = cmul_conj(c[2], c[3], d[2], d[3]);
  if (K == 0) return {ab.re + ba.re, ab.im + ba.im};                   // sigma_x
  if (K == 1) return {ab.im - ba.im, -(ab.re - ba.re)};                // sigma_y: -i ab + i ba
  return {aa.re - bb.re, aa.im - bb.im};                               // sigma_z
}

__global__ void __launch_bounds__(DENS_THREADS) k_density_spinor(DensityArgs a) {
  __shared__ double ck[4][MAX_N];
  __shared__ double cl[4][MAX_N];
  __shared__ double red[DENS_THREADS / 64];
  const int64_t row = blockIdx.x;
  const int cls = a.cls[row];
  const int n = a.n;
  const int i0 = a.i0, i1 = a.i1;
  double *Drow = a.D + row * a.ld;
  if (cls < 0) {
    if (!a.bound_only)
      for (int c = threadIdx.x; c < 4 * (i1 - i0); c += DENS_THREADS) Drow[c] = 0.0;
    else if (threadIdx.x == 0)
      a.Dmax[row] = 0.0;
    return;
  }
  const double *C = cls == 0 ? a.CL : a.CS;
  const int N = cls == 0 ? a.NL : a.NS;
  const int ka = a.mu[row], la = a.nu[row];
  for (int t = threadIdx.x; t < 4 * n; t += DENS_THREADS) {
    int z = t / n, r = t % n;
    ck[z][r] = C[((int64_t)z * N + ka) * n + r];
    cl[z][r] = C[((int64_t)z * N + la) * n + r];
  }
  __syncthreads();
  const bool offdiag = ka != la;
  double mx = 0.0;
  // one thread per spinor pair i of the groups [i0, i1)
  for (int i = 2 * i0 + threadIdx.x; i < 2 * i1; i += DENS_THREADS) {
    double dr = 0.0, di = 0.0;
    if (i < a.nspair) {
      const int rs = a.rs[i];
      const int c = rs & 0xffff, d = rs >> 16;
      const Cx x1 = cmul_conj(ck[0][c], ck[1][c], cl[0][d], cl[1][d]);
      const Cx x2 = cmul_conj(ck[2][c], ck[3][c], cl[2][d], cl[3][d]);
      dr = x1.re + x2.re;
      di = x1.im + x2.im;
      mx = fmax(mx, fmax(fabs(dr), fabs(di)));
      if (offdiag) {
        const Cx y1 = cmul_conj(cl[0][c], cl[1][c], ck[0][d], ck[1][d]);
        const Cx y2 = cmul_conj(cl[2][c], cl[3][c], ck[2][d], ck[3][d]);
        const double er = y1.re + y2.re, ei = y1.im + y2.im;
        mx = fmax(mx, fmax(fabs(er), fabs(ei)));
        dr += er;
        di += ei;
      }
    }
    if (!a.bound_only)
      *reinterpret_cast<double2 *>(Drow + 2 * (i - 2 * i0)) = make_double2(dr, di);
  }
  if (a.bound_only) {
    double m = block_max(mx, red);
    if (threadIdx.x == 0) a.Dmax[row] = m;
  }
}

__global__ void __launch_bounds__(DENS_THREADS) k_density_spinor_gaunt(DensityArgs a) {
  __shared__ double ck[4][MAX_N];  // C^L row ka
  __shared__ double cl[4][MAX_N];  // C^S row la
  __shared__ double red[DENS_THREADS / 64];
  const int64_t row = blockIdx.x;
  const int cls = a.cls[row];
  const int n = a.n;
  const int i0 = a.i0, i1 = a.i1;
  double *Drow = a.D + row * a.ld;
  if (cls < 0) {
    if (!a.bound_only) {
      for (int K = 0; K < 3; ++K)
        for (int c = threadIdx.x; c < 4 * (i1 - i0); c += DENS_THREADS)
          Drow[K * a.ldK + c] = 0.0;
    } else if (threadIdx.x == 0) {
      a.Dmax[row] = 0.0;
    }
    return;
  }
  const int ka = a.mu[row], la = a.nu[row];
  for (int t = threadIdx.x; t < 4 * n; t += DENS_THREADS) {
    int z = t / n, r = t % n;
    ck[z][r] = a.CL[((int64_t)z * a.NL + ka) * n + r];
    cl[z][r] = a.CS[((int64_t)z * a.NS + la) * n + r];
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = 2 * i0 + threadIdx.x; i < 2 * i1; i += DENS_THREADS) {
    const bool real_pair = i < a.nspair;
    int c = 0, d = 0;
    if (real_pair) {
      const int rs = a.rs[i];
      c = rs & 0xffff;
      d = rs >> 16;
    }
    const double lc[4] = {ck[0][c], ck[1][c], ck[2][c], ck[3][c]};
    const double sc[4] = {cl[0][c], cl[1][c], cl[2][c], cl[3][c]};
    const double ld_[4] = {ck[0][d], ck[1][d], ck[2][d], ck[3][d]};
    const double sd[4] = {cl[0][d], cl[1][d], cl[2][d], cl[3][d]};
    for (int K = 0; K < 3; ++K) {
      double pr = 0.0, pi = 0.0;
      if (real_pair) {
        const Cx u = sigma_form(K, lc, sd), v = sigma_form(K, sc, ld_);
        pr = u.re + v.re;
        pi = u.im + v.im;
        mx = fmax(mx, fmax(fabs(pr), fabs(pi)));
      }
      if (!a.bound_only)
        *reinterpret_cast<double2 *>(Drow + K * a.ldK + 2 * (i - 2 * i0)) = make_double2(pr, pi);
    }
  }
  if (a.bound_only) {
    double m = block_max(mx, red);
    if (threadIdx.x == 0) a.Dmax[row] = m;
  }
}

void launch_density(const DensityArgs &a, hipStream_t s) {
  if (a.nrows <= 0) return;
  if (a.spinor) {
    if (a.gaunt)
      hipLaunchKernelGGL(k_density_spinor_gaunt, dim3((unsigned)a.nrows), dim3(DENS_THREADS), 0,
                         s, a);
    else
      hipLaunchKernelGGL(k_density_spinor, dim3((unsigned)a.nrows), dim3(DENS_THREADS), 0, s, a);
    return;
  }
  if (a.gaunt)
    hipLaunchKernelGGL(k_density_gaunt, dim3((unsigned)a.nrows), dim3(DENS_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL(k_density, dim3((unsigned)a.nrows), dim3(DENS_THREADS), 0, s, a);
}

}  // namespace qdcb
