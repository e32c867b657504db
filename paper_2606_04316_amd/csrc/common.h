// common.h -- device helpers shared by the qdcb HIP kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qdcb {

constexpr int TILE = 64;  // pairs per bra/ket tile (one wavefront of bra rows)
constexpr double PI = 3.14159265358979323846;
constexpr double TWO_OVER_SQRTPI = 1.1283791670955126;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Primitive-pair data of the Gaussian product
//   c_a exp(-a|r-A|^2) c_b exp(-b|r-B|^2) = c_a c_b K_ab exp(-p|r-P|^2),
// p = a + b, K_ab = exp(-ab/p |A-B|^2), stored as structure of arrays:
//   ip = 1/p,  P,  e = c_a c_b K_ab (pi/p)^{3/2}  (the charge of the product).
// The s-type ERI of two such charge distributions is
//   [ab|cd] = e_ab e_cd erf(sqrt(rho) R) / R,  R = |P - Q|, 1/rho = 1/p + 1/q,
// i.e. 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd F0(rho R^2) with the Boys
// function in its erf form F0(T) = (1/2) sqrt(pi/T) erf(sqrt T).
// Bases with p functions add, per primitive pair of functions (f, g),
//   pa = P_i - A_i for f = p_i on centre A (0 for s), pb = P_j - B_j for g.
struct PrimPairs {
  double *ip;
  double *x;
  double *y;
  double *z;
  double *e;
  double *pa = nullptr;
  double *pb = nullptr;
};

struct PrimPairsC {
  const double *ip, *x, *y, *z, *e, *pa, *pb;
  __host__ __device__ PrimPairsC()
      : ip(nullptr), x(nullptr), y(nullptr), z(nullptr), e(nullptr), pa(nullptr), pb(nullptr) {}
  __host__ __device__ PrimPairsC(const PrimPairs &s)
      : ip(s.ip), x(s.x), y(s.y), z(s.z), e(s.e), pa(s.pa), pb(s.pb) {}
};

// erf(sqrt(rho) R) / R for one primitive quartet; two Taylor terms of
// (2/sqrt(pi)) sqrt(rho) (1 - rho R^2 / 3 + ...) where rho R^2 is too small for
// the quotient; erfc(6) < 2.2e-17, so erf is 1 to double precision beyond 6.
__device__ __forceinline__ double coulomb_kernel(double ip, double px, double py, double pz,
                                                 double iq, double qx, double qy, double qz) {
  const double t = ip + iq;  // 1/rho
  const double sr = rsqrt(t);
  const double dx = px - qx, dy = py - qy, dz = pz - qz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double T = r2 * (sr * sr);
  if (T < 1e-20) return TWO_OVER_SQRTPI * sr * (1.0 - T * (1.0 / 3.0));
  const double iR = rsqrt(r2);
  const double x = r2 * iR * sr;
  return x >= 6.0 ? iR : erf(x) * iR;
}

// Boys F0 by Taylor expansion about a grid: T_i = i / 8 (i = 0 .. BOYS_N - 1,
// T < 36), tab[8 i + k] = (2 / sqrt(pi)) (-1)^k F_k(T_i) / k!, so that for
// |d| <= 1/16
//   (2 / sqrt(pi)) F0(T_i + d) = sum_k tab[8 i + k] d^k  (k <= 7),
// remainder below F_8(T_i) (1/16)^8 / 8! < 3e-16 relative.  For T >= 36
// erf(sqrt T) = 1 to double precision and the kernel is 1 / R.  Same value
// as coulomb_kernel, without the range branches of erf.
constexpr int BOYS_N = 289;
constexpr double BOYS_TMAX = 36.0;
// LDS copies of the table pad each row to BOYS_LD doubles (80 bytes: rows
// stay 16-byte aligned and rows i, i' share banks only when i = i' mod 16)
constexpr int BOYS_LD = 10;
// Columns of the table of the Cartesian (s/p) integral tiles: F_0 .. F_11, so
// that F_0 .. F_4 each take eight Taylor terms
constexpr int BOYS_LDC = 12;

// 1/sqrt(x) for finite x > 0: the hardware estimate y and one second-order
// correction from the binomial series, y (1 + e/2 + 3 e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

template <int LD = 8>
__device__ __forceinline__ double coulomb_kernel_tab(const double *tab, double ip, double px,
                                                     double py, double pz, double iq, double qx,
                                                     double qy, double qz) {
  const double t = ip + iq;  // 1/rho > 0
  const double sr = rsqrt_pos(t);
  const double dx = px - qx, dy = py - qy, dz = pz - qz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double T = r2 * (sr * sr);
  if (T < BOYS_TMAX) {
    const int i = (int)fma(T, 8.0, 0.5);  // nearest grid point (T >= 0)
    const double d = fma(-0.125, (double)i, T);
    const double *c = tab + LD * i;
    double f = c[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) f = fma(f, d, c[k]);
    return sr * f;  // the table carries the factor 2 / sqrt(pi)
  }
  // far field, 1/R (r2 > 0 here): the refined hardware estimate, a short
  // branch for the lanes of a wavefront that take it
  return rsqrt_pos(r2);
}

__device__ __forceinline__ double prim_quartet(double ip, double px, double py, double pz,
                                               double pe, double iq, double qx, double qy,
                                               double qz, double qe) {
  return pe * qe * coulomb_kernel(ip, px, py, pz, iq, qx, qy, qz);
}

// Contracted ERI between pair a (primitive pairs [a0, a1)) and pair b ([b0, b1)).
__device__ __forceinline__ double contracted_eri(const PrimPairsC &A, int64_t a0, int64_t a1,
                                                 const PrimPairsC &B, int64_t b0, int64_t b1) {
  double acc = 0.0;
  for (int64_t i = a0; i < a1; ++i) {
    const double ip = A.ip[i], px = A.x[i], py = A.y[i], pz = A.z[i];
    double s = 0.0;
    for (int64_t k = b0; k < b1; ++k)
      s += B.e[k] * coulomb_kernel(ip, px, py, pz, B.ip[k], B.x[k], B.y[k], B.z[k]);
    acc += A.e[i] * s;
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Integrals over Cartesian s and p functions (McMurchie-Davidson form).
//
// A function pair (f, g) has the code cf | (cg << 2), c = 0 for s and
// 1, 2, 3 for p_x, p_y, p_z.  With Lambda_t the Hermite Gaussians
// d^t/dP^t exp(-p|r-P|^2), a pair's product expands over at most four of
// them: for f = p_i on A and g = p_j on B
//   (PA_i PB_j + delta_ij / 2p) L_0 + PB_j / 2p L_{e_i} + PA_i / 2p L_{e_j}
//     + 1 / 4p^2 L_{e_i + e_j},
// which drops to PA_i L_0 + 1/2p L_{e_i} (f = p_i, g = s) and to L_0 for two
// s functions.  [L_t(P) | L_u(Q)] = (-1)^{|u|} R_{t+u}(P - Q) times the
// charge factors, where R_t is the derivative d^t/dX^t of
// g_0(X) = (2/sqrt(pi)) sqrt(rho) F_0(rho |X|^2).  For a function of |X|^2
// the derivatives up to order four are, with G_n = (-2 rho)^n g_n and
// g_n = (2/sqrt(pi)) sqrt(rho) F_n(rho |X|^2):
//   R_i = X_i G_1,  R_ij = d_ij G_1 + X_i X_j G_2,
//   R_ijk = (d_ij X_k + d_ik X_j + d_jk X_i) G_2 + X_i X_j X_k G_3,
//   R_ijkl = (d_ij d_kl + d_ik d_jl + d_il d_jk) G_2
//          + (d_ij X_k X_l + d_ik X_j X_l + d_il X_j X_k + d_jk X_i X_l
//             + d_jl X_i X_k + d_kl X_i X_j) G_3 + X_i X_j X_k X_l G_4.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double xcomp(const double X[3], int i) {
  return i == 0 ? X[0] : (i == 1 ? X[1] : X[2]);
}
__device__ __forceinline__ double kd(int i, int j) { return i == j ? 1.0 : 0.0; }

__device__ __forceinline__ double herm_r2(int i, int j, const double X[3], const double G[5]) {
  return kd(i, j) * G[1] + xcomp(X, i) * xcomp(X, j) * G[2];
}
__device__ __forceinline__ double herm_r3(int i, int j, int k, const double X[3],
                                          const double G[5]) {
  const double xi = xcomp(X, i), xj = xcomp(X, j), xk = xcomp(X, k);
  return (kd(i, j) * xk + kd(i, k) * xj + kd(j, k) * xi) * G[2] + xi * xj * xk * G[3];
}
__device__ __forceinline__ double herm_r4(int i, int j, int k, int l, const double X[3],
                                          const double G[5]) {
  const double xi = xcomp(X, i), xj = xcomp(X, j), xk = xcomp(X, k), xl = xcomp(X, l);
  const double d2 = kd(i, j) * kd(k, l) + kd(i, k) * kd(j, l) + kd(i, l) * kd(j, k);
  const double d1 = kd(i, j) * xk * xl + kd(i, k) * xj * xl + kd(i, l) * xj * xk +
                    kd(j, k) * xi * xl + kd(j, l) * xi * xk + kd(k, l) * xi * xj;
  return d2 * G[2] + d1 * G[3] + xi * xj * xk * xl * G[4];
}

// Hermite coefficients of one side: h[0] of L_0, h[1] of L_{e_a}, h[2] of
// L_{e_b}, h[3] of L_{e_a + e_b}; a, b = direction (0..2) of the first and
// second function, or -1 for an s function.  inv2p = 1 / (2p).
__device__ __forceinline__ void herm_side(int code, double pa, double pb, double inv2p,
                                          double h[4], int &a, int &b) {
  a = (code & 3) - 1;
  b = ((code >> 2) & 3) - 1;
  const double fa = a >= 0 ? pa : 1.0, fb = b >= 0 ? pb : 1.0;
  h[0] = fa * fb + ((a >= 0 && a == b) ? inv2p : 0.0);
  h[1] = a >= 0 ? fb * inv2p : 0.0;
  h[2] = b >= 0 ? fa * inv2p : 0.0;
  h[3] = (a >= 0 && b >= 0) ? inv2p * inv2p : 0.0;
}

// Sum over the Hermite terms of bra (hb, directions a, b) and ket (hk,
// directions c, d) of hb hk (-1)^{ket order} R; G as above, X = P - Q.
__device__ inline double herm_contract(const double hb[4], int a, int b, const double hk[4],
                                       int c, int d, const double X[3], const double G[5]) {
  // bra terms: (order, dirs) = (0), (1: a), (1: b), (2: a, b); ket likewise
  double s = 0.0;
  // ket L_0
  {
    double t = hb[0] * G[0];
    if (a >= 0) t += hb[1] * xcomp(X, a) * G[1];
    if (b >= 0) t += hb[2] * xcomp(X, b) * G[1];
    if (a >= 0 && b >= 0) t += hb[3] * herm_r2(a, b, X, G);
    s += hk[0] * t;
  }
  if (c >= 0) {  // ket L_{e_c}, sign -1
    double t = hb[0] * xcomp(X, c) * G[1];
    if (a >= 0) t += hb[1] * herm_r2(a, c, X, G);
    if (b >= 0) t += hb[2] * herm_r2(b, c, X, G);
    if (a >= 0 && b >= 0) t += hb[3] * herm_r3(a, b, c, X, G);
    s -= hk[1] * t;
  }
  if (d >= 0) {  // ket L_{e_d}, sign -1
    double t = hb[0] * xcomp(X, d) * G[1];
    if (a >= 0) t += hb[1] * herm_r2(a, d, X, G);
    if (b >= 0) t += hb[2] * herm_r2(b, d, X, G);
    if (a >= 0 && b >= 0) t += hb[3] * herm_r3(a, b, d, X, G);
    s -= hk[2] * t;
  }
  if (c >= 0 && d >= 0) {  // ket L_{e_c + e_d}, sign +1
    double t = hb[0] * herm_r2(c, d, X, G);
    if (a >= 0) t += hb[1] * herm_r3(a, c, d, X, G);
    if (b >= 0) t += hb[2] * herm_r3(b, c, d, X, G);
    if (a >= 0 && b >= 0) t += hb[3] * herm_r4(a, b, c, d, X, G);
    s += hk[3] * t;
  }
  return s;
}

// g_n = (2/sqrt(pi)) sqrt(rho) F_n(T), n = 0..4, without a table: below
// T = 10 from the series of F_4 and the downward recursion
// F_{m-1} = (2T F_m + e^-T) / (2m - 1); from T = 10 on from the erf form of
// F_0 and the upward recursion F_{m+1} = ((2m+1) F_m - e^-T) / (2T).
__device__ inline void boys_g_exact(double T, double sr, double g[5]) {
  const double c = TWO_OVER_SQRTPI * sr;
  const double eT = exp(-T);
  if (T < 10.0) {
    double term = 1.0 / 9.0, sum = term;
    for (int k = 1; k < 200; ++k) {
      term *= 2.0 * T / (9.0 + 2.0 * k);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    double f = eT * sum;
    g[4] = c * f;
    for (int m = 4; m >= 1; --m) {
      f = (2.0 * T * f + eT) / (2.0 * m - 1.0);
      g[m - 1] = c * f;
    }
  } else {
    double f = 0.5 * sqrt(PI / T) * erf(sqrt(T));
    g[0] = c * f;
    for (int m = 0; m < 4; ++m) {
      f = ((2.0 * m + 1.0) * f - eT) / (2.0 * T);
      g[m + 1] = c * f;
    }
  }
}

// One primitive quartet over Cartesian s/p functions (no charge factors):
// bra pair (ip = 1/p, P, pa, pb, code cb), ket pair (iq, Q, qa, qb, code ck).
__device__ inline double cart_quartet_exact(double ip, double px, double py, double pz, double pa,
                                            double pb, int cb, double iq, double qx, double qy,
                                            double qz, double qa, double qb, int ck) {
  const double t = ip + iq;  // 1 / rho
  const double rho = 1.0 / t;
  const double sr = sqrt(rho);
  const double X[3] = {px - qx, py - qy, pz - qz};
  const double T = rho * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double g[5];
  boys_g_exact(T, sr, g);
  double G[5];
  double f = 1.0;
  for (int n = 0; n < 5; ++n) {
    G[n] = f * g[n];
    f *= -2.0 * rho;
  }
  double hb[4], hk[4];
  int a, b, c, d;
  herm_side(cb, pa, pb, 0.5 * ip, hb, a, b);
  herm_side(ck, qa, qb, 0.5 * iq, hk, c, d);
  return herm_contract(hb, a, b, hk, c, d, X, G);
}

// Contracted integral of two pairs with codes (Cartesian bases; a store
// without pa / pb belongs to an s-only basis, code 0).
__device__ inline double contracted_eri_cart(const PrimPairsC &A, int64_t a0, int64_t a1, int ca,
                                             const PrimPairsC &B, int64_t b0, int64_t b1,
                                             int cb) {
  double acc = 0.0;
  for (int64_t i = a0; i < a1; ++i) {
    const double pa = A.pa ? A.pa[i] : 0.0, pb = A.pb ? A.pb[i] : 0.0;
    double s = 0.0;
    for (int64_t k = b0; k < b1; ++k)
      s += B.e[k] * cart_quartet_exact(A.ip[i], A.x[i], A.y[i], A.z[i], pa, pb, ca, B.ip[k],
                                       B.x[k], B.y[k], B.z[k], B.pa ? B.pa[k] : 0.0,
                                       B.pb ? B.pb[k] : 0.0, cb);
    acc += A.e[i] * s;
  }
  return acc;
}

// Quaternion product conj(a) * b (a, b as 4 components).
__device__ __forceinline__ void qconjmul(double a0, double a1, double a2, double a3, double b0,
                                         double b1, double b2, double b3, double &r0,
                                         double &r1, double &r2, double &r3) {
  // conj(a) = (a0, -a1, -a2, -a3)
  r0 = a0 * b0 + a1 * b1 + a2 * b2 + a3 * b3;
  r1 = a0 * b1 - a1 * b0 - a2 * b3 + a3 * b2;
  r2 = a0 * b2 + a1 * b3 - a2 * b0 - a3 * b1;
  r3 = a0 * b3 - a1 * b2 + a2 * b1 - a3 * b0;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace qdcb
