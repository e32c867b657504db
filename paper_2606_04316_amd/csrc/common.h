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
// Code of a function pair (f, g) of Cartesian functions (function codes 0 .. 19:
// s; p_x, p_y, p_z; six d; ten f) and its two function codes.
__host__ __device__ __forceinline__ int pair_code(int cf, int cg) { return cf | (cg << 5); }
__host__ __device__ __forceinline__ int code_f(int c) { return c & 31; }
__host__ __device__ __forceinline__ int code_g(int c) { return (c >> 5) & 31; }

// Primitive-pair data: 1/p, P, the charge factor e, and for Cartesian bases
// pa / pb = (P - A) and (P - B) along the direction of a p function (0 for
// an s function), the full vectors P - A = (ax, ay, az), P - B = (bx, by, bz)
// and the pair's Hermite coefficients E^{ij}_t of each direction
// (E[PAIR_E * i + 7 d + t], t <= 6; the general kernels of bases with d or f
// functions).
constexpr int PAIR_E = 21;  // Hermite coefficients per primitive pair (3 directions x 7)
struct PrimPairs {
  double *ip;
  double *x;
  double *y;
  double *z;
  double *e;
  double *pa = nullptr;
  double *pb = nullptr;
  double *ax = nullptr, *ay = nullptr, *az = nullptr;
  double *bx = nullptr, *by = nullptr, *bz = nullptr;
  double *E = nullptr;
};

struct PrimPairsC {
  const double *ip, *x, *y, *z, *e, *pa, *pb;
  const double *ax, *ay, *az, *bx, *by, *bz;
  const double *E;
  __host__ __device__ PrimPairsC()
      : ip(nullptr), x(nullptr), y(nullptr), z(nullptr), e(nullptr), pa(nullptr), pb(nullptr),
        ax(nullptr), ay(nullptr), az(nullptr), bx(nullptr), by(nullptr), bz(nullptr),
        E(nullptr) {}
  __host__ __device__ PrimPairsC(const PrimPairs &s)
      : ip(s.ip), x(s.x), y(s.y), z(s.z), e(s.e), pa(s.pa), pb(s.pb), ax(s.ax), ay(s.ay),
        az(s.az), bx(s.bx), by(s.by), bz(s.bz), E(s.E) {}
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
// Columns of the table of the general (s .. f) tiles: F_0 .. F_21 (F_0 .. F_14
// with eight Taylor terms each: Boys orders to 12 for the Coulomb kernel, to
// 14 for the gauge kernel)
constexpr int BOYS_LDG = 22;

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
// A function pair (f, g) has the code cf | (cg << 5) (pair_code), c = 0 for s
// and 1, 2, 3 for p_x, p_y, p_z (4 .. 19 for d and f functions, general form
// below).  With Lambda_t the Hermite Gaussians
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
  a = code_f(code) - 1;
  b = code_g(code) - 1;
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

// ---------------------------------------------------------------------------
// Integrals over Cartesian s, p, d and f functions, general form (bases with
// d or f functions).  Codes 4 .. 9 are d_xx, d_yy, d_zz, d_xy, d_xz, d_yz and
// 10 .. 19 f_xxx, f_yyy, f_zzz, f_xxy, f_xxz, f_xyy, f_yyz, f_xzz, f_yzz, f_xyz,
// i.e. the monomial (x - A_x)^{l_x} (y - A_y)^{l_y} (z - A_z)^{l_z}.
// McMurchie-Davidson form: per Cartesian direction the product of the two
// functions of a pair expands in Hermite Gaussians with the coefficients
// E^{ij}_t (t <= i + j) of the recursion
//   E^{i+1,j}_t = E^{ij}_{t-1} / (2p) + X_PA E^{ij}_t + (t + 1) E^{ij}_{t+1}
// (likewise j + 1 with X_PB), E^{00}_0 = 1.  The Hermite integral of orders
// (T, U, V) is the derivative of g_0 (a function of |X|^2, X = P - Q):
//   R_TUV = sum_{a, b, c} h_T^a(X_x) h_U^b(X_y) h_V^c(X_z) G_{T+U+V-a-b-c},
//   h_T^a(x) = T! / (a! (T - 2a)! 2^a) x^{T-2a},   G_n = (-2 rho)^n g_n,
// so with H_x[T] = sum_{t + u = T} Ebra_x[t] (-1)^u Eket_x[u] and
// P_x[s] = sum_T H_x[T] h_T^{T-s}(X_x) the value of a primitive quartet is
//   sum_{s_x, s_y, s_z} P_x[s_x] P_y[s_y] P_z[s_z] G_{s_x + s_y + s_z}
// (the same sums, factorized by direction).  TB, TK: bounds of the bra and
// ket pairs' Hermite orders per direction (l_f + l_g of the pair, rounded up
// to 2, 4 or 6), which size every array statically.
// ---------------------------------------------------------------------------
constexpr int GEN_TMAX = 6;                  // Hermite order of a pair per direction (two f)
constexpr int GEN_NGMAX = 2 * GEN_TMAX + 1;  // Boys orders g_0 .. g_12 (four f functions)
static_assert(PAIR_E == 3 * (GEN_TMAX + 1), "pair Hermite coefficients: 3 directions");

// a pair code with a d or f function (the general form)
__host__ __device__ __forceinline__ bool gen_code(int c) {
  return code_f(c) >= 4 || code_g(c) >= 4;
}

// powers (l_x, l_y, l_z) of a function code 0 .. 19, two bits each, six bits
// per code in two words (codes 0 .. 9, 10 .. 19)
__host__ __device__ __forceinline__ int cart_pow(int code, int dir) {
  constexpr unsigned long long PK0 =
      (0ull) | (1ull << 6) | (4ull << 12) | (16ull << 18) | (2ull << 24) | (8ull << 30) |
      (32ull << 36) | (5ull << 42) | (17ull << 48) | (20ull << 54);
  constexpr unsigned long long PK1 =
      (3ull) | (12ull << 6) | (48ull << 12) | (6ull << 18) | (18ull << 24) | (9ull << 30) |
      (24ull << 36) | (33ull << 42) | (36ull << 48) | (21ull << 54);
  const unsigned long long pk = code < 10 ? PK0 : PK1;
  const int c = code < 10 ? code : code - 10;
  return (int)((pk >> (6 * c + 2 * dir)) & 3ull);
}
// angular momentum of a function code
__host__ __device__ __forceinline__ int cart_l(int code) {
  return code == 0 ? 0 : (code < 4 ? 1 : (code < 10 ? 2 : 3));
}
// Hermite order bound of a pair code: l_f + l_g rounded up to 2, 4 or 6
__host__ __device__ __forceinline__ int gen_bucket(int c) {
  const int L = cart_l(code_f(c)) + cart_l(code_g(c));
  return L <= 2 ? 2 : (L <= 4 ? 4 : 6);
}

// E^{ij}_t, t <= T, for i, j <= 3 with i + j <= T (one direction of one
// primitive pair).
template <int T>
__device__ __forceinline__ void herm_raise(double E[T + 1], double x, double h) {
  double N[T + 1];
#pragma unroll
  for (int t = 0; t <= T; ++t) {
    double v = x * E[t];
    if (t + 1 <= T) v = fma((double)(t + 1), E[t + 1], v);
    if (t >= 1) v = fma(h, E[t - 1], v);
    N[t] = v;
  }
#pragma unroll
  for (int t = 0; t <= T; ++t) E[t] = N[t];
}
template <int T>
__device__ __forceinline__ void herm_1d(int i, int j, double pa, double pb, double h,
                                        double E[T + 1]) {
  E[0] = 1.0;
#pragma unroll
  for (int t = 1; t <= T; ++t) E[t] = 0.0;
#pragma unroll
  for (int k = 0; k < 3 && k < T; ++k)
    if (k < i) herm_raise<T>(E, pa, h);
#pragma unroll
  for (int k = 0; k < 3 && k < T; ++k)
    if (k < j) herm_raise<T>(E, pb, h);
}

// P[s] = sum_T H[T] h_T^{T-s}(x), H[T] = sum_{t+u=T} Eb[t] (-1)^u Ek[u].
template <int TB, int TK>
__device__ __forceinline__ void herm_dir(const double Eb[TB + 1], const double Ek[TK + 1],
                                         double x, double P[TB + TK + 1]) {
  constexpr int TS = TB + TK;
  double H[TS + 1];
#pragma unroll
  for (int t = 0; t <= TS; ++t) H[t] = 0.0;
#pragma unroll
  for (int t = 0; t <= TB; ++t)
#pragma unroll
    for (int u = 0; u <= TK; ++u) H[t + u] = fma(Eb[t], (u & 1) ? -Ek[u] : Ek[u], H[t + u]);
  double xp[TS + 1];
  xp[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= TS; ++k) xp[k] = xp[k - 1] * x;
#pragma unroll
  for (int q = 0; q <= TS; ++q) P[q] = 0.0;
  // h_T^a = T! / (a! (T - 2a)! 2^a): products of integers, exact in double
#pragma unroll
  for (int t = 0; t <= TS; ++t) {
    double c = 1.0;  // h_t^0
#pragma unroll
    for (int a = 0; 2 * a <= t; ++a) {
      P[t - a] = fma(H[t] * c, xp[t - 2 * a], P[t - a]);
      // h_t^{a+1} / h_t^a = (t - 2a)(t - 2a - 1) / (2 (a + 1))
      c = c * (double)((t - 2 * a) * (t - 2 * a - 1)) / (double)(2 * (a + 1));
    }
  }
}

// Sum over (s_x, s_y, s_z) of P_x P_y P_z G_{s_x+s_y+s_z} (orders above TS
// vanish: the Hermite orders of a quartet add up to at most TS).
template <int TS>
__device__ __forceinline__ double herm_sum(const double Px[TS + 1], const double Py[TS + 1],
                                           const double Pz[TS + 1], const double G[TS + 1]) {
  double Q[TS + 1];
#pragma unroll
  for (int n = 0; n <= TS; ++n) Q[n] = 0.0;
#pragma unroll
  for (int a = 0; a <= TS; ++a)
#pragma unroll
    for (int b = 0; a + b <= TS; ++b) Q[a + b] = fma(Px[a], Py[b], Q[a + b]);
  double v = 0.0;
#pragma unroll
  for (int m = 0; m <= TS; ++m) {
    double w = 0.0;
#pragma unroll
    for (int c = 0; m + c <= TS; ++c) w = fma(Pz[c], G[m + c], w);
    v = fma(Q[m], w, v);
  }
  return v;
}

// Gauge kernel r_K r_L / r^3 in the same form.  For two s distributions the
// gauge (or Breit) tile element is A(X^2) delta_KL + B(X^2) X_K X_L with
// A = g_1 / 2 + diag g_0 (diag = -1/2 gauge, +1/2 Breit) and
// B = rho (g_1 - g_2); the derivative of orders (T, U, V) of a radial
// function F(X^2) is sum h_T^a h_U^b h_V^c 2^n F^{(n)} (n = T+U+V-a-b-c), so
// A and B enter through D_A[n] = (-2 rho)^n (g_{n+1} / 2 + diag g_n) and
// D_B[n] = rho (-2 rho)^n (g_{n+1} - g_{n+2}), and the factor X_K X_L by the
// Leibniz rule, d^T (x f) = x d^T f + T d^{T-1} f and
// d^T (x^2 f) = x^2 d^T f + 2T x d^{T-1} f + T(T-1) d^{T-2} f.  Per direction
// three polynomials: P0 (no factor), P1 (factor x), P2 (factor x^2).
template <int TB, int TK>
__device__ __forceinline__ void herm_dir3(const double Eb[TB + 1], const double Ek[TK + 1],
                                          double x, double P0[TB + TK + 1],
                                          double P1[TB + TK + 1], double P2[TB + TK + 1]) {
  constexpr int TS = TB + TK;
  double H[TS + 1];
#pragma unroll
  for (int t = 0; t <= TS; ++t) H[t] = 0.0;
#pragma unroll
  for (int t = 0; t <= TB; ++t)
#pragma unroll
    for (int u = 0; u <= TK; ++u) H[t + u] = fma(Eb[t], (u & 1) ? -Ek[u] : Ek[u], H[t + u]);
  double xp[TS + 3];
  xp[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= TS + 2; ++k) xp[k] = xp[k - 1] * x;
#pragma unroll
  for (int q = 0; q <= TS; ++q) P0[q] = P1[q] = P2[q] = 0.0;
#pragma unroll
  for (int t = 0; t <= TS; ++t) {
    // d^t of f, x f, x^2 f: h_t^a at order t - a (times 1, x, x^2), h_{t-1}^a
    // at order t - 1 - a (times t for x f, 2t x for x^2 f), h_{t-2}^a at
    // order t - 2 - a (times t(t - 1) for x^2 f)
    double c = 1.0;
#pragma unroll
    for (int a = 0; 2 * a <= t; ++a) {
      const double hc = H[t] * c;
      P0[t - a] = fma(hc, xp[t - 2 * a], P0[t - a]);
      P1[t - a] = fma(hc, xp[t - 2 * a + 1], P1[t - a]);
      P2[t - a] = fma(hc, xp[t - 2 * a + 2], P2[t - a]);
      c = c * (double)((t - 2 * a) * (t - 2 * a - 1)) / (double)(2 * (a + 1));
    }
    if (t >= 1) {
      double c1 = 1.0;
#pragma unroll
      for (int a = 0; 2 * a <= t - 1; ++a) {
        const double hc = H[t] * c1 * (double)t;
        P1[t - 1 - a] = fma(hc, xp[t - 1 - 2 * a], P1[t - 1 - a]);
        P2[t - 1 - a] = fma(2.0 * hc, xp[t - 2 * a], P2[t - 1 - a]);
        c1 = c1 * (double)((t - 1 - 2 * a) * (t - 2 - 2 * a)) / (double)(2 * (a + 1));
      }
    }
    if (t >= 2) {
      double c2 = 1.0;
#pragma unroll
      for (int a = 0; 2 * a <= t - 2; ++a) {
        const double hc = H[t] * c2 * (double)(t * (t - 1));
        P2[t - 2 - a] = fma(hc, xp[t - 2 - 2 * a], P2[t - 2 - a]);
        c2 = c2 * (double)((t - 2 - 2 * a) * (t - 3 - 2 * a)) / (double)(2 * (a + 1));
      }
    }
  }
}

// g_n = (2/sqrt(pi)) sqrt(rho) F_n(T), n < NG, without a table: below T = 15
// from the series of F_{NG-1} and the downward recursion; from T = 15 on
// from the erf form of F_0 and the upward recursion (stable there for
// n <= 12: each step multiplies an error by (2m + 1) / 2T < 1).
template <int NG>
__device__ inline void boys_g_exact_n(double T, double sr, double g[NG]) {
  const double c = TWO_OVER_SQRTPI * sr;
  const double eT = exp(-T);
  if (T < 15.0) {
    constexpr int M = NG - 1;
    double term = 1.0 / (2.0 * M + 1.0), sum = term;
    for (int k = 1; k < 400; ++k) {
      term *= 2.0 * T / (2.0 * M + 1.0 + 2.0 * k);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    double f = eT * sum;
    g[M] = c * f;
    for (int m = M; m >= 1; --m) {
      f = (2.0 * T * f + eT) / (2.0 * m - 1.0);
      g[m - 1] = c * f;
    }
  } else {
    double f = 0.5 * sqrt(PI / T) * erf(sqrt(T));
    g[0] = c * f;
    for (int m = 0; m + 1 < NG; ++m) {
      f = ((2.0 * m + 1.0) * f - eT) / (2.0 * T);
      g[m + 1] = c * f;
    }
  }
}

// One primitive quartet in the general form (no charge factors): bra pair
// (ip = 1/p, P, P - A, P - B, codes fa, fb), ket pair likewise.
__device__ inline double gen_quartet_exact(double ip, const double P[3], const double PA[3],
                                           const double PB[3], int fa, int fb, double iq,
                                           const double Q[3], const double QC[3],
                                           const double QD[3], int fc, int fd) {
  constexpr int T = GEN_TMAX, TS = 2 * GEN_TMAX;
  const double rho = 1.0 / (ip + iq);
  const double X[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
  const double Tb = rho * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double g[TS + 1];
  boys_g_exact_n<TS + 1>(Tb, sqrt(rho), g);
  double f = 1.0;
  for (int n = 0; n <= TS; ++n) {
    g[n] *= f;
    f *= -2.0 * rho;
  }
  double Pd[3][TS + 1];
  for (int d = 0; d < 3; ++d) {
    double Eb[T + 1], Ek[T + 1];
    herm_1d<T>(cart_pow(fa, d), cart_pow(fb, d), PA[d], PB[d], 0.5 * ip, Eb);
    herm_1d<T>(cart_pow(fc, d), cart_pow(fd, d), QC[d], QD[d], 0.5 * iq, Ek);
    herm_dir<T, T>(Eb, Ek, X[d], Pd[d]);
  }
  return herm_sum<TS>(Pd[0], Pd[1], Pd[2], g);
}

// Contracted integral of two pairs with codes pair_code(cf, cg) in the general
// form (the pair stores carry the P - A, P - B vectors).
__device__ inline double contracted_eri_gen(const PrimPairsC &A, int64_t a0, int64_t a1, int ca,
                                            const PrimPairsC &B, int64_t b0, int64_t b1,
                                            int cb) {
  const int fa = code_f(ca), fb = code_g(ca), fc = code_f(cb), fd = code_g(cb);
  double acc = 0.0;
  for (int64_t i = a0; i < a1; ++i) {
    const double P[3] = {A.x[i], A.y[i], A.z[i]};
    const bool va = A.ax != nullptr, vb = B.ax != nullptr;
    const double PA[3] = {va ? A.ax[i] : 0.0, va ? A.ay[i] : 0.0, va ? A.az[i] : 0.0};
    const double PB[3] = {va ? A.bx[i] : 0.0, va ? A.by[i] : 0.0, va ? A.bz[i] : 0.0};
    double s = 0.0;
    for (int64_t k = b0; k < b1; ++k) {
      const double Q[3] = {B.x[k], B.y[k], B.z[k]};
      const double QC[3] = {vb ? B.ax[k] : 0.0, vb ? B.ay[k] : 0.0, vb ? B.az[k] : 0.0};
      const double QD[3] = {vb ? B.bx[k] : 0.0, vb ? B.by[k] : 0.0, vb ? B.bz[k] : 0.0};
      s += B.e[k] * gen_quartet_exact(A.ip[i], P, PA, PB, fa, fb, B.ip[k], Q, QC, QD, fc, fd);
    }
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
