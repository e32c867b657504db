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
struct PrimPairs {
  double *ip;
  double *x;
  double *y;
  double *z;
  double *e;
};

struct PrimPairsC {
  const double *ip, *x, *y, *z, *e;
  __host__ __device__ PrimPairsC() : ip(nullptr), x(nullptr), y(nullptr), z(nullptr), e(nullptr) {}
  __host__ __device__ PrimPairsC(const PrimPairs &s) : ip(s.ip), x(s.x), y(s.y), z(s.z), e(s.e) {}
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
  // far field, 1/R: the library rsqrt, whose longer sequence the compiler
  // keeps behind a branch that wavefronts without such lanes skip
  return rsqrt(r2);
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
