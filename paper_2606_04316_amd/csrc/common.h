// common.h -- device helpers shared by the qdcb HIP kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qdcb {

constexpr int TILE = 64;  // pairs per bra/ket tile (one wavefront of bra rows)
constexpr double PI = 3.14159265358979323846;
// sqrt(2) * pi^(5/4): folded into every primitive-pair prefactor so that
// E_ij E_kl = 2 pi^(5/2) c_i c_j c_k c_l K_ij K_kl / (p q).
constexpr double SQRT2_PI54 = 5.914967172795613;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Primitive-pair data of the Gaussian product exp(-a|r-A|^2) exp(-b|r-B|^2)
// = K_ab exp(-p|r-P|^2), structure of arrays indexed by primitive pair.
struct PrimPairs {
  double *p;   // a + b
  double *x;   // P
  double *y;
  double *z;
  double *e;   // c_a c_b K_ab sqrt(2) pi^(5/4) / p
};

struct PrimPairsC {
  const double *p, *x, *y, *z, *e;
  __host__ __device__ PrimPairsC() : p(nullptr), x(nullptr), y(nullptr), z(nullptr), e(nullptr) {}
  __host__ __device__ PrimPairsC(const PrimPairs &s) : p(s.p), x(s.x), y(s.y), z(s.z), e(s.e) {}
};

// Boys function F0(T) = (1/2) sqrt(pi/T) erf(sqrt(T)); two Taylor terms where
// T is too small for the closed form (T = 0 for concentric distributions).
__device__ __forceinline__ double boys0(double T) {
  if (T < 1e-12) return 1.0 - T * (1.0 / 3.0);
  return 0.5 * sqrt(PI / T) * erf(sqrt(T));
}

// One primitive quartet: E_ij E_kl F0(pq/(p+q) |P-Q|^2) / sqrt(p+q).
__device__ __forceinline__ double prim_quartet(double p, double px, double py, double pz,
                                               double pe, double q, double qx, double qy,
                                               double qz, double qe) {
  double s = p + q;
  double is = 1.0 / s;
  double dx = px - qx, dy = py - qy, dz = pz - qz;
  double r2 = dx * dx + dy * dy + dz * dz;
  double T = p * q * is * r2;
  return pe * qe * boys0(T) * sqrt(is);
}

// Contracted ERI between pair a (primitive pairs [a0, a1)) and pair b ([b0, b1)).
__device__ __forceinline__ double contracted_eri(const PrimPairsC &A, int64_t a0, int64_t a1,
                                                 const PrimPairsC &B, int64_t b0, int64_t b1) {
  double acc = 0.0;
  for (int64_t i = a0; i < a1; ++i) {
    double p = A.p[i], px = A.x[i], py = A.y[i], pz = A.z[i], pe = A.e[i];
    for (int64_t k = b0; k < b1; ++k)
      acc += prim_quartet(p, px, py, pz, pe, B.p[k], B.x[k], B.y[k], B.z[k], B.e[k]);
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
