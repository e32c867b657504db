// k_density.hip -- quaternion MO-pair densities and their infinity-norm bound.
//
// For an AO pair (ka, la) of class X and MO pair r <= s the quaternion pair
// density is D^{rs}_{ka la} = conj(C_ka r) C_la s (the Kramers-paired form of
// Eqs. Den and QuaternionScatter: its four real components are the four
// Pauli-scalar densities of the Kramers block).  Because the AO integral is
// symmetric in ka <-> la, the first half contracts with the symmetrized
//   D~ = D_{ka la} + D_{la ka}   (ka != la),   D_{ka ka}   (ka = la),
// stored as D~[row][4*idx(r,s) + y].  Dmax_{ka la} is the largest |component|
// of D over all ordered MO pairs (r, t), the ||D~||_inf of Eq. (SchwarzDen);
// the r <= s loop covers it because conj(D^{rt}_{ka la}) = D^{tr}_{la ka}.
//
// One workgroup per AO pair row: the two coefficient rows are staged in LDS,
// threads stride over MO pairs and write 32 contiguous bytes each (coalesced
// rows), and a block reduction forms Dmax.  HBM-bound (write of D~).
#include "kernels.h"

namespace qdcb {

constexpr int DENS_THREADS = 256;
constexpr int MAX_N = 512;

__global__ void __launch_bounds__(DENS_THREADS) k_density(DensityArgs a) {
  __shared__ double ck[4][MAX_N];
  __shared__ double cl[4][MAX_N];
  __shared__ double red[DENS_THREADS / 64];
  const int64_t row = blockIdx.x;
  const int cls = a.cls[row];
  const int n = a.n;
  double *Drow = a.D + row * a.ld;
  if (cls < 0) {  // padding row: zero density, zero bound
    for (int c = threadIdx.x; c < 4 * a.npair_mo; c += DENS_THREADS) Drow[c] = 0.0;
    if (threadIdx.x == 0) a.Dmax[row] = 0.0;
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
  for (int idx = threadIdx.x; idx < a.npair_mo; idx += DENS_THREADS) {
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
    double2 *dst = reinterpret_cast<double2 *>(Drow + 4 * idx);
    dst[0] = make_double2(d0, d1);
    dst[1] = make_double2(d2, d3);
  }
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < DENS_THREADS / 64; ++w) m = fmax(m, red[w]);
    a.Dmax[row] = m;
  }
}

void launch_density(const DensityArgs &a, hipStream_t s) {
  if (a.nrows <= 0) return;
  hipLaunchKernelGGL(k_density, dim3((unsigned)a.nrows), dim3(DENS_THREADS), 0, s, a);
}

}  // namespace qdcb
