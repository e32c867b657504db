// k_basis.hip -- basis-level device work: contracted normalization,
// primitive-pair (Gaussian product) data and Schwarz factors.
//
// Schwarz factors Q_mn = sqrt((mn|mn)) are the integral part of the
// density-weighted Cauchy-Schwarz bound of Eq. (SchwarzDen); one wavefront
// sums the (K_m K_n)^2 primitive quartets of a pair and reduces them with
// cross-lane shuffles.
#include "kernels.h"

namespace qdcb {

// nc[i] = c_i N(a_i) / sqrt(<chi|chi>) multiplies exp(-a_i r^2) (s),
// (x - A_x) exp(-a_i r^2) (p_x; likewise p_y, p_z) or the monomial
// (x - A_x)^{l_x} (y - A_y)^{l_y} (z - A_z)^{l_z} exp(-a_i r^2) of a d or f
// code, with the primitive normalization
// N(a) = (2a/pi)^{3/4} (4a)^{L/2} / sqrt(prod_k (2 l_k - 1)!!)
// (s: (2a/pi)^{3/4}; p: (2a/pi)^{3/4} 2 sqrt(a)).  Two primitives of one
// function overlap by (pi/q)^{3/2} prod_k (2 l_k - 1)!! / (2q)^{l_k}, q = a + b.
__global__ void k_norm_coefs(int nfunc, const int32_t *first, const double *exps,
                             const double *coefs, const int32_t *cart, double *nc) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfunc) return;
  const int code = cart ? cart[f] : 0;
  const bool pf = code >= 1 && code <= 3, df = code >= 4 && code <= 9, ff = code >= 10;
  // prod_k (2 l_k - 1)!! (1, 3 or 15 per direction)
  double dd = 1.0;
  for (int k = 0; k < 3; ++k) {
    const int l = cart_pow(code, k);
    dd *= l == 3 ? 15.0 : (l == 2 ? 3.0 : 1.0);
  }
  auto nrm = [&](double a) {
    const double n = pow(2.0 * a / PI, 0.75);
    return pf ? 2.0 * sqrt(a) * n
              : (df ? 4.0 * a * n / sqrt(dd) : (ff ? 8.0 * a * sqrt(a) * n / sqrt(dd) : n));
  };
  int i0 = first[f], i1 = first[f + 1];
  double s = 0.0;
  for (int i = i0; i < i1; ++i) {
    double di = coefs[i] * nrm(exps[i]);
    for (int j = i0; j < i1; ++j) {
      double dj = coefs[j] * nrm(exps[j]);
      const double q = exps[i] + exps[j];
      double ov = pow(PI / q, 1.5);
      if (pf) ov /= 2.0 * q;
      if (df) ov *= dd / (4.0 * q * q);
      if (ff) ov *= dd / (8.0 * q * q * q);
      s += di * dj * ov;
    }
  }
  double inv = 1.0 / sqrt(s);
  for (int i = i0; i < i1; ++i) nc[i] = coefs[i] * nrm(exps[i]) * inv;
}

void launch_norm_coefs(int nfunc, const int32_t *first, const double *exps, const double *coefs,
                       const int32_t *cart, double *nc, hipStream_t s) {
  if (nfunc <= 0) return;
  hipLaunchKernelGGL(k_norm_coefs, dim3((nfunc + 127) / 128), dim3(128), 0, s, nfunc, first,
                     exps, coefs, cart, nc);
}

__global__ void k_pair_data(int64_t npairs, const int32_t *mu, const int32_t *nu,
                            const int64_t *pair_first, const double *cA, const int32_t *fA,
                            const double *eA, const double *nA, const int32_t *kA,
                            const double *cB, const int32_t *fB, const double *eB,
                            const double *nB, const int32_t *kB, PrimPairs out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  int m = mu[i], n = nu[i];
  double Ax = cA[3 * m], Ay = cA[3 * m + 1], Az = cA[3 * m + 2];
  double Bx = cB[3 * n], By = cB[3 * n + 1], Bz = cB[3 * n + 2];
  double r2 = (Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By) + (Az - Bz) * (Az - Bz);
  // Cartesian direction of each p function (-1: s or d)
  const int ca = kA ? kA[m] : 0, cb = kB ? kB[n] : 0;
  const int da = ca >= 1 && ca <= 3 ? ca - 1 : -1, db = cb >= 1 && cb <= 3 ? cb - 1 : -1;
  const double Ad = da == 0 ? Ax : (da == 1 ? Ay : Az);
  const double Bd = db == 0 ? Bx : (db == 1 ? By : Bz);
  int64_t o = pair_first[i];
  for (int a = fA[m]; a < fA[m + 1]; ++a)
    for (int b = fB[n]; b < fB[n + 1]; ++b) {
      double ea = eA[a], eb = eB[b];
      double p = ea + eb;
      double ip = 1.0 / p;
      const double Px = (ea * Ax + eb * Bx) * ip, Py = (ea * Ay + eb * By) * ip,
                   Pz = (ea * Az + eb * Bz) * ip;
      out.ip[o] = ip;
      out.x[o] = Px;
      out.y[o] = Py;
      out.z[o] = Pz;
      double pp = PI * ip;
      out.e[o] = nA[a] * nB[b] * exp(-ea * eb * ip * r2) * pp * sqrt(pp);
      if (out.pa) {
        out.pa[o] = da >= 0 ? (da == 0 ? Px : (da == 1 ? Py : Pz)) - Ad : 0.0;
        out.pb[o] = db >= 0 ? (db == 0 ? Px : (db == 1 ? Py : Pz)) - Bd : 0.0;
        out.ax[o] = Px - Ax;
        out.ay[o] = Py - Ay;
        out.az[o] = Pz - Az;
        out.bx[o] = Px - Bx;
        out.by[o] = Py - By;
        out.bz[o] = Pz - Bz;
        // Hermite coefficients of the pair per direction
        const double PA[3] = {Px - Ax, Py - Ay, Pz - Az}, PB[3] = {Px - Bx, Py - By, Pz - Bz};
        for (int d = 0; d < 3; ++d) {
          double Ed[GEN_TMAX + 1];
          herm_1d<GEN_TMAX>(cart_pow(ca, d), cart_pow(cb, d), PA[d], PB[d], 0.5 * ip, Ed);
          for (int t = 0; t <= GEN_TMAX; ++t) out.E[PAIR_E * o + 7 * d + t] = Ed[t];
        }
      }
      ++o;
    }
}

void launch_pair_data(int64_t npairs, const int32_t *mu, const int32_t *nu,
                      const int64_t *pair_first, const double *centA, const int32_t *firstA,
                      const double *expA, const double *ncA, const int32_t *cartA,
                      const double *centB, const int32_t *firstB, const double *expB,
                      const double *ncB, const int32_t *cartB, PrimPairs out, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_pair_data, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s,
                     npairs, mu, nu, pair_first, centA, firstA, expA, ncA, cartA, centB, firstB,
                     expB, ncB, cartB, out);
}

// One wavefront per pair: lanes stride over the (ij, kl) primitive quartets.
// code: pair codes of a Cartesian basis (see common.h), else NULL.
__global__ void __launch_bounds__(256) k_schwarz(int64_t npairs, const int64_t *pair_first,
                                                 PrimPairsC pp, const int32_t *code, double *Q) {
  int lane = threadIdx.x & 63;
  int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pair >= npairs) return;
  int64_t f0 = pair_first[pair];
  int k = (int)(pair_first[pair + 1] - f0);
  double acc = 0.0;
  const int c = code ? code[pair] : 0;
  const bool gen = gen_code(c);  // uniform
  for (int t = lane; t < k * k; t += 64) {
    int64_t i = f0 + t / k, j = f0 + t % k;
    if (gen) {
      const double Pi[3] = {pp.x[i], pp.y[i], pp.z[i]}, Pj[3] = {pp.x[j], pp.y[j], pp.z[j]};
      const double Ai[3] = {pp.ax[i], pp.ay[i], pp.az[i]}, Aj[3] = {pp.ax[j], pp.ay[j], pp.az[j]};
      const double Bi[3] = {pp.bx[i], pp.by[i], pp.bz[i]}, Bj[3] = {pp.bx[j], pp.by[j], pp.bz[j]};
      acc += pp.e[i] * pp.e[j] *
             gen_quartet_exact(pp.ip[i], Pi, Ai, Bi, code_f(c), code_g(c), pp.ip[j], Pj, Aj, Bj,
                               code_f(c), code_g(c));
    } else if (c)
      acc += pp.e[i] * pp.e[j] *
             cart_quartet_exact(pp.ip[i], pp.x[i], pp.y[i], pp.z[i], pp.pa[i], pp.pb[i], c,
                                pp.ip[j], pp.x[j], pp.y[j], pp.z[j], pp.pa[j], pp.pb[j], c);
    else
      acc += prim_quartet(pp.ip[i], pp.x[i], pp.y[i], pp.z[i], pp.e[i], pp.ip[j], pp.x[j],
                          pp.y[j], pp.z[j], pp.e[j]);
  }
  acc = wave_sum(acc);
  if (lane == 0) Q[pair] = sqrt(acc);
}

void launch_schwarz(int64_t npairs, const int64_t *pair_first, PrimPairsC pp,
                    const int32_t *code, double *Q, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_schwarz, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, s, npairs,
                     pair_first, pp, code, Q);
}

// Primitive-pair screening.  With q_i = |e_i| p_i^{1/4} proportional to the
// primitive Schwarz factor sqrt([i|i]) and S = sum_i q_i over the n primitive
// pairs of a row, a primitive pair with q_i <= eps S / n is dropped.  Every
// primitive integral obeys |[i|k]| <= sqrt([i|i][k|k]), so the dropped part of
// any contracted integral (A|B) is at most 2 eps S_A S_B in Schwarz units:
// about eps of the sum of its absolute primitive contributions.  Rows of
// pairs with a p, d or f function keep every primitive pair (code[r] != 0), since
// their primitive Schwarz factors are not proportional to q_i.
__device__ __forceinline__ double prim_weight(const PrimPairsC &s, int64_t i) {
  return fabs(s.e[i]) * sqrt(sqrt(1.0 / s.ip[i]));
}

__device__ __forceinline__ double row_cut(const PrimPairsC &s, int64_t s0, int n, double eps) {
  double S = 0.0;
  for (int i = 0; i < n; ++i) S += prim_weight(s, s0 + i);
  return eps * S / (double)(n > 0 ? n : 1);
}

__global__ void k_prim_count(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                             const int32_t *code, PrimPairsC src, double eps, int32_t *kept) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t s0 = src_first[r];
  const int n = cnt[r];
  const double cut = (code && code[r]) ? -1.0 : row_cut(src, s0, n, eps);
  int k = 0;
  for (int i = 0; i < n; ++i) k += prim_weight(src, s0 + i) > cut ? 1 : 0;
  kept[r] = k;
}

void launch_prim_count(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                       const int32_t *code, PrimPairsC src, double eps, int32_t *kept,
                       hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_prim_count, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s, nrows,
                     src_first, cnt, code, src, eps, kept);
}

__global__ void k_gather_pairs(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                               const int32_t *code, const int64_t *dst_first, PrimPairsC src,
                               PrimPairs dst, double eps) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t s0 = src_first[r];
  const int n = cnt[r];
  const double cut = (code && code[r]) ? -1.0 : row_cut(src, s0, n, eps);
  int64_t d = dst_first[r];
  for (int i = 0; i < n; ++i) {
    const int64_t si = s0 + i;
    if (!(prim_weight(src, si) > cut)) continue;
    dst.ip[d] = src.ip[si];
    dst.x[d] = src.x[si];
    dst.y[d] = src.y[si];
    dst.z[d] = src.z[si];
    dst.e[d] = src.e[si];
    if (dst.pa) {  // a store of an s-only basis has no pa / pb (its codes are 0)
      const bool c = src.pa != nullptr;
      dst.pa[d] = c ? src.pa[si] : 0.0;
      dst.pb[d] = c ? src.pb[si] : 0.0;
      dst.ax[d] = c ? src.ax[si] : 0.0;
      dst.ay[d] = c ? src.ay[si] : 0.0;
      dst.az[d] = c ? src.az[si] : 0.0;
      dst.bx[d] = c ? src.bx[si] : 0.0;
      dst.by[d] = c ? src.by[si] : 0.0;
      dst.bz[d] = c ? src.bz[si] : 0.0;
      // an s pair's coefficients: E_0 = 1 in each direction
      for (int k = 0; k < PAIR_E; ++k)
        dst.E[PAIR_E * d + k] = c ? src.E[PAIR_E * si + k] : (k % 7 == 0 ? 1.0 : 0.0);
    }
    ++d;
  }
}

void launch_gather_pairs(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                         const int32_t *code, const int64_t *dst_first, PrimPairsC src,
                         PrimPairs dst, double eps, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_gather_pairs, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s,
                     nrows, src_first, cnt, code, dst_first, src, dst, eps);
}

// codes (NULL for two s-only bases): per quartet, the bra and ket pair codes
__global__ void k_eri_list(int64_t nq, const int64_t *af, const int64_t *bf, const int32_t *ac,
                           const int32_t *bc, const int32_t *codes, PrimPairsC A, PrimPairsC B,
                           double *out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  if (codes && (gen_code(codes[2 * q]) || gen_code(codes[2 * q + 1])))
    out[q] = contracted_eri_gen(A, af[q], af[q] + ac[q], codes[2 * q], B, bf[q], bf[q] + bc[q],
                                codes[2 * q + 1]);
  else if (codes)
    out[q] = contracted_eri_cart(A, af[q], af[q] + ac[q], codes[2 * q], B, bf[q], bf[q] + bc[q],
                                 codes[2 * q + 1]);
  else
    out[q] = contracted_eri(A, af[q], af[q] + ac[q], B, bf[q], bf[q] + bc[q]);
}

void launch_eri_list(int64_t nq, const int64_t *a_first, const int64_t *b_first,
                     const int32_t *a_cnt, const int32_t *b_cnt, const int32_t *codes,
                     PrimPairsC A, PrimPairsC B, double *out, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_eri_list, dim3((unsigned)((nq + 127) / 128)), dim3(128), 0, s, nq,
                     a_first, b_first, a_cnt, b_cnt, codes, A, B, out);
}

}  // namespace qdcb
