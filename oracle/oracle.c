/* oracle.c -- plain FP64 CPU oracle for the quaternion AO->MO two-electron
 * integral transformation (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Written for checkability, not speed: every quantity is computed from its
 * textbook or paper definition with no blocking, fusion or reordering beyond
 * what that definition states.  Complex arithmetic is C99 `double complex`.
 *
 * Paper references (arXiv 2606.04316):
 *   Sec. 2, notation           alpha_K = [[0, sigma_K], [sigma_K, 0]] and the
 *                              Pauli matrices as printed.
 *   Eq. (breit)                Gaunt (magnetic) term -alpha_1 . alpha_2 / r12
 *                              and the gauge term
 *                              (alpha_1 x r12) . (alpha_2 x r12) / (2 r12^3).
 *   Eq. (gaugeInt)             the gauge integrals: L/S classes of the
 *                              r12 r12^T / r12^3 kernel.
 *   Eqs. (Lspinor), (Sspinor)  two-spinor expansions of the L and S parts.
 *   Eq. (AOtoMO), (DCInt),     the MO integrals as sums over AO integrals and
 *   (GauntInt)                 the L/S class decomposition.
 *   Eq. (Den)                  density matrix D_{nu mu} = sum_i c*_{mu i} c_{nu i}.
 *   Eq. (QuaternionScatter)    Pauli components D_s, D_x, D_y, D_z.
 *   Eq. (firsthalf)            first-half contraction of AO integrals with
 *                              pair densities.
 *   Sec. 2.4.2, Eq. (secondhalf)  Pauli -> two-spinor block conversion and the
 *                              two-spinor second half as two matrix products.
 *   Eq. (SchwarzDen)           density-weighted Cauchy-Schwarz bound.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Boys function and AO integrals over s- and p-type Gaussians              */
/* ------------------------------------------------------------------------ */

/* F0(T) = int_0^1 exp(-T u^2) du = (1/2) sqrt(pi/T) erf(sqrt(T)); the first
 * two terms of its Taylor series are used where T is too small for the
 * closed form to be evaluated (T = 0 for concentric charge distributions). */
double orc_boys0(double T)
{
    if (T < 1e-12) return 1.0 - T / 3.0;
    return 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
}

/* F_m(T) = int_0^1 u^{2m} exp(-T u^2) du.  Below T = 30 from the series of
 * positive terms F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1));
 * from T = 30 on, upward from the erf form of F0 by
 * F_{j+1} = ((2j+1) F_j - exp(-T)) / (2T), where exp(-T) is negligible next
 * to the terms it is subtracted from. */
double orc_boys(int m, double T)
{
    if (T < 30.0) {
        double term = 1.0 / (2 * m + 1), sum = term;
        for (int k = 1; k < 400; ++k) {
            term *= 2.0 * T / (2 * m + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return exp(-T) * sum;
    }
    double f = orc_boys0(T), e = exp(-T);
    for (int j = 0; j < m; ++j) f = ((2 * j + 1) * f - e) / (2.0 * T);
    return f;
}

static int64_t *prim_offsets(const orc_basis *b)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(b->nfunc + 1));
    off[0] = 0;
    for (int f = 0; f < b->nfunc; ++f) off[f + 1] = off[f] + b->nprim[f];
    return off;
}

static int cart_of(const orc_basis *b, int f) { return b->cart ? b->cart[f] : 0; }

static int carts_valid(const orc_basis *b)
{
    for (int f = 0; b && b->cart && f < b->nfunc; ++f)
        if (b->cart[f] < 0 || b->cart[f] > 19) return 0;
    return 1;
}

/* Cartesian exponents of a function code: 0 = s; 1, 2, 3 = p_x, p_y, p_z;
 * 4 .. 9 = d_xx, d_yy, d_zz, d_xy, d_xz, d_yz; 10 .. 19 = f_xxx, f_yyy, f_zzz,
 * f_xxy, f_xxz, f_xyy, f_yyz, f_xzz, f_yzz, f_xyz. */
static void cart_powers(int code, int l[3])
{
    static const int tab[20][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                   {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                                   {3, 0, 0}, {0, 3, 0}, {0, 0, 3}, {2, 1, 0}, {2, 0, 1},
                                   {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {1, 1, 1}};
    for (int k = 0; k < 3; ++k) l[k] = tab[code][k];
}

/* (2l - 1)!! for l = 0 .. 3 */
static double dfact(int l) { return l == 3 ? 15.0 : (l == 2 ? 3.0 : 1.0); }

/* Normalized primitive (x-A_x)^lx (y-A_y)^ly (z-A_z)^lz exp(-a r^2) with
 * N = (2a/pi)^{3/4} (4a)^{L/2} / sqrt((2lx-1)!! (2ly-1)!! (2lz-1)!!),
 * L = lx + ly + lz: the square of the unnormalized primitive integrates to
 * (pi/(2a))^{3/2} prod_k (2l_k-1)!! / (4a)^{l_k}.  Overlap of two
 * unnormalized primitives of one function (same centre and factor),
 * exponents a, b, p = a + b: (pi/p)^{3/2} prod_k (2l_k-1)!! / (2p)^{l_k}. */
static double prim_norm(double a, int cart)
{
    int l[3];
    cart_powers(cart, l);
    double n = pow(2.0 * a / M_PI, 0.75);
    for (int k = 0; k < 3; ++k) n *= pow(4.0 * a, 0.5 * l[k]) / sqrt(dfact(l[k]));
    return n;
}

static double prim_overlap_same(double p, int cart)
{
    int l[3];
    cart_powers(cart, l);
    double ov = pow(M_PI / p, 1.5);
    for (int k = 0; k < 3; ++k) ov *= dfact(l[k]) / pow(2.0 * p, l[k]);
    return ov;
}

void orc_norm_coefs(const orc_basis *b, double *out)
{
    int64_t *off = prim_offsets(b);
    for (int f = 0; f < b->nfunc; ++f) {
        int c = cart_of(b, f);
        double s = 0.0;
        for (int64_t i = off[f]; i < off[f + 1]; ++i)
            for (int64_t j = off[f]; j < off[f + 1]; ++j) {
                double di = b->coefs[i] * prim_norm(b->exps[i], c);
                double dj = b->coefs[j] * prim_norm(b->exps[j], c);
                s += di * dj * prim_overlap_same(b->exps[i] + b->exps[j], c);
            }
        for (int64_t i = off[f]; i < off[f + 1]; ++i)
            out[i] = b->coefs[i] * prim_norm(b->exps[i], c) / sqrt(s);
    }
    free(off);
}

/* Primitive ERIs over unnormalized Cartesian Gaussians
 * (x-A_x)^{a_x} (y-A_y)^{a_y} (z-A_z)^{a_z} exp(-a|r-A|^2), by the recursion
 * of Obara and Saika (J. Chem. Phys. 84, 3963 (1986)): the vertical relation
 * builds [a0|c0]^(m) from the auxiliary integrals
 * [00|00]^(m) = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd F_m(T), and the
 * horizontal relations [a, b+1_i | cd] = [a+1_i, b | cd] + (A-B)_i [ab|cd]
 * (likewise on the ket) move angular momentum onto the second centre of
 * each pair.  Notation: p = a+b, P = (aA+bB)/p, q = c+d, Q = (cC+dD)/q,
 * W = (pP+qQ)/(p+q), rho = pq/(p+q), T = rho |P-Q|^2. */
typedef struct {
    double p, q, rho;
    double PA[3], QC[3], WP[3], WQ[3], AB[3], CD[3];
    double aux[13]; /* [00|00]^(m), m = 0..12 (four f functions) */
} os_data;

static double os_vrr(const os_data *o, const int a[3], const int c[3], int m)
{
    int i;
    for (i = 0; i < 3; ++i)
        if (a[i] > 0) break;
    if (i < 3) {
        int a1[3] = {a[0], a[1], a[2]};
        a1[i] -= 1;
        double v = o->PA[i] * os_vrr(o, a1, c, m) + o->WP[i] * os_vrr(o, a1, c, m + 1);
        if (a1[i] > 0) {
            int a2[3] = {a1[0], a1[1], a1[2]};
            a2[i] -= 1;
            v += a1[i] / (2.0 * o->p) *
                 (os_vrr(o, a2, c, m) - o->rho / o->p * os_vrr(o, a2, c, m + 1));
        }
        if (c[i] > 0) {
            int c1[3] = {c[0], c[1], c[2]};
            c1[i] -= 1;
            v += c[i] / (2.0 * (o->p + o->q)) * os_vrr(o, a1, c1, m + 1);
        }
        return v;
    }
    for (i = 0; i < 3; ++i)
        if (c[i] > 0) break;
    if (i < 3) {
        int c1[3] = {c[0], c[1], c[2]};
        c1[i] -= 1;
        double v = o->QC[i] * os_vrr(o, a, c1, m) + o->WQ[i] * os_vrr(o, a, c1, m + 1);
        if (c1[i] > 0) {
            int c2[3] = {c1[0], c1[1], c1[2]};
            c2[i] -= 1;
            v += c1[i] / (2.0 * o->q) *
                 (os_vrr(o, a, c2, m) - o->rho / o->q * os_vrr(o, a, c2, m + 1));
        }
        return v;
    }
    return o->aux[m];
}

static double os_eri(const os_data *o, const int a[3], const int b[3], const int c[3],
                     const int d[3])
{
    for (int i = 0; i < 3; ++i)
        if (b[i] > 0) {
            int a1[3] = {a[0], a[1], a[2]}, b1[3] = {b[0], b[1], b[2]};
            a1[i] += 1;
            b1[i] -= 1;
            return os_eri(o, a1, b1, c, d) + o->AB[i] * os_eri(o, a, b1, c, d);
        }
    for (int i = 0; i < 3; ++i)
        if (d[i] > 0) {
            int c1[3] = {c[0], c[1], c[2]}, d1[3] = {d[0], d[1], d[2]};
            c1[i] += 1;
            d1[i] -= 1;
            return os_eri(o, a, b, c1, d1) + o->CD[i] * os_eri(o, a, b, c, d1);
        }
    return os_vrr(o, a, c, 0);
}

double orc_prim_eri_cart(double a, const double *A, int ca, double b, const double *B, int cb,
                         double c, const double *C, int cc, double d, const double *D, int cd)
{
    os_data o;
    double p = a + b, q = c + d, rab2 = 0, rcd2 = 0, rpq2 = 0;
    o.p = p;
    o.q = q;
    o.rho = p * q / (p + q);
    for (int k = 0; k < 3; ++k) {
        double P = (a * A[k] + b * B[k]) / p;
        double Q = (c * C[k] + d * D[k]) / q;
        double W = (p * P + q * Q) / (p + q);
        o.PA[k] = P - A[k];
        o.QC[k] = Q - C[k];
        o.WP[k] = W - P;
        o.WQ[k] = W - Q;
        o.AB[k] = A[k] - B[k];
        o.CD[k] = C[k] - D[k];
        rab2 += o.AB[k] * o.AB[k];
        rcd2 += o.CD[k] * o.CD[k];
        rpq2 += (P - Q) * (P - Q);
    }
    double pre = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * exp(-a * b / p * rab2) *
                 exp(-c * d / q * rcd2);
    double T = o.rho * rpq2;
    for (int m = 0; m < 13; ++m) o.aux[m] = pre * orc_boys(m, T);
    int la[3], lb[3], lc[3], ld[3];
    cart_powers(ca, la);
    cart_powers(cb, lb);
    cart_powers(cc, lc);
    cart_powers(cd, ld);
    return os_eri(&o, la, lb, lc, ld);
}

/* Primitive ERI over unnormalized s Gaussians exp(-a|r-A|^2) ... :
 * [ab|cd] = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd F0(p q/(p+q) |P-Q|^2),
 * p = a+b, P = (aA+bB)/p, K_ab = exp(-ab/p |A-B|^2). */
static double prim_eri(double a, const double *A, double b, const double *B, double c,
                       const double *C, double d, const double *D)
{
    double p = a + b, q = c + d;
    double rab2 = 0, rcd2 = 0, rpq2 = 0;
    for (int k = 0; k < 3; ++k) {
        double P = (a * A[k] + b * B[k]) / p;
        double Q = (c * C[k] + d * D[k]) / q;
        rab2 += (A[k] - B[k]) * (A[k] - B[k]);
        rcd2 += (C[k] - D[k]) * (C[k] - D[k]);
        rpq2 += (P - Q) * (P - Q);
    }
    double T = p * q / (p + q) * rpq2;
    return 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * exp(-a * b / p * rab2) *
           exp(-c * d / q * rcd2) * orc_boys0(T);
}

/* Primitive integrals of the kernel r12_K r12_L / r12^3 (the gauge
 * integrals' kernel, Eq. (gaugeInt)) over unnormalized s Gaussians:
 *   [ab|K L|cd] = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd
 *                 (delta_KL F1(T) + 2 rho R_K R_L (F1(T) - F2(T))),
 * R = P - Q, rho = p q / (p + q), T = rho R^2.  Derivation: write
 * 1/r^3 = (4/sqrt(pi)) int_0^inf s^2 exp(-s^2 r^2) ds, integrate the
 * Gaussian product over the electron coordinates, and substitute
 * t^2 = s^2 / (rho + s^2), which turns the s integral into Boys functions.
 * The trace over K = L is the Coulomb integral (3 F1 + 2T (F1 - F2) = F0). */
static void prim_eri3(double a, const double *A, double b, const double *B, double c,
                      const double *C, double d, const double *D, double out[9])
{
    double p = a + b, q = c + d, R[3];
    double rab2 = 0, rcd2 = 0, rpq2 = 0;
    for (int k = 0; k < 3; ++k) {
        double P = (a * A[k] + b * B[k]) / p;
        double Q = (c * C[k] + d * D[k]) / q;
        rab2 += (A[k] - B[k]) * (A[k] - B[k]);
        rcd2 += (C[k] - D[k]) * (C[k] - D[k]);
        R[k] = P - Q;
        rpq2 += R[k] * R[k];
    }
    double rho = p * q / (p + q), T = rho * rpq2;
    double pre = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * exp(-a * b / p * rab2) *
                 exp(-c * d / q * rcd2);
    double F1 = orc_boys(1, T), F2 = orc_boys(2, T);
    for (int K = 0; K < 3; ++K)
        for (int L = 0; L < 3; ++L)
            out[K * 3 + L] = pre * ((K == L ? F1 : 0.0) + 2.0 * rho * R[K] * R[L] * (F1 - F2));
}

/* Gauge-kernel integrals over unnormalized Cartesian Gaussians,
 * out[K * 3 + L] = [ab| r12_K r12_L / r12^3 |cd], in McMurchie-Davidson form
 * (a different method from the Obara-Saika recursion of the Coulomb
 * integrals; the two meet in the trace, sum_K [ab|KK|cd] = [ab|cd]).
 * Per direction the product of a pair's two functions is a sum of Hermite
 * Gaussians with the coefficients E^{ij}_t of the recursion
 *   E^{i+1,j}_t = E^{ij}_{t-1} / (2p) + (P - A) E^{ij}_t + (t + 1) E^{ij}_{t+1}
 * (likewise j with P - B), E^{00}_0 = 1.  For Hermite Gaussians of orders t
 * at P and u at Q the integral is (-1)^{|u|} times the derivative of orders
 * t + u, with respect to X = P - Q, of the kernel of two s distributions
 * (prim_eri3)
 *   W_KL(X) = pre (delta_KL F1(rho X^2) + 2 rho X_K X_L (F1 - F2)(rho X^2)).
 * The derivatives of F_k(rho X^2) come from the Hermite recursion
 * R^{(n)}_{t+1,u,v} = t R^{(n+1)}_{t-1,u,v} + X_x R^{(n+1)}_{t,u,v} (likewise
 * u, v) with R^{(n)}_{000} = (-2 rho)^n F_{k+n}, and those of X_K X_L g by
 * the Leibniz rule. */
#define GMAXL 12 /* highest total Hermite order (four f functions) */
#define GDIM (GMAXL + 1)

static void herm_E_table(double PA, double PB, double p, double E[4][4][7])
{
    memset(E, 0, sizeof(double) * 4 * 4 * 7);
    E[0][0][0] = 1.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            if (i == 0 && j == 0) continue;
            /* raise i from (i - 1, j) when i > 0, else j from (i, j - 1) */
            const double(*src)[7] = i > 0 ? &E[i - 1][j] : &E[i][j - 1];
            const double X = i > 0 ? PA : PB;
            for (int t = 0; t < 7; ++t) {
                double v = X * (*src)[t];
                if (t + 1 < 7) v += (t + 1) * (*src)[t + 1];
                if (t > 0) v += (*src)[t - 1] / (2.0 * p);
                E[i][j][t] = v;
            }
        }
}

/* R^{(0)}_{tuv} for t + u + v <= L of F_k(rho X^2), out[(t * GDIM + u) * GDIM + v]. */
static void herm_R_table(int k, double rho, const double X[3], double T, int L, double *out)
{
    double *R = (double *)calloc((size_t)(L + 1) * GDIM * GDIM * GDIM, sizeof(double));
#define RI(n, t, u, v) R[(((size_t)(n) * GDIM + (t)) * GDIM + (u)) * GDIM + (v)]
    for (int n = 0; n <= L; ++n) RI(n, 0, 0, 0) = pow(-2.0 * rho, n) * orc_boys(k + n, T);
    for (int n = L - 1; n >= 0; --n)
        for (int t = 0; t <= L - n; ++t)
            for (int u = 0; t + u <= L - n; ++u)
                for (int v = 0; t + u + v <= L - n; ++v) {
                    if (t > 0)
                        RI(n, t, u, v) = (t > 1 ? (t - 1) * RI(n + 1, t - 2, u, v) : 0.0) +
                                         X[0] * RI(n + 1, t - 1, u, v);
                    else if (u > 0)
                        RI(n, t, u, v) = (u > 1 ? (u - 1) * RI(n + 1, t, u - 2, v) : 0.0) +
                                         X[1] * RI(n + 1, t, u - 1, v);
                    else if (v > 0)
                        RI(n, t, u, v) = (v > 1 ? (v - 1) * RI(n + 1, t, u, v - 2) : 0.0) +
                                         X[2] * RI(n + 1, t, u, v - 1);
                }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; t + u <= L; ++u)
            for (int v = 0; t + u + v <= L; ++v) out[(t * GDIM + u) * GDIM + v] = RI(0, t, u, v);
#undef RI
    free(R);
}

void orc_prim_eri3_cart(double a, const double *A, int ca, double b, const double *B, int cb,
                        double c, const double *C, int cc, double d, const double *D, int cd,
                        double out[9])
{
    int la[3], lb[3], lc[3], ld[3];
    cart_powers(ca, la);
    cart_powers(cb, lb);
    cart_powers(cc, lc);
    cart_powers(cd, ld);
    const double p = a + b, q = c + d, rho = p * q / (p + q);
    double X[3], Eb[3][4][4][7], Ek[3][4][4][7], rab2 = 0, rcd2 = 0, x2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double P = (a * A[k] + b * B[k]) / p, Q = (c * C[k] + d * D[k]) / q;
        herm_E_table(P - A[k], P - B[k], p, Eb[k]);
        herm_E_table(Q - C[k], Q - D[k], q, Ek[k]);
        X[k] = P - Q;
        x2 += X[k] * X[k];
        rab2 += (A[k] - B[k]) * (A[k] - B[k]);
        rcd2 += (C[k] - D[k]) * (C[k] - D[k]);
    }
    const double pre = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * exp(-a * b / p * rab2) *
                       exp(-c * d / q * rcd2);
    int L = 0;
    for (int k = 0; k < 3; ++k) L += la[k] + lb[k] + lc[k] + ld[k];
    const size_t nr = (size_t)GDIM * GDIM * GDIM;
    double *R1 = (double *)calloc(nr, sizeof(double)), *G = (double *)calloc(nr, sizeof(double));
    herm_R_table(1, rho, X, rho * x2, L, R1);
    herm_R_table(2, rho, X, rho * x2, L, G);
    for (size_t i = 0; i < nr; ++i) G[i] = R1[i] - G[i]; /* derivatives of F1 - F2 */
#define AT(arr, t, u, v) ((t) < 0 || (u) < 0 || (v) < 0 ? 0.0 : (arr)[((t) * GDIM + (u)) * GDIM + (v)])
    for (int K = 0; K < 3; ++K)
        for (int Lc = 0; Lc < 3; ++Lc) {
            double sum = 0.0;
            for (int t0 = 0; t0 <= la[0] + lb[0]; ++t0)
                for (int t1 = 0; t1 <= la[1] + lb[1]; ++t1)
                    for (int t2 = 0; t2 <= la[2] + lb[2]; ++t2) {
                        const double eb = Eb[0][la[0]][lb[0]][t0] * Eb[1][la[1]][lb[1]][t1] *
                                          Eb[2][la[2]][lb[2]][t2];
                        if (eb == 0.0) continue;
                        for (int u0 = 0; u0 <= lc[0] + ld[0]; ++u0)
                            for (int u1 = 0; u1 <= lc[1] + ld[1]; ++u1)
                                for (int u2 = 0; u2 <= lc[2] + ld[2]; ++u2) {
                                    const double ek = Ek[0][lc[0]][ld[0]][u0] *
                                                      Ek[1][lc[1]][ld[1]][u1] *
                                                      Ek[2][lc[2]][ld[2]][u2];
                                    if (ek == 0.0) continue;
                                    const int n[3] = {t0 + u0, t1 + u1, t2 + u2};
                                    const double sg = ((u0 + u1 + u2) & 1) ? -1.0 : 1.0;
                                    /* derivative of orders n of delta_KL F1 + 2 rho X_K X_L g */
                                    double w = K == Lc ? AT(R1, n[0], n[1], n[2]) : 0.0;
                                    int m1[3] = {n[0], n[1], n[2]}, m2[3] = {n[0], n[1], n[2]},
                                        m12[3] = {n[0], n[1], n[2]};
                                    double lz;
                                    if (K != Lc) {
                                        m1[K] -= 1;
                                        m2[Lc] -= 1;
                                        m12[K] -= 1;
                                        m12[Lc] -= 1;
                                        lz = X[K] * X[Lc] * AT(G, n[0], n[1], n[2]) +
                                             n[K] * X[Lc] * AT(G, m1[0], m1[1], m1[2]) +
                                             n[Lc] * X[K] * AT(G, m2[0], m2[1], m2[2]) +
                                             n[K] * n[Lc] * AT(G, m12[0], m12[1], m12[2]);
                                    } else {
                                        m1[K] -= 1;
                                        m2[K] -= 2;
                                        lz = X[K] * X[K] * AT(G, n[0], n[1], n[2]) +
                                             2.0 * n[K] * X[K] * AT(G, m1[0], m1[1], m1[2]) +
                                             n[K] * (n[K] - 1) * AT(G, m2[0], m2[1], m2[2]);
                                    }
                                    w += 2.0 * rho * lz;
                                    sum += sg * eb * ek * w;
                                }
                    }
            out[K * 3 + Lc] = pre * sum;
        }
#undef AT
    free(R1);
    free(G);
}

/* Contracted ERI with per-basis normalized coefficient arrays; s-type
 * quartets take the closed form, quartets with a p function the recursion. */
static double eri4(const orc_basis *A, const double *nA, const int64_t *oA, int i,
                   const orc_basis *B, const double *nB, const int64_t *oB, int j,
                   const orc_basis *C, const double *nC, const int64_t *oC, int k,
                   const orc_basis *D, const double *nD, const int64_t *oD, int l)
{
    int ca = cart_of(A, i), cb = cart_of(B, j), cc = cart_of(C, k), cd = cart_of(D, l);
    int ang = ca || cb || cc || cd;
    double s = 0.0;
    for (int64_t pi = oA[i]; pi < oA[i + 1]; ++pi)
        for (int64_t pj = oB[j]; pj < oB[j + 1]; ++pj)
            for (int64_t pk = oC[k]; pk < oC[k + 1]; ++pk)
                for (int64_t pl = oD[l]; pl < oD[l + 1]; ++pl) {
                    double w = nA[pi] * nB[pj] * nC[pk] * nD[pl];
                    if (ang)
                        s += w * orc_prim_eri_cart(A->exps[pi], A->centers + 3 * i, ca,
                                                   B->exps[pj], B->centers + 3 * j, cb,
                                                   C->exps[pk], C->centers + 3 * k, cc,
                                                   D->exps[pl], D->centers + 3 * l, cd);
                    else
                        s += w * prim_eri(A->exps[pi], A->centers + 3 * i, B->exps[pj],
                                          B->centers + 3 * j, C->exps[pk], C->centers + 3 * k,
                                          D->exps[pl], D->centers + 3 * l);
                }
    return s;
}

/* Contracted r12 r12^T / r12^3 integrals, out[K * 3 + L]; s-type quartets
 * take the closed form, quartets with a Cartesian function the Hermite form. */
static void eri4_3(const orc_basis *A, const double *nA, const int64_t *oA, int i,
                   const orc_basis *B, const double *nB, const int64_t *oB, int j,
                   const orc_basis *C, const double *nC, const int64_t *oC, int k,
                   const orc_basis *D, const double *nD, const int64_t *oD, int l, double out[9])
{
    int ca = cart_of(A, i), cb = cart_of(B, j), cc = cart_of(C, k), cd = cart_of(D, l);
    int ang = ca || cb || cc || cd;
    for (int c = 0; c < 9; ++c) out[c] = 0.0;
    for (int64_t pi = oA[i]; pi < oA[i + 1]; ++pi)
        for (int64_t pj = oB[j]; pj < oB[j + 1]; ++pj)
            for (int64_t pk = oC[k]; pk < oC[k + 1]; ++pk)
                for (int64_t pl = oD[l]; pl < oD[l + 1]; ++pl) {
                    double t[9], w = nA[pi] * nB[pj] * nC[pk] * nD[pl];
                    if (ang)
                        orc_prim_eri3_cart(A->exps[pi], A->centers + 3 * i, ca, B->exps[pj],
                                           B->centers + 3 * j, cb, C->exps[pk],
                                           C->centers + 3 * k, cc, D->exps[pl],
                                           D->centers + 3 * l, cd, t);
                    else
                        prim_eri3(A->exps[pi], A->centers + 3 * i, B->exps[pj],
                                  B->centers + 3 * j, C->exps[pk], C->centers + 3 * k,
                                  D->exps[pl], D->centers + 3 * l, t);
                    for (int c = 0; c < 9; ++c) out[c] += w * t[c];
                }
}

typedef struct {
    const orc_basis *b;
    double *nc;
    int64_t *off;
} nbasis;

static nbasis nb_make(const orc_basis *b)
{
    nbasis r;
    r.b = b;
    int64_t *off = prim_offsets(b);
    r.off = off;
    r.nc = (double *)malloc(sizeof(double) * (size_t)(off[b->nfunc] > 0 ? off[b->nfunc] : 1));
    orc_norm_coefs(b, r.nc);
    return r;
}

static void nb_free(nbasis *r)
{
    free(r->nc);
    free(r->off);
}

static double nb_eri(const nbasis *A, int i, const nbasis *B, int j, const nbasis *C, int k,
                     const nbasis *D, int l)
{
    return eri4(A->b, A->nc, A->off, i, B->b, B->nc, B->off, j, C->b, C->nc, C->off, k, D->b,
                D->nc, D->off, l);
}

static void nb_eri3(const nbasis *A, int i, const nbasis *B, int j, const nbasis *C, int k,
                    const nbasis *D, int l, double out[9])
{
    eri4_3(A->b, A->nc, A->off, i, B->b, B->nc, B->off, j, C->b, C->nc, C->off, k, D->b, D->nc,
           D->off, l, out);
}

void orc_eri3(const orc_basis *A, int mu, const orc_basis *B, int nu, const orc_basis *C, int ka,
              const orc_basis *D, int la, double out[9])
{
    nbasis a = nb_make(A), b = nb_make(B), c = nb_make(C), d = nb_make(D);
    nb_eri3(&a, mu, &b, nu, &c, ka, &d, la, out);
    nb_free(&a);
    nb_free(&b);
    nb_free(&c);
    nb_free(&d);
}

double orc_eri(const orc_basis *A, int mu, int nu, const orc_basis *B, int ka, int la)
{
    nbasis a = nb_make(A), b = nb_make(B);
    double v = nb_eri(&a, mu, &a, nu, &b, ka, &b, la);
    nb_free(&a);
    nb_free(&b);
    return v;
}

void orc_eri_tensor(const orc_basis *A, const orc_basis *B, const orc_basis *C,
                    const orc_basis *D, double *out)
{
    nbasis a = nb_make(A), b = nb_make(B), c = nb_make(C), d = nb_make(D);
    int NA = A->nfunc, NB = B->nfunc, NC = C->nfunc, ND = D->nfunc;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < NA; ++i)
        for (int j = 0; j < NB; ++j)
            for (int k = 0; k < NC; ++k)
                for (int l = 0; l < ND; ++l)
                    out[(((size_t)i * NB + j) * NC + k) * ND + l] =
                        nb_eri(&a, i, &b, j, &c, k, &d, l);
    nb_free(&a);
    nb_free(&b);
    nb_free(&c);
    nb_free(&d);
}

void orc_schwarz(const orc_basis *A, const orc_basis *B, double *Q)
{
    nbasis a = nb_make(A), b = nb_make(B);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < A->nfunc; ++i)
        for (int j = 0; j < B->nfunc; ++j)
            Q[(size_t)i * B->nfunc + j] = sqrt(nb_eri(&a, i, &b, j, &a, i, &b, j));
    nb_free(&a);
    nb_free(&b);
}

/* Terms of each ham code: 0 LL, 1 DC, 2 DCG, 3 Gaunt alone, 4 DCB (DC + Gaunt
 * + gauge), 5 gauge alone. */
static int ham_coulomb(int ham) { return ham == 0 || ham == 1 || ham == 2 || ham == 4; }
static int ham_ls(int ham) { return ham >= 2 && ham <= 5; }
static int ham_gaunt(int ham) { return ham == 2 || ham == 3 || ham == 4; }
static int ham_gauge(int ham) { return ham == 4 || ham == 5; }

/* Levi-Civita symbol over {0, 1, 2} = {x, y, z}. */
static int levi(int i, int j, int k) { return (i - j) * (j - k) * (k - i) / 2; }

/* ------------------------------------------------------------------------ */
/* Quaternions, the 2x2 spinor representation and Pauli matrices              */
/* ------------------------------------------------------------------------ */

/* Q(q) = q0 I + q1 (i sigma_z) + q2 (i sigma_y) + q3 (i sigma_x). */
static void qrep(const double q[4], cplx M[2][2])
{
    M[0][0] = q[0] + I * q[1];
    M[0][1] = q[2] + I * q[3];
    M[1][0] = -q[2] + I * q[3];
    M[1][1] = q[0] - I * q[1];
}

/* Pauli matrices as printed in Sec. 2: index 0 = x, 1 = y, 2 = z. */
static const cplx *pauli(int K)
{
    static cplx s[3][2][2];
    static int init = 0;
    if (!init) {
        s[0][0][0] = 0; s[0][0][1] = 1; s[0][1][0] = 1; s[0][1][1] = 0;
        s[1][0][0] = 0; s[1][0][1] = -I; s[1][1][0] = I; s[1][1][1] = 0;
        s[2][0][0] = 1; s[2][0][1] = 0; s[2][1][0] = 0; s[2][1][1] = -1;
        init = 1;
    }
    return &s[K][0][0];
}

/* Two-spinor coefficients c[mu][tau][a] (a over 2n spinors) from planar
 * quaternion C[4][N][n]: the columns of Q(C_{mu p}) are spinors 2p, 2p+1. */
static cplx *spinor_coefs(int N, int n, const double *C)
{
    cplx *c = (cplx *)calloc((size_t)N * 2 * 2 * n, sizeof(cplx));
    for (int mu = 0; mu < N; ++mu)
        for (int p = 0; p < n; ++p) {
            double q[4];
            cplx M[2][2];
            for (int z = 0; z < 4; ++z) q[z] = C[((size_t)z * N + mu) * n + p];
            qrep(q, M);
            for (int tau = 0; tau < 2; ++tau)
                for (int s = 0; s < 2; ++s)
                    c[((size_t)mu * 2 + tau) * 2 * n + 2 * p + s] = M[tau][s];
        }
    return c;
}

/* Two-spinor coefficients c[mu][tau][a] of m general (Kramers-unrestricted)
 * spinors from planes C[4][N][m]: alpha re, alpha im, beta re, beta im. */
static cplx *spinor_coefs_general(int N, int m, const double *C)
{
    cplx *c = (cplx *)calloc((size_t)N * 2 * m, sizeof(cplx));
    for (int mu = 0; mu < N; ++mu)
        for (int tau = 0; tau < 2; ++tau)
            for (int a = 0; a < m; ++a)
                c[((size_t)mu * 2 + tau) * m + a] = C[((size_t)(2 * tau) * N + mu) * m + a] +
                                                    I * C[((size_t)(2 * tau + 1) * N + mu) * m + a];
    return c;
}

/* Quaternion component x of a Kramers block B[2][2] of a quantity that equals
 * Q(g) for some quaternion g: g_x = (1/2) tr(Q(e_x)^dagger B).  Returns the
 * real part; *im receives the imaginary part (zero in exact arithmetic). */
static double qproject(int x, const cplx B[2][2], double *im)
{
    double e[4] = {0, 0, 0, 0};
    cplx E[2][2];
    e[x] = 1.0;
    qrep(e, E);
    cplx s = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += conj(E[a][b]) * B[a][b];
    s *= 0.5;
    if (im) *im = cimag(s);
    return creal(s);
}

/* G[p][q][r][s][x][y] = (1/4) sum conj(Q(e_x)_{a'b'}) conj(Q(e_y)_{c'd'})
 *                        (2p+a', 2q+b' | 2r+c', 2s+d'). */
static void project_G(int n, const cplx *sp, double *G, double *imag_max)
{
    int m = 2 * n;
    double imx = 0.0;
    cplx E[4][2][2];
    for (int x = 0; x < 4; ++x) {
        double e[4] = {0, 0, 0, 0};
        e[x] = 1.0;
        qrep(e, E[x]);
    }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s)
                    for (int x = 0; x < 4; ++x)
                        for (int y = 0; y < 4; ++y) {
                            cplx acc = 0;
                            for (int a = 0; a < 2; ++a)
                                for (int b = 0; b < 2; ++b)
                                    for (int c = 0; c < 2; ++c)
                                        for (int d = 0; d < 2; ++d)
                                            acc += conj(E[x][a][b]) * conj(E[y][c][d]) *
                                                   sp[(((size_t)(2 * p + a) * m + 2 * q + b) * m +
                                                       2 * r + c) * m + 2 * s + d];
                            acc *= 0.25;
                            if (fabs(cimag(acc)) > imx) imx = fabs(cimag(acc));
                            G[(((((size_t)p * n + q) * n + r) * n + s) * 4 + x) * 4 + y] =
                                creal(acc);
                        }
    if (imag_max) *imag_max = imx;
}

/* Quaternion product a*b. */
static void qmul(const double a[4], const double b[4], double r[4])
{
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Both bounds loop over MO pairs (r, t) with t innermost; the t loop is a
 * max reduction (order-independent), written for SIMD. */
void orc_dmax_coulomb(int NA, const double *CA, int n, double *Dmax)
{
    const size_t pl = (size_t)NA * n;  /* plane stride */
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < NA; ++k)
        for (int l = 0; l < NA; ++l) {
            double m = 0.0;
            const double *b0 = CA + (size_t)l * n, *b1 = b0 + pl, *b2 = b1 + pl, *b3 = b2 + pl;
            for (int r = 0; r < n; ++r) {
                /* a = conj(C_kr) */
                const double a0 = CA[(size_t)k * n + r], a1 = -CA[pl + (size_t)k * n + r];
                const double a2 = -CA[2 * pl + (size_t)k * n + r];
                const double a3 = -CA[3 * pl + (size_t)k * n + r];
#pragma omp simd reduction(max : m)
                for (int t = 0; t < n; ++t) {
                    /* d = a * C_lt, the quaternion product written out */
                    double d0 = a0 * b0[t] - a1 * b1[t] - a2 * b2[t] - a3 * b3[t];
                    double d1 = a0 * b1[t] + a1 * b0[t] + a2 * b3[t] - a3 * b2[t];
                    double d2 = a0 * b2[t] - a1 * b3[t] + a2 * b0[t] + a3 * b1[t];
                    double d3 = a0 * b3[t] + a1 * b2[t] - a2 * b1[t] + a3 * b0[t];
                    d0 = fabs(d0); d1 = fabs(d1); d2 = fabs(d2); d3 = fabs(d3);
                    m = m > d0 ? m : d0;
                    m = m > d1 ? m : d1;
                    m = m > d2 ? m : d2;
                    m = m > d3 ? m : d3;
                }
            }
            Dmax[(size_t)k * NA + l] = m;
        }
}

void orc_dmax_gaunt(int NL, const double *CL, int NS, const double *CS, int n, double *Dmax)
{
    /* e_K for K = x, y, z: the quaternion units with sigma_K = -i Q(e_K) */
    const double unit[3][4] = {{0, 0, 0, 1}, {0, 0, 1, 0}, {0, 1, 0, 0}};
    const size_t pL = (size_t)NL * n, pS = (size_t)NS * n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int mu = 0; mu < NL; ++mu)
        for (int nu = 0; nu < NS; ++nu) {
            double m = 0.0;
            const double *l0 = CL + (size_t)mu * n, *l1 = l0 + pL, *l2 = l1 + pL, *l3 = l2 + pL;
            const double *s0 = CS + (size_t)nu * n, *s1 = s0 + pS, *s2 = s1 + pS, *s3 = s2 + pS;
            for (int K = 0; K < 3; ++K)
                for (int r = 0; r < n; ++r) {
                    /* a = conj(C^L_mu r) e_K, b = conj(C^S_nu r) e_K */
                    double lr[4] = {l0[r], -l1[r], -l2[r], -l3[r]};
                    double sr[4] = {s0[r], -s1[r], -s2[r], -s3[r]};
                    double a[4], b[4];
                    qmul(lr, unit[K], a);
                    qmul(sr, unit[K], b);
#pragma omp simd reduction(max : m)
                    for (int t = 0; t < n; ++t) {
                        /* a * C^S_nu t + b * C^L_mu t */
                        double d0 = a[0] * s0[t] - a[1] * s1[t] - a[2] * s2[t] - a[3] * s3[t]
                                  + (b[0] * l0[t] - b[1] * l1[t] - b[2] * l2[t] - b[3] * l3[t]);
                        double d1 = a[0] * s1[t] + a[1] * s0[t] + a[2] * s3[t] - a[3] * s2[t]
                                  + (b[0] * l1[t] + b[1] * l0[t] + b[2] * l3[t] - b[3] * l2[t]);
                        double d2 = a[0] * s2[t] - a[1] * s3[t] + a[2] * s0[t] + a[3] * s1[t]
                                  + (b[0] * l2[t] - b[1] * l3[t] + b[2] * l0[t] + b[3] * l1[t]);
                        double d3 = a[0] * s3[t] + a[1] * s2[t] - a[2] * s1[t] + a[3] * s0[t]
                                  + (b[0] * l3[t] + b[1] * l2[t] - b[2] * l1[t] + b[3] * l0[t]);
                        d0 = fabs(d0); d1 = fabs(d1); d2 = fabs(d2); d3 = fabs(d3);
                        m = m > d0 ? m : d0;
                        m = m > d1 ? m : d1;
                        m = m > d2 ? m : d2;
                        m = m > d3 ? m : d3;
                    }
                }
            Dmax[(size_t)mu * NS + nu] = m;
        }
}

/* ------------------------------------------------------------------------ */
/* Definition route: literal four-spinor operator matrices                     */
/* ------------------------------------------------------------------------ */

/* Four-spinor basis: each scalar function f of the combined list F = L (+ S)
 * carries two four-component basis spinors; L functions occupy components
 * 0,1 (alpha, beta of the large part), S functions components 2,3.
 * c4[f][w][a] is the coefficient of spinor a on basis spinor (f, w). */
static int def_impl(const orc_basis *L, const orc_basis *S, const double *CL, const double *CS,
                    int n, int ham, int general, double *G, double *spinor_out,
                    double *imag_max);

int orc_transform_def(const orc_basis *L, const orc_basis *S, const double *CL,
                      const double *CS, int n, int ham, double *G, double *spinor_out,
                      double *imag_max)
{
    return def_impl(L, S, CL, CS, n, ham, 0, G, spinor_out, imag_max);
}

int orc_transform_spinor_def(const orc_basis *L, const orc_basis *S, const double *CL,
                             const double *CS, int m, int ham, double *spinor_out)
{
    if (!spinor_out) return -1;
    return def_impl(L, S, CL, CS, m, ham, 1, NULL, spinor_out, NULL);
}

/* n: Kramers pairs (quaternion C, m = 2n spinors) or, with general, the
 * number m of general spinors. */
static int def_impl(const orc_basis *L, const orc_basis *S, const double *CL, const double *CS,
                    int n, int ham, int general, double *G, double *spinor_out,
                    double *imag_max)
{
    int with_S = (ham != 0);
    if (ham < 0 || ham > 5) return -1;
    if (with_S && (!S || !CS)) return -1;
    int NL = L->nfunc, NS = with_S ? S->nfunc : 0, NF = NL + NS, m = general ? n : 2 * n;
    if (NF > 64 || m > 64 || n <= 0) return -1;
    if (ham_gauge(ham) && NF > 32) return -1;
    if (!carts_valid(L) || (with_S && !carts_valid(S))) return -1;

    /* combined scalar basis */
    nbasis bl = nb_make(L), bs;
    if (with_S) bs = nb_make(S);
    const nbasis **fb = (const nbasis **)malloc(sizeof(nbasis *) * NF);
    int *fi = (int *)malloc(sizeof(int) * NF);
    for (int f = 0; f < NF; ++f) {
        fb[f] = f < NL ? &bl : &bs;
        fi[f] = f < NL ? f : f - NL;
    }
    size_t nf2 = (size_t)NF * NF;
    double *eri = (double *)malloc(sizeof(double) * nf2 * nf2);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < NF; ++i)
        for (int j = 0; j < NF; ++j)
            for (int k = 0; k < NF; ++k)
                for (int l = 0; l < NF; ++l)
                    eri[((size_t)i * NF + j) * nf2 + (size_t)k * NF + l] =
                        nb_eri(fb[i], fi[i], fb[j], fi[j], fb[k], fi[k], fb[l], fi[l]);

    cplx *cl = general ? spinor_coefs_general(NL, m, CL) : spinor_coefs(NL, n, CL);
    cplx *cs = !with_S ? NULL : general ? spinor_coefs_general(NS, m, CS) : spinor_coefs(NS, n, CS);
    cplx *c4 = (cplx *)calloc((size_t)NF * 4 * m, sizeof(cplx));
    for (int f = 0; f < NF; ++f)
        for (int tau = 0; tau < 2; ++tau)
            for (int a = 0; a < m; ++a) {
                if (f < NL)
                    c4[((size_t)f * 4 + tau) * m + a] = cl[((size_t)f * 2 + tau) * m + a];
                else
                    c4[((size_t)f * 4 + 2 + tau) * m + a] =
                        cs[((size_t)(f - NL) * 2 + tau) * m + a];
            }

    /* operator list: (weight, 4x4 matrix) */
    cplx ops[4][4][4];
    double w[4];
    int nops = 0;
    if (ham_coulomb(ham)) { /* Coulomb: identity */
        memset(ops[nops], 0, sizeof(ops[nops]));
        for (int d = 0; d < 4; ++d) ops[nops][d][d] = 1;
        w[nops++] = 1.0;
    }
    if (ham_gaunt(ham)) { /* Gaunt: -sum_K alpha_K x alpha_K */
        for (int K = 0; K < 3; ++K) {
            const cplx *sg = pauli(K);
            memset(ops[nops], 0, sizeof(ops[nops]));
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    ops[nops][a][2 + b] = sg[a * 2 + b];
                    ops[nops][2 + a][b] = sg[a * 2 + b];
                }
            w[nops++] = -1.0;
        }
    }

    size_t m2 = (size_t)m * m;
    cplx *sp = (cplx *)calloc(m2 * m2, sizeof(cplx));
    cplx *T = (cplx *)malloc(sizeof(cplx) * nf2 * m2);
    cplx *X = (cplx *)malloc(sizeof(cplx) * nf2 * m2);
    for (int o = 0; o < nops; ++o) {
        /* T_{ij,ab} = sum_{w,w'} conj(c4[i][w][a]) O[w][w'] c4[j][w'][b] */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < NF; ++i)
            for (int j = 0; j < NF; ++j)
                for (int a = 0; a < m; ++a)
                    for (int b = 0; b < m; ++b) {
                        cplx s = 0;
                        for (int u = 0; u < 4; ++u)
                            for (int v = 0; v < 4; ++v)
                                s += conj(c4[((size_t)i * 4 + u) * m + a]) * ops[o][u][v] *
                                     c4[((size_t)j * 4 + v) * m + b];
                        T[((size_t)i * NF + j) * m2 + (size_t)a * m + b] = s;
                    }
        /* X_{ij,cd} = sum_{kl} (ij|kl) T_{kl,cd} */
#pragma omp parallel for schedule(static)
        for (size_t ij = 0; ij < nf2; ++ij) {
            for (size_t cd = 0; cd < m2; ++cd) X[ij * m2 + cd] = 0;
            for (size_t kl = 0; kl < nf2; ++kl) {
                double e = eri[ij * nf2 + kl];
                for (size_t cd = 0; cd < m2; ++cd) X[ij * m2 + cd] += e * T[kl * m2 + cd];
            }
        }
        /* (ab|cd) += w sum_{ij} T_{ij,ab} X_{ij,cd} */
#pragma omp parallel for schedule(static)
        for (size_t ab = 0; ab < m2; ++ab)
            for (size_t ij = 0; ij < nf2; ++ij) {
                cplx t = w[o] * T[ij * m2 + ab];
                for (size_t cd = 0; cd < m2; ++cd) sp[ab * m2 + cd] += t * X[ij * m2 + cd];
            }
    }
    if (ham_gauge(ham)) {
        /* Gauge term, Eq. (breit): (alpha_1 x r) . (alpha_2 x r) / (2 r^3)
         *   = sum_{j,l} alpha_1j alpha_2l N_jl,
         *   N_jl = (1/2) sum_{i,k,k'} eps_ijk eps_ilk' r_k r_k' / r^3,
         * the cross products written out component by component; the AO
         * integrals of r_k r_k' / r^3 are those of Eq. (gaugeInt). */
        double *e3 = (double *)malloc(sizeof(double) * 9 * nf2 * nf2);
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < NF; ++i)
            for (int j = 0; j < NF; ++j)
                for (int k = 0; k < NF; ++k)
                    for (int l = 0; l < NF; ++l) {
                        double t[9];
                        nb_eri3(fb[i], fi[i], fb[j], fi[j], fb[k], fi[k], fb[l], fi[l], t);
                        size_t q = ((size_t)i * NF + j) * nf2 + (size_t)k * NF + l;
                        for (int c = 0; c < 9; ++c) e3[(size_t)c * nf2 * nf2 + q] = t[c];
                    }
        /* alpha_K densities T^K_{ij,ab} of each electron */
        cplx *TA = (cplx *)malloc(sizeof(cplx) * 3 * nf2 * m2);
        for (int K = 0; K < 3; ++K) {
            const cplx *sg = pauli(K);
            cplx al[4][4];
            memset(al, 0, sizeof(al));
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    al[a][2 + b] = sg[a * 2 + b];
                    al[2 + a][b] = sg[a * 2 + b];
                }
            cplx *TK = TA + (size_t)K * nf2 * m2;
#pragma omp parallel for schedule(static)
            for (int i = 0; i < NF; ++i)
                for (int j = 0; j < NF; ++j)
                    for (int a = 0; a < m; ++a)
                        for (int b = 0; b < m; ++b) {
                            cplx v = 0;
                            for (int u = 0; u < 4; ++u)
                                for (int w2 = 0; w2 < 4; ++w2)
                                    v += conj(c4[((size_t)i * 4 + u) * m + a]) * al[u][w2] *
                                         c4[((size_t)j * 4 + w2) * m + b];
                            TK[((size_t)i * NF + j) * m2 + (size_t)a * m + b] = v;
                        }
        }
        double *N = (double *)malloc(sizeof(double) * nf2 * nf2);
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
                double wt[9];
                for (int k = 0; k < 3; ++k)
                    for (int k2 = 0; k2 < 3; ++k2) {
                        wt[k * 3 + k2] = 0.0;
                        for (int i = 0; i < 3; ++i)
                            wt[k * 3 + k2] += 0.5 * levi(i, j, k) * levi(i, l, k2);
                    }
                for (size_t q = 0; q < nf2 * nf2; ++q) {
                    double v = 0.0;
                    for (int c = 0; c < 9; ++c)
                        if (wt[c] != 0.0) v += wt[c] * e3[(size_t)c * nf2 * nf2 + q];
                    N[q] = v;
                }
                const cplx *Tj = TA + (size_t)j * nf2 * m2, *Tl = TA + (size_t)l * nf2 * m2;
#pragma omp parallel for schedule(static)
                for (size_t ij = 0; ij < nf2; ++ij) {
                    for (size_t cd = 0; cd < m2; ++cd) X[ij * m2 + cd] = 0;
                    for (size_t kl = 0; kl < nf2; ++kl) {
                        double e = N[ij * nf2 + kl];
                        for (size_t cd = 0; cd < m2; ++cd) X[ij * m2 + cd] += e * Tl[kl * m2 + cd];
                    }
                }
#pragma omp parallel for schedule(static)
                for (size_t ab = 0; ab < m2; ++ab)
                    for (size_t ij = 0; ij < nf2; ++ij) {
                        cplx t = Tj[ij * m2 + ab];
                        for (size_t cd = 0; cd < m2; ++cd) sp[ab * m2 + cd] += t * X[ij * m2 + cd];
                    }
            }
        free(N);
        free(TA);
        free(e3);
    }
    if (G) project_G(n, sp, G, imag_max);
    if (spinor_out) memcpy(spinor_out, sp, sizeof(cplx) * m2 * m2);

    free(sp);
    free(T);
    free(X);
    free(c4);
    free(cl);
    free(cs);
    free(eri);
    free(fb);
    free(fi);
    nb_free(&bl);
    if (with_S) nb_free(&bs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's direct route                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int cls;   /* 0 = LL, 1 = SS, 2 = LS (mu in L, nu in S) */
    int mu, nu;
} opair;

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

int64_t orc_num_bra_pairs(const orc_basis *L, const orc_basis *S, int ham)
{
    int64_t NL = L->nfunc, NS = (S && ham != 0) ? S->nfunc : 0;
    int64_t np = 0;
    if (ham_coulomb(ham)) np += NL * (NL + 1) / 2 + NS * (NS + 1) / 2;
    if (ham_ls(ham)) np += NL * NS;
    return np;
}

/* Pauli-scalar pair density of spinor pair (c,d), Eqs. (Den) and
 * (QuaternionScatter): D_s = D_aa + D_bb with D_{lambda kappa} = c*_kappa c_lambda. */
static cplx dens_s(const cplx *cx, int m, int ka, int la, int c, int d)
{
    cplx s = 0;
    for (int tau = 0; tau < 2; ++tau)
        s += conj(cx[((size_t)ka * 2 + tau) * m + c]) * cx[((size_t)la * 2 + tau) * m + d];
    return s;
}

/* Pauli-vector pair density (component K) of the L-S product distribution
 * chi^L_ka chi^S_la for spinor pair (c,d): the sigma_K-weighted density of both
 * L-S orderings of the four-spinor product psi_c^dagger alpha_K psi_d. */
static cplx dens_gaunt(const cplx *cl, const cplx *cs, int m, int K, int ka, int la, int c,
                       int d)
{
    const cplx *sg = pauli(K);
    cplx s = 0;
    for (int t1 = 0; t1 < 2; ++t1)
        for (int t2 = 0; t2 < 2; ++t2) {
            cplx sk = sg[t1 * 2 + t2];
            if (sk == 0) continue;
            s += conj(cl[((size_t)ka * 2 + t1) * m + c]) * sk * cs[((size_t)la * 2 + t2) * m + d];
            s += conj(cs[((size_t)la * 2 + t1) * m + c]) * sk * cl[((size_t)ka * 2 + t2) * m + d];
        }
    return s;
}

static int direct_impl(const orc_basis *L, const orc_basis *S, const double *CL,
                       const double *CS, int n, int ham, double tau, const int64_t *rows,
                       int64_t nrows_sel, int do_second, double *G, orc_stats *st, double *Vq,
                       int general, double *sp_out, const double *dmax_in,
                       const int64_t *cols, int64_t ncols);

int orc_transform_direct_dmax(const orc_basis *L, const orc_basis *S, const double *CL,
                              const double *CS, int n, int ham, double tau,
                              const double *dmax_in, double *G, orc_stats *st)
{
    if (!dmax_in) return -1;
    return direct_impl(L, S, CL, CS, n, ham, tau, NULL, 0, 1, G, st, NULL, 0, NULL, dmax_in,
                       NULL, 0);
}

int orc_transform_direct(const orc_basis *L, const orc_basis *S, const double *CL,
                         const double *CS, int n, int ham, double tau, const int64_t *rows,
                         int64_t nrows_sel, int do_second, double *G, orc_stats *st)
{
    return direct_impl(L, S, CL, CS, n, ham, tau, rows, nrows_sel, do_second, G, st, NULL, 0,
                       NULL, NULL, NULL, 0);
}

int orc_first_half_rows(const orc_basis *L, const orc_basis *S, const double *CL,
                        const double *CS, int n, int ham, double tau, const int64_t *rows,
                        int64_t nrows, double *Vq)
{
    if (!rows || nrows <= 0 || !Vq) return -1;
    return direct_impl(L, S, CL, CS, n, ham, tau, rows, nrows, 0, NULL, NULL, Vq, 0, NULL, NULL,
                       NULL, 0);
}

int orc_first_half_rows_cols(const orc_basis *L, const orc_basis *S, const double *CL,
                             const double *CS, int n, int ham, double tau, const int64_t *rows,
                             int64_t nrows, const int64_t *cols, int64_t ncols,
                             const double *dmax_in, double *Vq)
{
    if (!rows || nrows <= 0 || !Vq || !cols || ncols <= 0) return -1;
    return direct_impl(L, S, CL, CS, n, ham, tau, rows, nrows, 0, NULL, NULL, Vq, 0, NULL,
                       dmax_in, cols, ncols);
}

int orc_transform_spinor_direct(const orc_basis *L, const orc_basis *S, const double *CL,
                                const double *CS, int m, int ham, double tau,
                                double *spinor_out, orc_stats *st)
{
    if (!spinor_out) return -1;
    return direct_impl(L, S, CL, CS, m, ham, tau, NULL, 0, 1, NULL, st, NULL, 1, spinor_out,
                       NULL, NULL, 0);
}

/* n: Kramers pairs (quaternion C, m = 2n spinors, output G projected onto the
 * quaternion basis) or, with general, the number m of general spinors (output
 * the spinor integrals sp_out). */
static int direct_impl(const orc_basis *L, const orc_basis *S, const double *CL,
                       const double *CS, int n, int ham, double tau, const int64_t *rows,
                       int64_t nrows_sel, int do_second, double *G, orc_stats *st, double *Vq,
                       int general, double *sp_out, const double *dmax_in,
                       const int64_t *cols, int64_t ncols)
{
    int with_S = (ham != 0);
    if (with_S && (!S || !CS)) return -1;
    if (n <= 0 || tau < 0 || ham < 0 || ham > 5) return -1;
    if (general && Vq) return -1;
    if (!carts_valid(L) || (with_S && !carts_valid(S))) return -1;
    int NL = L->nfunc, NS = with_S ? S->nfunc : 0, m = general ? n : 2 * n;
    size_t m2 = (size_t)m * m;
    /* spinor pairs (c, d) of the first half: all m^2, or (cols: first-half
     * rows only) the four of each selected MO pair p <= q, c in {2p, 2p+1},
     * d in {2q, 2q+1}; the MO pair index counts p <= q with p outer */
    if (cols && (general || !Vq || do_second)) return -1;
    const int64_t npair_mo = (int64_t)n * (n + 1) / 2;
    int64_t ncd = cols ? 4 * ncols : (int64_t)m2;
    int *cd_c = (int *)malloc(sizeof(int) * (size_t)ncd), *cd_d = (int *)malloc(sizeof(int) * (size_t)ncd);
    int64_t *col_p = cols ? (int64_t *)malloc(sizeof(int64_t) * (size_t)ncols) : NULL;
    int64_t *col_q = cols ? (int64_t *)malloc(sizeof(int64_t) * (size_t)ncols) : NULL;
    if (cols) {
        for (int64_t j = 0; j < ncols; ++j) {
            if (cols[j] < 0 || cols[j] >= npair_mo) {
                free(cd_c); free(cd_d); free(col_p); free(col_q);
                return -1;
            }
            int p = 0;
            int64_t rest = cols[j];
            while (rest >= n - p) { rest -= n - p; ++p; }
            col_p[j] = p;
            col_q[j] = p + rest;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    cd_c[4 * j + 2 * a + b] = (int)(2 * col_p[j] + a);
                    cd_d[4 * j + 2 * a + b] = (int)(2 * col_q[j] + b);
                }
        }
    } else {
        for (int c = 0; c < m; ++c)
            for (int d = 0; d < m; ++d) {
                cd_c[(size_t)c * m + d] = c;
                cd_d[(size_t)c * m + d] = d;
            }
    }
    /* gaunt: L-S rows present (Gaunt and/or gauge term) */
    int coul = ham_coulomb(ham), gaunt = ham_ls(ham);
    int gaunt_term = ham_gaunt(ham), gauge_term = ham_gauge(ham);

    nbasis bl = nb_make(L), bs;
    if (with_S) bs = nb_make(S);
    cplx *cl = general ? spinor_coefs_general(NL, m, CL) : spinor_coefs(NL, n, CL);
    cplx *cs = !with_S ? NULL : general ? spinor_coefs_general(NS, m, CS) : spinor_coefs(NS, n, CS);

    /* bra/ket pair lists */
    int64_t nLL = (int64_t)NL * (NL + 1) / 2, nSS = (int64_t)NS * (NS + 1) / 2;
    int64_t nLS = gaunt ? (int64_t)NL * NS : 0;
    int64_t np = (coul ? nLL + nSS : 0) + nLS;
    opair *pl = (opair *)malloc(sizeof(opair) * (size_t)(np > 0 ? np : 1));
    int64_t k = 0;
    if (coul) {
        for (int nu = 0; nu < NL; ++nu)
            for (int mu = 0; mu <= nu; ++mu) pl[k++] = (opair){0, mu, nu};
        for (int nu = 0; nu < NS; ++nu)
            for (int mu = 0; mu <= nu; ++mu) pl[k++] = (opair){1, mu, nu};
    }
    for (int mu = 0; mu < NL && gaunt; ++mu)
        for (int nu = 0; nu < NS; ++nu) pl[k++] = (opair){2, mu, nu};
    /* selected bra rows: slot[i] = position of pair i among the selected rows, or -1 */
    int64_t nrow = rows ? nrows_sel : np;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nrow > 0 ? nrow : 1));
    for (int64_t i = 0; i < np; ++i) slot[i] = rows ? -1 : i;
    for (int64_t r = 0; r < nrow; ++r) {
        int64_t i = rows ? rows[r] : r;
        if (i < 0 || i >= np || (rows && slot[i] >= 0)) {
            free(cd_c);
            free(cd_d);
            free(col_p);
            free(col_q);
            free(slot);
            free(sel);
            free(pl);
            free(cl);
            free(cs);
            nb_free(&bl);
            if (with_S) nb_free(&bs);
            return -1;
        }
        slot[i] = r;
        sel[r] = i;
    }

    /* Schwarz factors Q = sqrt((mn|mn)) of each pair, Eq. (SchwarzDen) */
    double *Q = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < np; ++i) {
        const nbasis *A = pl[i].cls == 1 ? &bs : &bl;
        const nbasis *B = pl[i].cls == 0 ? &bl : &bs;
        Q[i] = sqrt(nb_eri(A, pl[i].mu, B, pl[i].nu, A, pl[i].mu, B, pl[i].nu));
    }

    /* Density bound per ket pair: infinity norm over all MO pairs (r,t) of the
     * quaternion pair density, read off the spinor-pair densities of each
     * Kramers block (Coulomb: D_s; Gaunt: the sigma_K densities, which equal
     * -i Q(D^K)). */
    double *Dmax = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
    if (dmax_in) {
        /* a bound given by the caller (the MO-driven variant's per-batch bound) */
        for (int64_t i = 0; i < np; ++i) Dmax[i] = dmax_in[i];
    } else if (general) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < np; ++i) {
        /* general spinors: the largest |real| or |imaginary| part of the
         * Pauli-scalar (Coulomb, both orderings of the pair) or sigma_K-weighted
         * (Gaunt) pair density over all ordered spinor pairs (c, d) */
        double mx = 0.0;
        const opair P = pl[i];
        for (int c = 0; c < m; ++c)
            for (int d = 0; d < m; ++d) {
                cplx v[6];
                int nv = 0;
                if (P.cls == 2) {
                    for (int K = 0; K < 3; ++K) v[nv++] = dens_gaunt(cl, cs, m, K, P.mu, P.nu, c, d);
                } else {
                    const cplx *cx = P.cls == 0 ? cl : cs;
                    v[nv++] = dens_s(cx, m, P.mu, P.nu, c, d);
                    v[nv++] = dens_s(cx, m, P.nu, P.mu, c, d);
                }
                for (int k2 = 0; k2 < nv; ++k2) {
                    if (fabs(creal(v[k2])) > mx) mx = fabs(creal(v[k2]));
                    if (fabs(cimag(v[k2])) > mx) mx = fabs(cimag(v[k2]));
                }
            }
        Dmax[i] = mx;
    }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < np; ++i) {
        double mx = 0.0;
        const opair P = pl[i];
        for (int r = 0; r < n; ++r)
            for (int t = 0; t < n; ++t) {
                int nK = P.cls == 2 ? 3 : 1;
                for (int K = 0; K < nK; ++K)
                    for (int orient = 0; orient < (P.cls == 2 ? 1 : 2); ++orient) {
                        cplx B[2][2];
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) {
                                if (P.cls == 2) {
                                    B[a][b] = I * dens_gaunt(cl, cs, m, K, P.mu, P.nu, 2 * r + a,
                                                             2 * t + b);
                                } else {
                                    const cplx *cx = P.cls == 0 ? cl : cs;
                                    int ka = orient ? P.nu : P.mu, la = orient ? P.mu : P.nu;
                                    B[a][b] = dens_s(cx, m, ka, la, 2 * r + a, 2 * t + b);
                                }
                            }
                        for (int x = 0; x < 4; ++x) {
                            double v = fabs(qproject(x, B, NULL));
                            if (v > mx) mx = v;
                        }
                    }
            }
        Dmax[i] = mx;
    }
    }

    /* First half, Eq. (firsthalf): V_{mn,cd} = sum_{kl kept} (mn|kl) D_{kl,cd},
     * complex spinor-pair columns (c,d); ket pairs are unordered, so both
     * orderings (kl) and (lk) of the Coulomb density enter. */
    int nvK = gaunt ? 3 : 1;
    cplx *V = (cplx *)calloc((size_t)(nrow > 0 ? nrow : 1) * nvK * m2, sizeof(cplx));
    int64_t kept[4] = {0, 0, 0, 0}, total[4] = {0, 0, 0, 0}, keptG = 0, totalG = 0, ties = 0;
    double t0 = now_s();
    int nthreads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        cplx *Dk = (cplx *)malloc(sizeof(cplx) * 3 * m2);
        int64_t lk[4] = {0, 0, 0, 0}, lt[4] = {0, 0, 0, 0}, lkG = 0, ltG = 0, lties = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrow; ++r) {
            const int64_t i = sel[r];
            const opair B = pl[i];
            cplx *Vi = V + (size_t)r * nvK * m2;
            const nbasis *bA = B.cls == 1 ? &bs : &bl;
            const nbasis *bB = B.cls == 0 ? &bl : &bs;
            for (int64_t j = 0; j < np; ++j) {
                const opair Kp = pl[j];
                if ((B.cls == 2) != (Kp.cls == 2)) continue; /* Coulomb and Gaunt never mix */
                int cp = (B.cls == 2) ? -1 : B.cls * 2 + Kp.cls;
                if (cp >= 0) lt[cp]++;
                else ltG++;
                double bound = Q[i] * Q[j] * Dmax[j];
                if (tau > 0 && fabs(bound / tau - 1.0) < 1e-12) lties++;
                if (!(bound >= tau)) continue;
                if (cp >= 0) lk[cp]++;
                else lkG++;
                const nbasis *kA = Kp.cls == 1 ? &bs : &bl;
                const nbasis *kB = Kp.cls == 0 ? &bl : &bs;
                double e = nb_eri(bA, B.mu, bB, B.nu, kA, Kp.mu, kB, Kp.nu);
                if (Kp.cls == 2) {
                    /* weight of the sigma_L density in V^K.  Gaunt: (mn|kl)
                     * delta_KL.  Gauge: the second half below applies -sigma_K
                     * (the sign of -alpha.alpha), and the gauge operator is
                     * +sum_KL alpha_1K alpha_2L N_KL with
                     * N_KL = (delta_KL / r - r_K r_L / r^3) / 2, so V^K takes
                     * -N_KL = ((mn|K L|kl) - delta_KL (mn|kl)) / 2. */
                    double wKL[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                    if (gaunt_term)
                        for (int K = 0; K < 3; ++K) wKL[K * 3 + K] += e;
                    if (gauge_term) {
                        double t3[9];
                        nb_eri3(bA, B.mu, bB, B.nu, kA, Kp.mu, kB, Kp.nu, t3);
                        for (int K = 0; K < 3; ++K)
                            for (int L2 = 0; L2 < 3; ++L2)
                                wKL[K * 3 + L2] += 0.5 * (t3[K * 3 + L2] - (K == L2 ? e : 0.0));
                    }
                    for (int L2 = 0; L2 < 3; ++L2)
                        for (int64_t t = 0; t < ncd; ++t) {
                                int c = cd_c[t], d = cd_d[t];
                                cplx D = dens_gaunt(cl, cs, m, L2, Kp.mu, Kp.nu, c, d);
                                for (int K = 0; K < 3; ++K)
                                    if (wKL[K * 3 + L2] != 0.0)
                                        Vi[(size_t)K * m2 + (size_t)c * m + d] +=
                                            wKL[K * 3 + L2] * D;
                            }
                } else {
                    const cplx *cx = Kp.cls == 0 ? cl : cs;
                    for (int64_t t = 0; t < ncd; ++t) {
                            int c = cd_c[t], d = cd_d[t];
                            cplx D = dens_s(cx, m, Kp.mu, Kp.nu, c, d);
                            if (Kp.mu != Kp.nu) D += dens_s(cx, m, Kp.nu, Kp.mu, c, d);
                            Vi[(size_t)c * m + d] += e * D;
                        }
                }
            }
        }
#pragma omp critical
        {
            for (int c = 0; c < 4; ++c) {
                kept[c] += lk[c];
                total[c] += lt[c];
            }
            keptG += lkG;
            totalG += ltG;
            ties += lties;
        }
        free(Dk);
    }
    double t1 = now_s();

    if (Vq) {
        /* First-half rows in quaternion components: the (r, s) spinor block of
         * a Coulomb row is Q(V^{rs}) and of a Gaunt row -i Q(V^{K,rs}); columns
         * (K, r <= s, y) at K * 4 * npair + 4 * idx(r, s) + y, idx counting the
         * pairs r <= s with r outer. */
        const int64_t npair = cols ? ncols : npair_mo, width = (int64_t)nvK * 4 * npair;
        for (int64_t r = 0; r < nrow; ++r) {
            const opair B = pl[sel[r]];
            const cplx *Vr = V + (size_t)r * nvK * m2;
            double *out = Vq + (size_t)r * width;
            for (int64_t c = 0; c < width; ++c) out[c] = 0.0;
            int nK = B.cls == 2 ? 3 : 1;
            for (int K = 0; K < nK; ++K)
                for (int64_t idx = 0; idx < npair; ++idx) {
                    /* MO pair idx (p <= q, p outer), or the idx-th selected one */
                    int p, q;
                    if (cols) {
                        p = (int)col_p[idx];
                        q = (int)col_q[idx];
                    } else {
                        p = 0;
                        int64_t rest = idx;
                        while (rest >= n - p) { rest -= n - p; ++p; }
                        q = p + (int)rest;
                    }
                    cplx blk[2][2];
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b) {
                            cplx v = Vr[(size_t)K * m2 + (size_t)(2 * p + a) * m + 2 * q + b];
                            blk[a][b] = B.cls == 2 ? I * v : v;
                        }
                    for (int y = 0; y < 4; ++y)
                        out[(int64_t)K * 4 * npair + 4 * idx + y] = qproject(y, blk, NULL);
                }
        }
    }

    if (do_second && (G || sp_out)) {
        /* Second half, Sec. 2.4.2: the Pauli components of V are converted to
         * 2x2 spin blocks V^{t1 t2} (Coulomb: V_s on the diagonal; Gaunt:
         * -sum_K sigma_K[t1][t2] V_K, the minus sign of -alpha.alpha), then
         * contracted with two-spinor coefficients, Eq. (secondhalf), as two
         * matrix products:  W[mu][t1][b][cd] = sum_{nu,t2} c_{nu t2,b} V^{t1 t2}_{mu nu,cd},
         * (ab|cd) = sum_{mu,t1} conj(c_{mu t1,a}) W[mu][t1][b][cd]. */
        cplx *sp = (cplx *)calloc(m2 * m2, sizeof(cplx));
        for (int cls = 0; cls < 3; ++cls) {
            if (cls == 2 && !gaunt) continue;
            if (cls < 2 && !coul) continue;
            if (cls == 1 && !with_S) continue;
            /* orientations: for LS pairs the bra product chi^L_mu chi^S_nu enters
             * as (L on the conjugated side, S unconjugated) and the reverse. */
            for (int orient = 0; orient < (cls == 2 ? 2 : 1); ++orient) {
                int NA, NB;
                const cplx *ca, *cb;
                if (cls == 0) { NA = NB = NL; ca = cb = cl; }
                else if (cls == 1) { NA = NB = NS; ca = cb = cs; }
                else if (orient == 0) { NA = NL; NB = NS; ca = cl; cb = cs; }
                else { NA = NS; NB = NL; ca = cs; cb = cl; }
                cplx *W = (cplx *)calloc((size_t)NA * 2 * m * m2, sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 1)
                for (int mu = 0; mu < NA; ++mu) {
                    for (int nu = 0; nu < NB; ++nu) {
                        /* locate the stored (unordered / LS) pair row */
                        int64_t idx;
                        if (cls == 0) {
                            int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
                            idx = (int64_t)b * (b + 1) / 2 + a;
                        } else if (cls == 1) {
                            int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
                            idx = nLL + (int64_t)b * (b + 1) / 2 + a;
                        } else {
                            int lmu = orient == 0 ? mu : nu, snu = orient == 0 ? nu : mu;
                            idx = (coul ? nLL + nSS : 0) + (int64_t)lmu * NS + snu;
                        }
                        if (slot[idx] < 0) continue;
                        const cplx *Vr = V + (size_t)slot[idx] * nvK * m2;
                        for (int t1 = 0; t1 < 2; ++t1)
                            for (int t2 = 0; t2 < 2; ++t2) {
                                /* spin block weight per Pauli component */
                                cplx wK[3] = {0, 0, 0};
                                cplx ws = 0;
                                if (cls < 2) {
                                    if (t1 != t2) continue;
                                    ws = 1.0;
                                } else {
                                    for (int K = 0; K < 3; ++K) wK[K] = -pauli(K)[t1 * 2 + t2];
                                    if (wK[0] == 0 && wK[1] == 0 && wK[2] == 0) continue;
                                }
                                for (int b = 0; b < m; ++b) {
                                    cplx cbv = cb[((size_t)nu * 2 + t2) * m + b];
                                    cplx *Wrow = W + (((size_t)mu * 2 + t1) * m + b) * m2;
                                    if (cls < 2) {
                                        cplx f = ws * cbv;
                                        for (size_t cd = 0; cd < m2; ++cd) Wrow[cd] += f * Vr[cd];
                                    } else {
                                        for (int K = 0; K < 3; ++K) {
                                            if (wK[K] == 0) continue;
                                            cplx f = wK[K] * cbv;
                                            const cplx *VK = Vr + (size_t)K * m2;
                                            for (size_t cd = 0; cd < m2; ++cd) Wrow[cd] += f * VK[cd];
                                        }
                                    }
                                }
                            }
                    }
                }
#pragma omp parallel for schedule(static)
                for (int a = 0; a < m; ++a)
                    for (int mu = 0; mu < NA; ++mu)
                        for (int t1 = 0; t1 < 2; ++t1) {
                            cplx ca_ = conj(ca[((size_t)mu * 2 + t1) * m + a]);
                            if (ca_ == 0) continue;
                            for (int b = 0; b < m; ++b) {
                                const cplx *Wrow = W + (((size_t)mu * 2 + t1) * m + b) * m2;
                                cplx *out = sp + ((size_t)a * m + b) * m2;
                                for (size_t cd = 0; cd < m2; ++cd) out[cd] += ca_ * Wrow[cd];
                            }
                        }
                free(W);
            }
        }
        if (G && !general) project_G(n, sp, G, NULL);
        if (sp_out) memcpy(sp_out, sp, sizeof(cplx) * m2 * m2);
        free(sp);
    }
    double t2 = now_s();

    if (st) {
        memset(st, 0, sizeof(*st));
        for (int c = 0; c < 4; ++c) {
            st->kept[c] = kept[c];
            st->total[c] = total[c];
        }
        st->kept_gaunt = keptG;
        st->total_gaunt = totalG;
        st->tie_band = ties;
        st->seconds_first_half = t1 - t0;
        st->seconds_second_half = t2 - t1;
        st->threads = nthreads;
    }
    free(V);
    free(cd_c);
    free(cd_d);
    free(col_p);
    free(col_q);
    free(Q);
    free(Dmax);
    free(slot);
    free(sel);
    free(pl);
    free(cl);
    free(cs);
    nb_free(&bl);
    if (with_S) nb_free(&bs);
    return 0;
}
