/* oracle.h -- plain FP64 CPU oracle for the quaternion AO->MO two-electron
 * integral transformation.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that
 * the GPU path is compared against.  It shares no code with the GPU library;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  Nothing in the product path calls it.
 *
 * Conventions (all arrays C-contiguous, FP64 unless stated):
 *   basis     contracted Cartesian Gaussians of s, p or d type; coefs
 *             multiply normalized primitives N x^lx y^ly z^lz exp(-a r^2)
 *             (coordinates relative to the centre), N = (2a/pi)^{3/4}
 *             (4a)^{L/2} / sqrt((2lx-1)!! (2ly-1)!! (2lz-1)!!); each
 *             contracted function is rescaled to unit self-overlap.
 *             Gauge-term hams (4, 5) take s functions only.
 *   C         quaternion MO coefficients, planar [4][N][n]:
 *             C = C0 + i C1 + j C2 + k C3.
 *   G         quaternion MO integrals [n][n][n][n][4][4] = G^{xy}_{pqrs}
 *             (x: bra quaternion component, y: ket component).
 *   spinors   quaternion MO p is the Kramers pair (2p, 2p+1); its two-spinor
 *             coefficients are the columns of the 2x2 complex matrix
 *             Q(q) = [[q0 + i q1, q2 + i q3], [-q2 + i q3, q0 - i q1]]
 *             with rows alpha, beta.
 *   ham       0 = LL (large-component Coulomb only), 1 = DC (all four L/S
 *             Coulomb classes), 2 = DCG (DC + Gaunt), 3 = Gaunt term alone,
 *             4 = DCB (DC + Gaunt + the gauge term of the Breit operator),
 *             5 = gauge term alone.  The gauge term enters as
 *             (alpha_1 x r12) . (alpha_2 x r12) / (2 r12^3), Eq. (breit).
 */
#ifndef QDCB_ORACLE_H
#define QDCB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nfunc;
    const double *centers; /* [nfunc][3] */
    const int32_t *nprim;  /* [nfunc] */
    const double *exps;    /* [sum nprim] */
    const double *coefs;   /* [sum nprim] */
    const int32_t *cart;   /* [nfunc] 0 = s, 1, 2, 3 = p_x, p_y, p_z, 4 .. 9 = d_xx,
                              d_yy, d_zz, d_xy, d_xz, d_yz, 10 .. 19 = f_xxx, f_yyy,
                              f_zzz, f_xxy, f_xxz, f_xyy, f_yyz, f_xzz, f_yzz, f_xyz;
                              NULL = all s */
} orc_basis;

typedef struct {
    int64_t kept[4];     /* kept directed pair contributions: LL<-LL, LL<-SS, SS<-LL, SS<-SS */
    int64_t total[4];    /* all directed pair contributions of those class pairs */
    int64_t kept_gaunt;  /* LS<-LS */
    int64_t total_gaunt;
    int64_t tie_band;    /* |Q Q Dmax / tau - 1| < 1e-12 */
    double seconds_first_half;
    double seconds_second_half;
    int32_t threads;
} orc_stats;

/* Boys function F0(T) = int_0^1 exp(-T u^2) du. */
double orc_boys0(double T);

/* Boys function F_m(T) = int_0^1 u^{2m} exp(-T u^2) du, m >= 0. */
double orc_boys(int m, double T);

/* Coefficients multiplying the unnormalized primitives exp(-a r^2) so that
 * each contracted function has unit norm; out has sum(nprim) entries. */
void orc_norm_coefs(const orc_basis *b, double *out);
/* Primitive ERI over unnormalized Cartesian Gaussians: centre X, exponent x,
 * cartesian code cx (as in orc_basis.cart), Obara-Saika recursion. */
double orc_prim_eri_cart(double a, const double *A, int ca, double b, const double *B, int cb,
                         double c, const double *C, int cc, double d, const double *D, int cd);

/* Primitive integrals of the kernel r12_K r12_L / r12^3 over unnormalized
 * Cartesian Gaussians (arguments as orc_prim_eri_cart), out[K * 3 + L],
 * McMurchie-Davidson form. */
void orc_prim_eri3_cart(double a, const double *A, int ca, double b, const double *B, int cb,
                        double c, const double *C, int cc, double d, const double *D, int cd,
                        double out[9]);

/* Contracted ERI (mu nu | ka la) in chemists' notation; mu, nu index basis A,
 * ka, la index basis B. */
double orc_eri(const orc_basis *A, int mu, int nu, const orc_basis *B, int ka, int la);

/* Contracted integrals of the kernel r12_K r12_L / r12^3 (K, L = x, y, z),
 * out[K * 3 + L] = (mu^A nu^B | K L | ka^C la^D), the kernel of the gauge
 * integrals, Eq. (gaugeInt). */
void orc_eri3(const orc_basis *A, int mu, const orc_basis *B, int nu, const orc_basis *C, int ka,
              const orc_basis *D, int la, double out[9]);

/* Full tensor out[i][j][k][l] = (i^A j^B | k^C l^D). */
void orc_eri_tensor(const orc_basis *A, const orc_basis *B, const orc_basis *C,
                    const orc_basis *D, double *out);

/* Schwarz factors Q[mu][nu] = sqrt((mu^A nu^B | mu^A nu^B)), [NA][NB]. */
void orc_schwarz(const orc_basis *A, const orc_basis *B, double *Q);

/* Density bound Dmax[ka][la] = max over all ordered quaternion MO pairs (r,t)
 * and components y of |[conj(C^A_{ka r}) e C^B_{la t}]_y| where e = 1
 * (Coulomb, A = B) -- i.e. the infinity norm over all MO pairs of the
 * quaternion pair density. */
void orc_dmax_coulomb(int NA, const double *CA, int n, double *Dmax);

/* Gaunt density bound of the L-S pair (mu in L, nu in S): Dmax[mu][nu] = max
 * over K, all ordered (r,t) and components x of
 * |[conj(C^L_{mu r}) e_K C^S_{nu t} + conj(C^S_{nu r}) e_K C^L_{mu t}]_x|
 * with e_x = k, e_y = j, e_z = i; [NL][NS]. */
void orc_dmax_gaunt(int NL, const double *CL, int NS, const double *CS, int n, double *Dmax);

/* Definition route (unscreened): four-spinor integrals built from the literal
 * 4x4 operator matrices (identity for Coulomb, alpha_K for Gaunt) and
 * projected onto the quaternion basis.  spinor_out (nullable) receives the
 * complex spinor integrals (ab|cd) as interleaved re/im, [2n]^4 x 2.
 * imag_max (nullable) receives the largest |imaginary part| met in the
 * projection.  Returns 0, or -1 when the problem is too large for it. */
int orc_transform_def(const orc_basis *L, const orc_basis *S, const double *CL,
                      const double *CS, int n, int ham, double *G, double *spinor_out,
                      double *imag_max);

/* The paper's direct route: quaternion (Pauli scalar / vector) pair densities
 * in two-spinor arithmetic, density-weighted Cauchy-Schwarz screening per
 * directed pair contribution, first-half contraction, conversion and
 * second-half two-spinor contraction, projected onto the quaternion basis.
 *   tau         screening threshold; a contribution (mu nu <- ka la) is kept
 *               iff (Q_mn * Q_kl) * Dmax_kl >= tau.
 *   rows,nrows  restrict the bra pairs to this list of distinct indices into
 *               the concatenated bra pair list (LL pairs mu <= nu in nu-major
 *               order, then SS pairs likewise, then LS pairs mu-major); pass
 *               NULL for all pairs.
 *   do_second   0 = stop after the first half (timing samples), G untouched.
 *   G           output (when do_second); only bra pairs in range contribute.
 * Returns 0, or -1 on invalid arguments. */
int orc_transform_direct(const orc_basis *L, const orc_basis *S, const double *CL,
                         const double *CS, int n, int ham, double tau, const int64_t *rows,
                         int64_t nrows, int do_second, double *G, orc_stats *st);

/* First-half rows of the direct route for the selected bra pairs (same
 * indexing as orc_transform_direct's rows), in quaternion components:
 * Vq[r][K * 4 * npair + 4 * idx(p <= q) + y], npair = n (n + 1) / 2, idx counting
 * the MO pairs p <= q with p outer, K = 0 only (Coulomb rows) or K = x, y, z
 * (Gaunt rows); rows are 3 * 4 * npair wide when ham includes Gaunt, else
 * 4 * npair.  Coulomb: V^{pq}_y = sum_kept (mn|kl) [D~^{pq}_kl]_y with the
 * symmetrized quaternion density; Gaunt likewise with D^{K,pq}.
 * Returns 0, or -1 on invalid arguments. */
int orc_first_half_rows(const orc_basis *L, const orc_basis *S, const double *CL,
                        const double *CS, int n, int ham, double tau, const int64_t *rows,
                        int64_t nrows, double *Vq);

/* orc_first_half_rows for a subset of the MO-pair columns and, optionally,
 * a density bound given per pair of the concatenated list (dmax_in[np], as
 * for orc_transform_direct_dmax; NULL: computed here).  cols[ncols] are MO
 * pair indices idx(p <= q) (p outer); Vq[r][K * 4 * ncols + 4 * j + y] holds
 * MO pair cols[j].  Returns 0, or -1 on invalid arguments. */
int orc_first_half_rows_cols(const orc_basis *L, const orc_basis *S, const double *CL,
                             const double *CS, int n, int ham, double tau, const int64_t *rows,
                             int64_t nrows, const int64_t *cols, int64_t ncols,
                             const double *dmax_in, double *Vq);

/* Kramers-unrestricted (general) two-spinor input, the paper's own setting:
 * m spinors with coefficients c_{mu tau, a} given as planes C[4][N][m] (alpha
 * re, alpha im, beta re, beta im).  Output: the complex spinor MO integrals
 * (ab|cd), interleaved re/im, [m]^4 x 2.
 *   _def     unscreened definition route (literal four-spinor operators),
 *            m and the basis size limited as for orc_transform_def.
 *   _direct  the direct route with the same screening predicate, where
 *            Dmax_kl is the largest |real| or |imaginary| part of the pair
 *            density over all ordered spinor pairs (c, d): the Pauli-scalar
 *            density of both orderings (k l) and (l k) for Coulomb pairs, the
 *            sigma_K-weighted density of every K for Gaunt (L-S) pairs.
 * Return 0, or -1 on invalid arguments. */
int orc_transform_spinor_def(const orc_basis *L, const orc_basis *S, const double *CL,
                             const double *CS, int m, int ham, double *spinor_out);
int orc_transform_spinor_direct(const orc_basis *L, const orc_basis *S, const double *CL,
                                const double *CS, int m, int ham, double tau,
                                double *spinor_out, orc_stats *st);

/* The direct route with the density bound given per pair of the
 * concatenated list (dmax_in[np], same order as the bra pairs), for the
 * MO-driven variant whose bound covers one batch of MO pairs. */
int orc_transform_direct_dmax(const orc_basis *L, const orc_basis *S, const double *CL,
                              const double *CS, int n, int ham, double tau,
                              const double *dmax_in, double *G, orc_stats *st);

/* Number of bra pairs of the concatenated list for this ham. */
int64_t orc_num_bra_pairs(const orc_basis *L, const orc_basis *S, int ham);

#ifdef __cplusplus
}
#endif
#endif
