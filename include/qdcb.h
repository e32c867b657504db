/* qdcb.h -- C ABI of the MI355X quaternion Dirac-Coulomb(-Breit) AO->MO
 * two-electron integral transformation (arXiv 2606.04316).
 *
 * The library implements the paper's AO-driven direct transformation
 * (Sec. 2.4): scalar AO two-electron integrals over contracted Cartesian
 * Gaussians (s, p, d and f functions; restricted-kinetic-balance gradient functions
 * for the small component, Eq. RKB) are generated on the GPU, filtered by the quaternion-density-
 * weighted Cauchy-Schwarz bound (Sec. 2.5, Eq. SchwarzDen), contracted with
 * quaternion MO-pair densities in the first half (Eq. firsthalf, Eqs. Den and
 * QuaternionScatter) and with the MO coefficients in the second half
 * (Sec. 2.4.2, Eq. secondhalf).  The result is the quaternion MO integral
 * tensor (pq|rs) of the Dirac-Coulomb classes of Eq. (DCInt) and, for the
 * DCG Hamiltonian, the Gaunt classes of Eq. (GauntInt); the DCB Hamiltonian
 * adds the gauge classes of Eq. (gaugeInt).
 *
 * Conventions
 *   - All functions return a qdcb_status; 0 is success, negative is an error.
 *     On error no output buffer has been written and qdcb_last_error()
 *     returns a message for the calling thread.  No C++ exception crosses
 *     this boundary.
 *   - Basis: contracted Gaussians, s type (qdcb_basis_create) or Cartesian s,
 *     p, d and f components (qdcb_basis_create_cart), and the gradient functions of
 *     an s basis as the restricted-kinetic-balance small-component basis
 *     (qdcb_basis_create_rkb).  coefs multiply normalized primitives
 *     ((2a/pi)^{3/4} exp(-a r^2) for s); the library rescales every
 *     contracted function to unit self-overlap.  Bohr units.
 *   - MO coefficients (Eqs. Lspinor, Sspinor in the Kramers-paired quaternion
 *     form): planar float64 [4][N][n_mo], C = C0 + i C1 + j C2 + k C3.
 *     Quaternion MO p stands for the Kramers pair of two-spinors given by the
 *     columns of Q(C) = [[C0 + i C1, C2 + i C3], [-C2 + i C3, C0 - i C1]].
 *   - Output G: float64 [n][n][n][n][4][4]; G[p][q][r][s][x][y] is component
 *     x (bra) and y (ket) of the quaternion MO integral
 *       G^{xy}_{pqrs} = sum [conj(C_mu p) C_nu q]_x (mu nu|ka la) [conj(C_ka r) C_la s]_y
 *     summed over the integral classes of the Hamiltonian.  The 16 spinor
 *     integrals of the Kramers block are (ab|cd) = sum_xy G^{xy} Q(e_x)_ab Q(e_y)_cd.
 *   - Ownership: the caller owns every pointer it passes; the library copies
 *     what it keeps.  Library objects own their device memory.
 *   - Threading: a context may be shared between threads; a plan is used by
 *     one call at a time (a concurrent call on the same plan returns
 *     QDCB_E_BUSY).
 */
#ifndef QDCB_H
#define QDCB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QDCB_ABI_VERSION 1

typedef enum {
    QDCB_OK = 0,
    QDCB_E_INVALID = -1,     /* bad argument (non-finite input, exponent <= 0, sizes) */
    QDCB_E_NOMEM = -2,       /* device memory budget exceeded */
    QDCB_E_DEVICE = -3,      /* HIP runtime error */
    QDCB_E_UNSUPPORTED = -4, /* valid request this build does not implement */
    QDCB_E_BUSY = -5,        /* the plan is in use by another call (plans are not reentrant) */
    QDCB_E_ABORTED = -6      /* a block callback asked to stop */
} qdcb_status;

typedef enum {
    QDCB_HAM_LL = 0,  /* (LL|LL) only: the nonrelativistic-like large-component block */
    QDCB_HAM_DC = 1,  /* Dirac-Coulomb, Eq. (DCInt): LL|LL + LL|SS + SS|LL + SS|SS */
    QDCB_HAM_DCG = 2, /* DC plus the Gaunt term, Eqs. (breit) and (GauntInt) */
    QDCB_HAM_DCB = 3  /* DC plus the whole Breit term: Gaunt and the gauge term
                         (alpha_1 x r12) . (alpha_2 x r12) / (2 r12^3) of Eq. (breit),
                         whose integrals, Eq. (gaugeInt), carry the kernel
                         r12 r12^T / r12^3 over the same L-S products as Gaunt */
} qdcb_ham;

typedef enum { QDCB_PREC_FP64 = 0, QDCB_PREC_MIXED = 1 } qdcb_prec;

/* transform flags */
#define QDCB_PTR_DEVICE 0x1u /* CL, CS and G are device pointers (else host) */
/* Integral classes to include (no class bit: every class of the plan's
 * Hamiltonian).  QDCB_CLASS_COULOMB: the Dirac-Coulomb classes of Eq. (DCInt)
 * (LL|LL for QDCB_HAM_LL); QDCB_CLASS_GAUNT: the Gaunt classes of Eq.
 * (GauntInt), DCG and DCB plans; QDCB_CLASS_GAUGE: the gauge classes of Eq.
 * (gaugeInt), DCB plans only.  The output holds the sum of the selected
 * classes, so a transform with every class equals the sum of the
 * single-class ones (to rounding). */
#define QDCB_CLASS_COULOMB 0x2u
#define QDCB_CLASS_GAUNT 0x4u
#define QDCB_CLASS_GAUGE 0x8u

typedef struct qdcb_ctx qdcb_ctx;
typedef struct qdcb_basis qdcb_basis;
typedef struct qdcb_plan qdcb_plan;

/* ABI version compiled into the library (QDCB_ABI_VERSION). */
int qdcb_abi_version(void);

/* Message describing the last error on the calling thread ("" if none). */
const char *qdcb_last_error(void);

/* Context bound to HIP device `device`; hbm_budget_bytes caps the device
 * memory all plans of this context may hold (0 = 90% of the device). */
qdcb_status qdcb_ctx_create(int device, size_t hbm_budget_bytes, qdcb_ctx **out);
void qdcb_ctx_destroy(qdcb_ctx *ctx);

/* s-type contracted basis (host arrays, copied).  centers [nfunc][3],
 * nprim [nfunc] (>= 1), exps and coefs [sum nprim] with exps > 0.  Builds
 * the primitive-pair data of all function pairs and the Schwarz factors
 * Q_mn = sqrt((mn|mn)) (Eq. SchwarzDen) on the device; both stay resident
 * for the basis's lifetime and are shared by every plan that uses it. */
qdcb_status qdcb_basis_create(qdcb_ctx *ctx, int32_t nfunc, const double *centers,
                              const int32_t *nprim, const double *exps, const double *coefs,
                              qdcb_basis **out);

/* Basis of contracted Cartesian Gaussians of s, p, d or f type (the angular
 * momenta of the paper's basis sets, Sec. 2.5; each Cartesian component is a
 * function of its own).  Arguments as for qdcb_basis_create, plus cart
 * [nfunc] (host, copied): 0 = s, 1, 2, 3 = p_x, p_y, p_z, 4 .. 9 = d_xx,
 * d_yy, d_zz, d_xy, d_xz, d_yz, 10 .. 19 = f_xxx, f_yyy, f_zzz, f_xxy, f_xxz,
 * f_xyy, f_yyz, f_xzz, f_yzz, f_xyz, i.e. the monomials (x - A_x)^{l_x}
 * (y - A_y)^{l_y} (z - A_z)^{l_z} times exp(-a |r - A|^2); NULL = all s (the
 * call is then qdcb_basis_create).  coefs multiply normalized primitives,
 * (2a/pi)^{3/4} (4a)^{L/2} / sqrt(prod_k (2 l_k - 1)!!) times the monomial
 * and the Gaussian (L = l_x + l_y + l_z), and each contracted function is
 * rescaled to unit self-overlap.  A shell is the functions of one centre,
 * exponent set and coefficient set (three p, six Cartesian d, ten Cartesian
 * f).  Integrals with p functions are generated in McMurchie-Davidson form,
 * and bases with a d or f function take its general form for every
 * integral; Schwarz factors are per function pair, and primitive-pair
 * screening is not applied to pairs with a p, d or f function.  Plans over
 * such bases support every Hamiltonian (QDCB_HAM_DCB: the gauge integrals in
 * the same general form).  QDCB_E_INVALID for a code outside [0, 19]. */
qdcb_status qdcb_basis_create_cart(qdcb_ctx *ctx, int32_t nfunc, const double *centers,
                                   const int32_t *nprim, const double *exps,
                                   const double *coefs, const int32_t *cart,
                                   qdcb_basis **out);
void qdcb_basis_destroy(qdcb_basis *basis);

/* Restricted kinetic balance (Eq. RKB): chi^S_{mu tau} = (1/2c) (sigma . p)
 * chi^L_{mu tau}, so the small component of a two-spinor is, per spin
 * component, a combination of the 3 N gradient functions d_K chi_mu
 * (K = x, y, z), which are p functions for s-type chi_mu.
 * qdcb_basis_create_rkb builds them as a basis of 3 nfunc(L) normalized
 * Cartesian p functions (function 3 mu + K on chi_mu's centre), with
 * norms[3 mu + K] = ||d_K chi_mu|| (host, caller-owned, may be NULL).  L must
 * be s-only (QDCB_E_UNSUPPORTED otherwise) and on ctx's device
 * (QDCB_E_INVALID otherwise); 3 nfunc <= 65535.  A general
 * two-spinor DC plan (QDCB_PLAN_SPINOR) with L and this basis as S then gives
 * the four-component Dirac-Coulomb integrals of RKB spinors (all classes of
 * Eq. DCInt, with their 1/(2c^2) and 1/(8c^4) factors). */
qdcb_status qdcb_basis_create_rkb(qdcb_ctx *ctx, const qdcb_basis *L, double *norms,
                                  qdcb_basis **out);
/* Small-component planes over that gradient basis: out [4][3 nfunc][m]
 * (alpha re, alpha im, beta re, beta im; function 3 mu + K) from the RKB
 * coefficients PS [4][nfunc][m] of m two-spinors (same plane layout), the
 * norms of qdcb_basis_create_rkb and the speed of light c:
 * out_{(mu K) u} = (-i / 2c) norms[3 mu + K] sum_tau (sigma_K)_{u tau} PS_{mu tau}.
 * Host arrays, host arithmetic (no device work). */
qdcb_status qdcb_rkb_small_planes(int32_t nfunc, int32_t m, const double *PS,
                                  const double *norms, double c, double *out);

/* The same small components in the Kramers-restricted (quaternion) form:
 * the Kramers pair of quaternion MO p with RKB coefficients C^S [4][nfunc][n]
 * (planes C0..C3, as for qdcb_transform) has, over the gradient basis, the
 * quaternion coefficients
 *   out_{(mu K) p} = -(norms[3 mu + K] / 2c) e_K C^S_{mu p},  e_x = k, e_y = j, e_z = i,
 * out [4][3 nfunc][n], because sigma_K = -i Q(e_K) makes (-i / 2c) sigma_K Q(C)
 * the matrix Q of that quaternion.  A quaternion DC or DCG plan with L and
 * the gradient basis as S then gives the RKB four-component integrals of the
 * n Kramers pairs with half the MO-pair columns of the general two-spinor
 * route.  Host arrays, host arithmetic (no device work). */
qdcb_status qdcb_rkb_small_quat(int32_t nfunc, int32_t n, const double *CS, const double *norms,
                                double c, double *out);

/* Schwarz factors of the basis's own function pairs: Q[mu][nu] (host,
 * [nfunc][nfunc], symmetric). */
qdcb_status qdcb_basis_schwarz(const qdcb_basis *basis, double *Q);

/* Contracted AO integrals (mu nu | ka la), mu, nu in basis A and ka, la in
 * basis B, for nq quartets idx[q] = {mu, nu, ka, la} (host arrays), computed
 * by the library's device integral code.  out: host [nq]. */
qdcb_status qdcb_eri_quartets(const qdcb_basis *A, const qdcb_basis *B, int64_t nq,
                              const int32_t *idx, double *out);

/* Allocation-free variant of qdcb_eri_quartets, for callers that cannot
 * allocate device memory (harnesses that forbid hipMalloc, tight loops that
 * must not touch the allocator).  Same arguments, results and errors as
 * qdcb_eri_quartets (the same device integral code, so bitwise the same
 * values); its device staging (the quartet list, each quartet's
 * primitive-pair ranges and codes, the results: 56 bytes per quartet) lives
 * in one fixed array of the library on each device, sized for
 * QDCB_NOALLOC_MAX_QUARTETS quartets (about 14 MiB, held from library load to
 * process exit), instead of being allocated.  nq above that limit:
 * QDCB_E_INVALID, nothing computed.  Synchronous, on the null stream: it
 * returns when out is written, and is not for capture into a HIP graph.
 * Calls on one device share the array; the library serializes them (calls
 * that overlapped on one device would otherwise race).  A context must have
 * been created on the bases' device (QDCB_E_DEVICE otherwise). */
#define QDCB_NOALLOC_MAX_QUARTETS 262144
qdcb_status qdcb_eri_quartets_noalloc(const qdcb_basis *A, const qdcb_basis *B, int64_t nq,
                                      const int32_t *idx, double *out);

typedef struct {
    int32_t ham;       /* qdcb_ham */
    int32_t prec;      /* qdcb_prec */
    int32_t n_mo;      /* number of quaternion MOs n (Kramers pairs) */
    int32_t flags;     /* QDCB_PLAN_* bits, 0 by default */
    double tau;        /* Schwarz threshold: a directed contribution (mn <- kl) is
                          kept iff (Q_mn * Q_kl) * Dmax_kl >= tau, Eq. (SchwarzDen) */
    double tier_fp32;  /* QDCB_PREC_MIXED: a kept directed tile (b, k) with bound
                          B = max_b' Q * max_k (Q Dmax), b' over the bra tile and
                          its pair partner (tiles 2i, 2i + 1; the first half
                          contracts them together), is contracted in FP64 when
                          B >= tier_fp32, with FP32 MFMA operands when
                          tier_bf16 <= B < tier_fp32, else with BF16 operands (FP32
                          accumulation, power-of-2 block scales, V and the second
                          half in FP64).  Requires 0 <= tier_bf16 <= tier_fp32. */
    double tier_bf16;
} qdcb_plan_desc;

/* plan flags.  By default the eager transform generates one integral tile
 * per unique tile pair (b >= k) of the symmetric matrix (mn|kl) = (kl|mn)
 * whenever all of them fit the integral panel, and the contraction reads it
 * for both directed tasks (b, k) and (k, b) with the directed predicate
 * applied per element; QDCB_PLAN_DIRECTED_TILES generates one tile per
 * directed task instead (the results agree to rounding). */
#define QDCB_PLAN_DIRECTED_TILES 0x1u
/* QDCB_PREC_MIXED: assign tiers by B = max_b (Q Dmax) * max_k (Q Dmax), which
 * also bounds the bra-side coefficient products that carry a first-half
 * contribution into G (Dmax of the bra pair bounds |conj(C_mp) C_nq|), instead
 * of the screening bound max_b Q * max_k (Q Dmax). */
#define QDCB_PLAN_TIER_BY_G 0x2u
/* General (Kramers-unrestricted) two-spinor MOs, the paper's own setting
 * (Eqs. Lspinor, Sspinor with arbitrary complex c_{mu tau, p}): n_mo counts
 * spinors (not Kramers pairs) and qdcb_transform reads and writes
 *   CL [4][N_L][n_mo], CS [4][N_S][n_mo]   planes alpha re, alpha im, beta re,
 *                                          beta im of the coefficients;
 *   G  [n][n][n][n][2]                      the complex spinor integrals
 *                                          (pq|rs) (re, im), summed over the
 *                                          selected classes.
 * The first half contracts the Pauli-scalar pair densities (Coulomb) and the
 * sigma_K-weighted L-S pair densities (Gaunt) of the spinor pairs r <= s as
 * real and imaginary columns, screened with Dmax = the largest |re| or |im|
 * part of the pair density over all ordered spinor pairs.  Spinor pair i
 * (r <= s, r outer) occupies columns 4 floor(i/2) + 2 (i mod 2) (re) and + 1
 * (im), which is also the column layout of qdcb_plan_fetch_v.  Blocked output
 * (qdcb_transform_blocks) is not offered for these plans. */
#define QDCB_PLAN_SPINOR 0x4u
/* Row order of the pair spaces.  By default the pairs of each space, ordered
 * by Schwarz factor, are regrouped in bands of 8 x 64 rows by the number of
 * primitive pairs that survive primitive screening (decreasing), so that the
 * 64 rows of an integral tile have similar primitive loops (lanes of the
 * integral kernel idle less).  A tile's bound then spans its band's Schwarz
 * range, so somewhat more tile pairs are kept; on uneven contraction depths
 * the integral tiles gain more than the first half loses.
 * QDCB_PLAN_SCHWARZ_ROWS keeps the plain order by decreasing Schwarz factor
 * (tightest tile bounds; even contraction depths gain nothing from bands).
 * QDCB_PLAN_PRIM_BANDS names the default explicitly; setting both is
 * QDCB_E_INVALID.  Results agree to rounding across the orders. */
#define QDCB_PLAN_PRIM_BANDS 0x8u
#define QDCB_PLAN_SCHWARZ_ROWS 0x10u

/* Plan for transforming with fixed bases and n_mo.  S must be NULL for
 * QDCB_HAM_LL and non-NULL otherwise.  Orders the pairs of each integral
 * class space (Coulomb: LL and SS pairs; Gaunt, for DCG: ordered LS pairs) by
 * their Schwarz factor (regrouped in primitive bands unless QDCB_PLAN_SCHWARZ_ROWS) and allocates the per-transform device buffers; the
 * MO-pair columns are processed in chunks when they do not fit at once.
 * QDCB_E_NOMEM if even the smallest chunk does not fit the context budget. */
qdcb_status qdcb_plan_create(qdcb_ctx *ctx, const qdcb_basis *L, const qdcb_basis *S,
                             const qdcb_plan_desc *desc, qdcb_plan **out);
void qdcb_plan_destroy(qdcb_plan *plan);

/* Device bytes the plan holds (pair data excluded: it belongs to the bases). */
qdcb_status qdcb_plan_footprint(const qdcb_plan *plan, size_t *bytes);

/* Device bytes a plan for (L, S, desc) needs to hold every MO-pair column at
 * once (no column chunking), with integral panels for up to 65,536 tiles per
 * pair space or the full set of tiles, whichever is smaller: the admission
 * size a request loop reserves before creating the plan in a context of that
 * budget.  Host-side arithmetic only; nothing is allocated. */
qdcb_status qdcb_plan_estimate(const qdcb_basis *L, const qdcb_basis *S,
                               const qdcb_plan_desc *desc, size_t *bytes);

typedef struct {
    double ms_total;         /* wall time of the transform on its stream */
    double ms_density;       /* pair densities + Dmax + tile bounds */
    double ms_screen;        /* task lists */
    double ms_eri;           /* AO integral tiles */
    double ms_first_half;    /* integral-density contraction */
    double ms_second_half;   /* MO-coefficient contraction and output */
    int64_t kept[4];         /* kept directed pair contributions LL<-LL, LL<-SS, SS<-LL, SS<-SS */
    int64_t total[4];        /* all directed pair contributions of the same class pairs */
    int64_t kept_gaunt;      /* LS<-LS (DCG, DCB: the Gaunt and gauge terms share them) */
    int64_t total_gaunt;
    int64_t tiles_kept;      /* kept (bra tile, ket tile) pairs */
    int64_t tiles_total;
    double flops_first_half; /* algorithmic: 2 * columns * kept contributions (Gaunt: 3
                                columns per MO-pair column, gauge: 9) */
    double flops_second_half;
    double flops_mfma;       /* MFMA flops issued by the first-half kernel (incl. masked
                                elements of kept tiles), summed over the column chunks */
    int32_t n_batches;       /* first-half kernel launches */
    int32_t n_chunks;        /* MO-pair column chunks (MO-driven variant: batches) */
    int32_t graph_replay;    /* 1: produced by qdcb_plan_replay */
    int32_t graph_fallback;  /* 1: the replay's kept tiles outgrew the panel; redone eagerly */
    int64_t tiles_made;      /* integral tiles generated (unique or directed, all chunks) */
    int64_t tiles_tier[3];   /* mixed: kept directed tiles contracted in FP64, FP32, BF16
                                (eager transforms) */
    double ms_tier[3];       /* mixed: first-half time per tier (eager transforms) */
    int32_t classes;         /* integral classes included, bits: 1 Coulomb, 2 Gaunt, 4 gauge */
    int32_t reserved;
} qdcb_stats;

/* Transform.  CL [4][N_L][n], CS [4][N_S][n] (NULL for LL), G [n^4][4][4];
 * host or device pointers per QDCB_PTR_DEVICE; class bits select integral
 * classes (see QDCB_CLASS_COULOMB).  Work is enqueued on hip_stream (a
 * hipStream_t; NULL = the null stream); the call returns after G is
 * complete.  stats may be NULL (its kept counts and tiles cover the selected
 * classes). */
qdcb_status qdcb_transform(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                           uint32_t flags, void *hip_stream, qdcb_stats *stats);

/* Blocked output, for callers that do not hold all of G at once.  The same
 * transformation as qdcb_transform, delivered in blocks of MO pairs (r <= s)
 * in the canonical order (r outer, s inner; pair index i of (r, s) is
 * r n - r (r - 1) / 2 + s - r).  For each block [i0, i1) the library calls
 * cb(user, i0, i1, B, on_device) after the block is complete, with
 *   B[i - i0][p][q][0][x][y] = G[p][q][r][s][x][y],
 *   B[i - i0][p][q][1][x][y] = G[p][q][s][r][x][y]   ((r, s) = pair i),
 * n^2 * 32 doubles per pair.  B is a device pointer (on_device = 1) when
 * flags has QDCB_PTR_DEVICE, else host memory; it belongs to the library and
 * is valid only during the call.  Blocks come in increasing order, each pair
 * exactly once; their size follows the plan's second-half slice.  A nonzero
 * return from cb stops the transformation: QDCB_E_ABORTED.  The callback runs
 * on the calling thread and must not use the same plan (QDCB_E_BUSY).  flags:
 * QDCB_PTR_DEVICE (CL, CS and the blocks on the device) and the class bits. */
typedef int (*qdcb_block_cb)(void *user, int64_t i0, int64_t i1, const double *B,
                             int on_device);
qdcb_status qdcb_transform_blocks(qdcb_plan *plan, const double *CL, const double *CS,
                                  qdcb_block_cb cb, void *user, uint32_t flags,
                                  void *hip_stream, qdcb_stats *stats);

/* Re-transforms (e.g. successive orbital updates): record one whole
 * transformation of the device buffers CL, CS -> G (which must stay valid)
 * into a HIP graph on the non-null stream hip_stream; every step, including
 * screening and task-list construction, stays on the device in fixed-capacity
 * buffers.  qdcb_plan_replay launches it on hip_stream after the caller has
 * written new coefficients into CL and CS, waits for it, and fills stats; if
 * the new coefficients keep more integral tiles than the plan's panel holds,
 * the replay is redone eagerly and stats->graph_fallback is set. */
qdcb_status qdcb_plan_capture(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                              void *hip_stream);
qdcb_status qdcb_plan_replay(qdcb_plan *plan, void *hip_stream, qdcb_stats *stats);

/* Intermediates of the plan's last transform, copied to host memory.
 *   QDCB_FETCH_DMAX        float64 [P]: density bound Dmax of every Coulomb pair
 *                          in canonical order (LL pairs mu <= nu by nu-major
 *                          packing nu(nu+1)/2 + mu, then SS pairs likewise).
 *   QDCB_FETCH_Q           float64 [P]: Schwarz factors in the same order.
 *   QDCB_FETCH_DMAX_GAUNT  float64 [N_L*N_S]: Gaunt density bound of the LS pair
 *                          (mu in L, nu in S) at mu*N_S + nu (DCG plans).
 *   QDCB_FETCH_Q_GAUNT     float64 [N_L*N_S]: Schwarz factors of the LS pairs. */
#define QDCB_FETCH_DMAX 1
#define QDCB_FETCH_Q 2
#define QDCB_FETCH_DMAX_GAUNT 3
#define QDCB_FETCH_Q_GAUNT 4
qdcb_status qdcb_plan_fetch(const qdcb_plan *plan, int32_t what, void *host_out,
                            size_t bytes);

/* First-half rows V (Eq. firsthalf) of the plan's last transform for the bra
 * pairs listed in pairs[npairs] (host), in quaternion components, for parity
 * checks at full size.  Pair indices follow the concatenated list: LL pairs
 * mu <= nu at nu (nu + 1) / 2 + mu, then SS pairs likewise from nLL, then
 * (DCG) LS pairs mu * N_S + nu from nLL + nSS.  out (host) is [npairs][W] with
 * W = (DCG ? 3 : 1) * 4 * npair_mo, npair_mo = n (n + 1) / 2; column
 * K * 4 * npair_mo + 4 * idx + y holds component y of MO pair idx (p <= q, p
 * outer) for Pauli component K of a Gaunt row; Coulomb rows fill K = 0 and
 * leave the rest 0.  When the plan processes its MO-pair columns in chunks, V
 * holds the last chunk only: columns of the other MO pairs are set to NaN. */
qdcb_status qdcb_plan_fetch_v(const qdcb_plan *plan, const int64_t *pairs, int64_t npairs,
                              double *out);

/* Launch choices of a plan: tile shapes and schedules that change how fast a
 * transform runs, not what it computes.  Integral tiles and first-half rows
 * are bitwise the same under every choice; the second-quarter tile changes
 * the summation order of that GEMM only (results agree to rounding).
 *   eri_sched  0: one workgroup per unique integral tile, in list order;
 *              1: a persistent integral launch (two workgroups per compute
 *                 unit) that takes the unique tiles from a device queue in
 *                 order of decreasing primitive-quartet count (longest first,
 *                 for bases of uneven contraction depth).  Applies when the
 *                 transform generates unique tiles (see QDCB_PLAN_DIRECTED_TILES).
 *   fh_order   0: XCD-aware workgroup order of the first-half contraction
 *                 (each XCD's L2 shares integral tiles and density rows);
 *              1: plain order, bra-tile pairs fastest.
 *   sq_tile    64 or 128: edge of the output tiles of the second half's second
 *              quarter (G_c = conj(C)^T W_c); 128 requires an even n_mo.
 * A new plan starts from eri_sched 1, fh_order 0 and sq_tile 128 when n_mo is
 * even and at least 128, else 64. */
typedef struct {
    int32_t eri_sched;
    int32_t fh_order;
    int32_t sq_tile;
    int32_t reserved;  /* 0 */
} qdcb_tune;

/* Set or read the launch choices.  QDCB_E_INVALID for a value outside the
 * lists above (sq_tile 128 with an odd n_mo included). */
qdcb_status qdcb_plan_set_tune(qdcb_plan *plan, const qdcb_tune *tune);
qdcb_status qdcb_plan_get_tune(const qdcb_plan *plan, qdcb_tune *tune);

/* MO-driven variant, for comparison with the AO-driven transformation (the
 * paper's Fig. 2 algorithms), quaternion plans only (QDCB_E_UNSUPPORTED for
 * spinor plans): pairs > 0 processes the MO pairs (r <= s in the canonical
 * order) in batches of that many, each with the density bound Dmax of its own pairs, its own
 * screening and task lists, and its own integral tiles; the results agree
 * with the AO-driven ones to rounding at tau = 0 and differ by what each
 * batch's tighter bound screens at tau > 0.  stats->kept sums the batches.
 * 0 (default) is the AO-driven transformation: one bound over all MO pairs
 * and integral tiles computed once.  Captures are not offered for pairs > 0. */
qdcb_status qdcb_plan_set_mo_batch(qdcb_plan *plan, int32_t pairs);

/* Shape key of a plan for the tuning cache: the Hamiltonian, precision,
 * n_mo, basis sizes, largest contraction depths, tau, tile counts and the
 * device's compute-unit count, as one line of text (no quotes or newlines).
 * QDCB_E_INVALID when len is too small (256 bytes always suffice). */
qdcb_status qdcb_plan_tune_key(const qdcb_plan *plan, char *buf, size_t len);

/* Tuning cache: a text file of JSON lines
 *   {"key": "<shape key>", "eri_sched": E, "fh_order": F, "sq_tile": T}
 * Lookup takes the last line with the given key (*found = 0 when none, also
 * when the file does not exist); store appends a line.  Host file access only:
 * neither needs a device. */
qdcb_status qdcb_tune_cache_lookup(const char *path, const char *key, qdcb_tune *tune,
                                   int32_t *found);
qdcb_status qdcb_tune_cache_store(const char *path, const char *key, const qdcb_tune *tune);

typedef struct {
    qdcb_tune chosen;       /* also set on the plan */
    int32_t from_cache;     /* 1: taken from the cache, nothing timed */
    int32_t trials;         /* timed transforms (the warm-up excluded) */
    double ms_eri[2];       /* best integral-tile time per eri_sched value (NaN: untimed) */
    double ms_first_half[2];/* best first-half time per fh_order value */
    double ms_second_half[2];/* best second-half time per sq_tile (64, 128) */
} qdcb_tune_report;

/* Autotuner.  Unless the cache holds the plan's key, runs one warm-up and four
 * timed transforms of the given coefficients that alternate between the two
 * values of every choice, each limited to the first MO-pair column chunk (the
 * integral tiles are generated in full, the contractions cover that chunk),
 * times each stage with HIP events on hip_stream, and keeps per choice the
 * value of the faster stage (the first value unless the other is faster by
 * more than 1%).  Arguments as for qdcb_transform; G is used as scratch and
 * its contents are unspecified afterwards.  cache_path may be NULL, in which
 * case the environment variable QDCB_TUNE_CACHE names the cache file if set;
 * with a cache file the result is appended to it.  report may be NULL. */
qdcb_status qdcb_plan_autotune(qdcb_plan *plan, const double *CL, const double *CS, double *G,
                               uint32_t flags, void *hip_stream, const char *cache_path,
                               qdcb_tune_report *report);

#ifdef __cplusplus
}
#endif
#endif
