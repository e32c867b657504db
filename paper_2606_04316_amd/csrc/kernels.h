// kernels.h -- launchers of the qdcb HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace qdcb {

// ---- basis: normalization, primitive pairs, Schwarz factors (k_basis.hip)
// cart: per function 0 = s, 1..3 = p_x, p_y, p_z (NULL: all s).
void launch_norm_coefs(int nfunc, const int32_t *prim_first, const double *exps,
                       const double *coefs, const int32_t *cart, double *nc, hipStream_t s);
// Primitive-pair data of pairs (mu[i] in A, nu[i] in B), written at pair_first[i]
// (out.pa / out.pb too when set; cartA, cartB as for launch_norm_coefs).
void launch_pair_data(int64_t npairs, const int32_t *mu, const int32_t *nu,
                      const int64_t *pair_first, const double *centA, const int32_t *firstA,
                      const double *expA, const double *ncA, const int32_t *cartA,
                      const double *centB, const int32_t *firstB, const double *expB,
                      const double *ncB, const int32_t *cartB, PrimPairs out, hipStream_t s);
// Q[i] = sqrt((i|i)) over the primitive pairs [pair_first[i], pair_first[i+1]).
// code: per pair pair_code(cf, cg) for Cartesian bases, else NULL.
void launch_schwarz(int64_t npairs, const int64_t *pair_first, PrimPairsC pp,
                    const int32_t *code, double *Q, hipStream_t s);
// Primitive-pair screening: kept[r] = number of the cnt[r] primitive pairs of
// row r (starting at src_first[r]) whose Schwarz weight exceeds eps times the
// row's mean weight; rows with code[r] != 0 (a p, d or f function) keep all.
void launch_prim_count(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                       const int32_t *code, PrimPairsC src, double eps, int32_t *kept,
                       hipStream_t s);
// Gather pair rows into a new order: row r takes its kept primitive pairs
// (same criterion) from src_first[r] and stores them from dst_first[r] on.
void launch_gather_pairs(int64_t nrows, const int64_t *src_first, const int32_t *cnt,
                         const int32_t *code, const int64_t *dst_first, PrimPairsC src,
                         PrimPairs dst, double eps, hipStream_t s);
// ERIs of explicit quartets (test entry point): out[q] = (pair a[q] | pair b[q]);
// codes[2q], codes[2q+1]: the two pair codes (NULL for s-only bases).
void launch_eri_list(int64_t nq, const int64_t *a_first, const int64_t *b_first,
                     const int32_t *a_cnt, const int32_t *b_cnt, const int32_t *codes,
                     PrimPairsC A, PrimPairsC B, double *out, hipStream_t s);

// ---- densities (k_density.hip)
struct DensityArgs {
  int gaunt;              // 0: Coulomb rows (LL/SS), 1: Gaunt rows (LS)
  int bound_only;         // 1: Dmax over the MO pairs [i0, i1), no D writes
  int64_t nrows;          // padded pair rows
  int n;                  // MOs
  int npair_mo;           // n(n+1)/2
  int i0, i1;             // MO-pair range written (or bounded)
  int64_t ld;             // row stride of D
  int64_t ldK;            // Gaunt: stride between the K blocks of a row
  const int32_t *cls;     // [nrows] 0 = L, 1 = S (Gaunt: 0), -1 = padding
  const int32_t *mu;      // [nrows]
  const int32_t *nu;      // [nrows]
  const double *CL;       // [4][NL][n]
  const double *CS;       // [4][NS][n]
  int NL, NS;
  const int32_t *rs;      // [npair_mo]: r | s << 16 (spinor mode: [2 npair_mo] spinor pairs)
  double *D;              // [nrows][ld]
  double *Dmax;           // [nrows]
  // general two-spinor mode: C planes are alpha re, alpha im, beta re, beta im
  // of n spinors; npair_mo counts groups of two spinor pairs (c <= d), nspair
  // the spinor pairs; pair i = 2 g + h fills columns 4 g + 2 h (re) and + 1 (im)
  int spinor = 0;
  int nspair = 0;
};
void launch_density(const DensityArgs &a, hipStream_t s);

// ---- screening (k_screen.hip)
// Tile bounds: Qmax[t] = max Q, Bmax[t] = max Q*Dmax over the 64 rows of tile t,
// and (when Dtmax is not NULL) Dtmax[t] = max Dmax.
void launch_tile_bounds(int ntiles, const double *Q, const double *Dmax, double *Qmax,
                        double *Bmax, double *Dtmax, hipStream_t s);
// Block-scale exponent of the reduced tiers: the e with bound < 2^e (0 for a
// zero bound).
__device__ __forceinline__ int scale_exp(double bound) {
  int e = 0;
  (void)frexp(bound, &e);
  return bound > 0.0 ? e : 0;
}

// Precision tiers of the directed tasks: tier 0 (FP64) when the tile bound
// B = max(Qmax[b], Qmax[b ^ 1]) * Bmax[k] >= t32, tier 1 (FP32) when >= t16,
// else tier 2 (BF16); gbound = 1 uses max(Bmax[b], Bmax[b ^ 1]) * Bmax[k]
// instead (bra-side density included).  The bra bound is the larger of the
// pair (b, b ^ 1), which the first half contracts together.  Each
// bra tile's ordered list tasks[slot_base[b] + i] (i < count[b]) is split into
// three ordered sub-lists stored in its own segment: ttasks[slot_base[b] +
// toff[t*ntiles + b] + i] for i < tcount[t*ntiles + b], with trank = the
// task's rank i in the full list (its panel slot is slot_base[b] + rank) and
// tdesc = the entry's descriptor for the reduced tiers: the 16-row steps bra
// tile b needs (1 + the steps s >= 1 with Qmax[b] sthr[4 k + s] >= tau (1 -
// 1e-12); 4 without sthr) | (eI + 1024) << 3 | (eD + 1024) << 14, with eI =
// scale_exp(Qmax[b] Qmax[k]) and eD = scale_exp(2 Dtmax[k]).
void launch_tier_split(int ntiles, const double *Qmax, const double *Bmax, const double *Dtmax,
                       const double *sthr, double tau, int gbound, double t32, double t16,
                       const int64_t *slot_base, const int32_t *count, const int32_t *tasks,
                       int32_t *ttasks, int32_t *trank, int32_t *tdesc, int32_t *tcount,
                       int32_t *toff, hipStream_t s);
// count[b] = number of ket tiles k with Qmax[b]*Bmax[k] >= tau*(1-1e-12).
void launch_screen_count(int ntiles, const double *Qmax, const double *Bmax, double tau,
                         int32_t *count, hipStream_t s);
// tasks[slot_base[b] + j] = j-th kept ket tile of bra tile b (ascending) and
// task_bra[slot_base[b] + j] = b, for b in [b0,b1).
void launch_screen_fill(int b0, int b1, int ntiles, const double *Qmax, const double *Bmax,
                        double tau, const int64_t *slot_base, int32_t *tasks,
                        int32_t *task_bra, hipStream_t s);

// Directed slot map: dmap[b*ntiles + k] = slot of the kept task (b, k), as
// written by launch_screen_fill (slots must fit int32).
void launch_screen_fill_map(int ntiles, const double *Qmax, const double *Bmax, double tau,
                            const int64_t *slot_base, int32_t *dmap, hipStream_t s);
// Unique tile pairs (k <= b, either direction kept): counts per row, then the
// ordered fill with utask_k/utask_b at ubase[b] + rank and, per unique pair,
// the directed slots of (b, k) and (k, b) from dmap (-1: direction not kept).
void launch_screen_count_u(int ntiles, const double *Qmax, const double *Bmax, double tau,
                           int32_t *ucount, hipStream_t s);
void launch_screen_fill_u(int ntiles, const double *Qmax, const double *Bmax, double tau,
                          const int64_t *ubase, const int32_t *dmap, int32_t *utask_k,
                          int32_t *utask_b, int32_t *uslot_bk, int32_t *uslot_kb,
                          hipStream_t s);
// Device-side scan of the counts: slot_base[b], *total, *overflow = total > capacity.
void launch_scan_counts(int ntiles, const int32_t *count, int64_t *slot_base, int64_t *total,
                        int64_t capacity, int32_t *overflow, hipStream_t s);
// Zero n 64-bit counters with a kernel (safe inside captured graphs).
void launch_zero_u64(unsigned long long *p, int n, hipStream_t s);

// Intra-tile row order (k_screen.hip): within each tile, rows ranked by
// decreasing Q Dmax (ties by row): perm[64 t + i] = the tile-local row at
// position i, sthr[4 t + s] = the Q Dmax at position 16 s.
void launch_tile_order(int ntiles, const double *Q, const double *Dmax, int32_t *perm,
                       double *sthr, hipStream_t s);
// Row data in that order: wQ, wDmax, wcls, wmu, wnu (and wcode when code is
// set) of position i are row perm[i]'s; each tile's primitive pairs keep the
// tile's range and are regrouped by position (wrow_first, wpp).
void launch_gather_rows(int ntiles, const int32_t *perm, const double *Q, const double *Dmax,
                        const int32_t *cls, const int32_t *mu, const int32_t *nu,
                        const int32_t *code, const int64_t *row_first, PrimPairsC pp, double *wQ,
                        double *wDmax, int32_t *wcls, int32_t *wmu, int32_t *wnu,
                        int32_t *wcode, int64_t *wrow_first, PrimPairs wpp, hipStream_t s);

// *out += the 16-row steps the first half runs over the directed task lists
// with that order (per task: 1 + the steps s >= 1 that pass against the bra
// tile's Qmax).
void launch_step_work(int ntiles, const int64_t *slot_base, const int32_t *count,
                      const int32_t *tasks, const double *Qmax, const double *sthr, double tau,
                      unsigned long long *out, hipStream_t s);

// ---- AO integral tiles (k_eri.hip)
struct EriTileArgs {
  const int64_t *d_total = nullptr;  // graph mode: slots beyond *d_total (or the
  int64_t cap = 0;                   // panel capacity cap) exit at once
  const int32_t *overflow = nullptr;  // graph mode: nothing to do when set
  // unique mode (uslot_bk != NULL): slot i is the unique pair (task_bra[i] >=
  // tasks[i]); an element is computed when either direction is kept and is
  // written, masked per direction, to directed slot uslot_bk[i] as is and to
  // uslot_kb[i] transposed (-1: that direction has no tile); both directions
  // are counted
  const int32_t *uslot_bk = nullptr, *uslot_kb = nullptr;
  const double *boys = nullptr;  // [BOYS_N][8] Taylor table of F0 (see common.h)
  // Cartesian bases: per sorted row its pair code (see common.h), and the
  // table [BOYS_N][BOYS_LDC] of (2/sqrt(pi)) F_k(T_i), k < BOYS_LDC; the
  // integral launches then run the Cartesian (s, p) tile kernels
  const int32_t *code = nullptr;
  const double *boysc = nullptr;
  // bases with d functions: the general tiles (codes as above) with the table
  // [BOYS_N][BOYS_LDG] of (2/sqrt(pi)) F_k(T_i), k < BOYS_LDG
  const double *boysg = nullptr;
  // the largest Hermite order bound of the general tiles: 2 when the rows
  // hold s and p functions only, 4 with d and no f functions, else 6 (the
  // kernels without the larger forms)
  int gen_tmax = 6;
  const int32_t *tasks;       // [slots] ket tile per slot
  const int32_t *task_bra;    // [slots] bra tile per slot
  int64_t slot0;              // slot index of the panel buffer's first entry
  const int64_t *row_first;   // [nrows+1] primitive-pair offsets of the sorted rows
  PrimPairsC pp;
  const double *Q;            // [nrows]
  const double *Dmax;         // [nrows]
  const int32_t *cls;         // [nrows]
  double tau;
  double *panel;              // [slots][64 ket][64 bra] ([slots][6][64][64] for gauge tiles)
  unsigned long long *kept;   // [4] kept directed contributions per class pair, or NULL
  // gauge tiles (launch_eri_gauge_tiles*): boys3 = [BOYS_N][BOYS_LD] table of
  // (2 / sqrt(pi)) F_k(T_i), k = 0 .. 9; gauge_diag = -1/2 makes the gauge
  // tiles B_KL below, +1/2 the Breit tiles B_KL + delta_KL (mn|kl) (Gaunt and
  // gauge terms in one)
  const double *boys3 = nullptr;
  double gauge_diag = -0.5;
};
void launch_eri_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s);
// Persistent integral launch of nblocks workgroups over the tasks order[i],
// i < n (n = min(*a.d_total, a.cap) when a.d_total is set, else n_host); the
// queue counter *qctr must be 0 at launch.
void launch_eri_tiles_queue(const EriTileArgs &a, const int32_t *order, unsigned long long *qctr,
                            int64_t n_host, int nblocks, hipStream_t s);
// Gauge-term tiles of the L-S space, same task lists and masks as the Gaunt
// tiles: panel slot s holds the six tiles (K, L) = xx, xy, xz, yy, yz, zz of
//   B_KL(mn, kl) = ((mn| r_K r_L / r^3 |kl) - delta_KL (mn|kl)) / 2
// (symmetric in K, L and under bra <-> ket), each [64 ket][64 bra].
void launch_eri_gauge_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s);
void launch_eri_gauge_tiles_queue(const EriTileArgs &a, const int32_t *order,
                                  unsigned long long *qctr, int64_t n_host, int nblocks,
                                  hipStream_t s);
// Longest-first order of n unique tile tasks (n as for launch_eri_tiles_queue,
// from d_total/cap or n_host): order lists the task indices by decreasing
// floor(log2(bra primitive pairs x ket primitive pairs)) of their tiles (order
// within a class unspecified).  work: LPT_WORK 64-bit words; its last word is
// the queue counter of the integral launch, zeroed here.
constexpr int LPT_CLASSES = 64;
constexpr int LPT_WORK = 2 * LPT_CLASSES + 1;
void launch_lpt_order(int64_t n_host, const int64_t *d_total, int64_t cap, int64_t grid_cap,
                      const int32_t *task_k, const int32_t *task_b, const int64_t *row_first,
                      unsigned long long *work, int32_t *order, hipStream_t s);

// ---- first-half contraction (k_gemm.hip)
struct FirstHalfArgs {
  const int32_t *overflow = nullptr;  // graph mode: nothing to do when set
  // tier sub-lists (NULL: the full directed lists): bra tile b's list starts at
  // slot_base[b] + toff[b], and entry e's panel slot is slot_base[b] + rank[e]
  const int32_t *toff = nullptr, *rank = nullptr;
  // per-tile bounds Qmax (step skipping); reduced tiers: the entries'
  // descriptors (launch_tier_split) and the scaled FP32 density rows
  const double *Qmax = nullptr;
  const int32_t *tdesc = nullptr;
  const float *Dlo = nullptr;
  int b0, b1;
  const int64_t *slot_base;
  const int32_t *count;
  const int32_t *tasks;
  int64_t slot0;
  const double *panel;   // [slots][64][64]
  const double *D;       // [nrows][ld]
  double *V;             // [nrows][ld]
  int64_t ld;
  int ncol_tiles;        // ld / 128
  // workgroup order: 0 = XCD-aware (with at least 8 column slices), 1 = plain
  // (bra-tile pairs fastest); the order does not change any result
  int plain_order = 0;
  // intra-tile row order of the integral tiles and density rows (NULL: the
  // rows' own order): position i of tile t is row 64 t + perm[64 t + i], and V
  // rows are written (and, when adding, read) through it.  sthr[4 t + s]: the
  // largest Q Dmax of the 16 rows of step s of tile t in that order
  // (decreasing in s); a task skips the steps whose rows fail the predicate
  // against every bra row of its tile (Qmax[bra tile] * sthr < tau (1 - 1e-12)):
  // their integrals are masked zeros, so the result is the same bits.
  const int32_t *perm = nullptr;
  const double *sthr = nullptr;
  double tau = 0.0;
};
void launch_first_half(const FirstHalfArgs &a, hipStream_t s);
// Gauge term (FP64): V[mn][K ldK + col] (+)= sum_L sum_kl B_KL(mn, kl)
// D~[kl][L ldK + col] with the six-tile gauge panel slots (ld = 3 ldK,
// ncol_tiles = ldK / 128); accumulate = 1 adds to V (after the Gaunt term),
// 0 stores.
void launch_first_half_gauge(const FirstHalfArgs &a, int64_t ldK, int accumulate,
                             hipStream_t s);
// Reduced-precision tiers: V += the tier's contributions, computed with FP32
// (tier 1) or BF16 (tier 2) MFMA operands and FP32 accumulation, over the
// tier sub-lists (toff, rank, tdesc), from the tiles rounded by
// launch_panel_lo and the density rows of Dlo.
void launch_first_half_lp(const FirstHalfArgs &a, int tier, hipStream_t s);
// Rounds the integral tiles of the FP32 and BF16 sub-lists of bra tiles
// [b0, b1) once, in their own panel slots (after the tiles are made, before
// any reduced-tier contraction reads them): x 2^-eI to FP32 [j][m] or to BF16
// [j / 4][m][j % 4] at the start of the slot.  Run once per generation of a
// tile: a second pass would read rounded bytes as FP64.
struct PanelLoArgs {
  const int32_t *overflow = nullptr;  // graph mode: nothing to do when set
  int b0, b1, ntiles;
  const int64_t *slot_base;
  const int32_t *tcount, *toff, *rank, *tdesc;  // [3][ntiles] counts, offsets; entries
  int64_t slot0;
  double *panel;  // [slots][64][64]
};
void launch_panel_lo(const PanelLoArgs &a, hipStream_t s);
// Dlo[r][c] = D[r][c] 2^-scale_exp(2 Dtmax[r / 64]) in FP32 for rows [0, rows)
// of stride ld (a multiple of 4): the reduced tiers' density operand.
void launch_density_lo(int64_t rows, int64_t ld, const double *D, const double *Dtmax, float *Dlo,
                       hipStream_t s);

// Batched FP64 GEMM, row-major: C[b] = alpha * op(A[b]) * B[b] + beta * C[b].
// op(A) = A (transA = 0, A[m][k] at m*lda + k) or A^T (transA = 1, A[k][m] at k*lda + m).
// tri_n > 0 (a multiple of 16): row m is (x, p) = (m / tri_n, m % tri_n) and
// column n is q; 16 x 16 blocks whose every p exceeds every q are skipped.
void launch_dgemm_batched(int transA, int M, int N, int K, double alpha, const double *A,
                          int64_t lda, int64_t strideA, const double *B, int64_t ldb,
                          int64_t strideB, double beta, double *C, int64_t ldc,
                          int64_t strideC, int batch, hipStream_t s, int tri_n = 0);

// Gathered GEMM, 128 x 128 tiles: for every batch b < nb, c < nc and j < J,
//   C[c * ldc_c + b * ldc_b + j] (+)= sum_{k < K} V[row(b, k) * ld + col0 + c] * B[b * sbB + k * ldb + j]
// with row(b, k) = rowmap[b * sb + k * sk], or k when rowmap is NULL; "+=" when
// accumulate is set.  Serves the second half's first quarter straight from
// the first-half rows (the dense V of a column is never formed) and, with
// identity rows, its second quarter.  col0, ld, ldb, sbB and J must be even
// (16-byte rows, two columns per lane).
struct GatherGemmArgs {
  const double *V;
  int64_t ld, col0;
  const int32_t *rowmap;
  int64_t sb, sk;
  int nc, K, J, nb;
  const double *B;
  int64_t ldb, sbB;
  double *C;
  int64_t ldc_c, ldc_b;
  int accumulate;
  // workgroup order: the tiles that share one operand tile run consecutively
  // on one XCD (one L2): the J tiles of an (nc tile, batch) share the A tile
  // (share_b = 0), the nc tiles of a (J tile, batch) share the B tile
  // (share_b = 1)
  int share_b = 0;
  // tri_n > 0 (a multiple of 16): output row c is (x, p) = (c / tri_n,
  // c % tri_n) and column j is q; 16 x 16 blocks whose every p exceeds every q
  // are neither computed nor stored (the p > q half is filled from p < q)
  int tri_n = 0;
};
void launch_gather_gemm(const GatherGemmArgs &a, hipStream_t s);

// ---- second half (k_second.hip)
// Call[nu][z*n + q] = C[z][nu][q] and Chat[(mu,z)][(x,p)] = L(a)[x][z] with
// a = conj(C_mu p) * e (e = 1 for unit < 0, else e_x = k, e_y = j, e_z = i for
// unit = 0, 1, 2) and L(a) the matrix of left multiplication by a.
void launch_build_coef_mats(int N, int n, const double *C, int unit, double *Call,
                            double *Chat, hipStream_t s);
// General two-spinor mode.  K < 0: Call[nu][z*n + q] = C[z][nu][q] and Chat, the
// matrix of the conjugated left factor with two output planes (re, im):
// G_c[(x, p)][q] = sum_(mu, z) Chat[(mu, z)][(x, p)] W_c[(mu, z)][q] is
// sum_tau conj(c_{mu tau p}) W_{mu tau q} (planes x = 2, 3 are zero).
// K = 0, 1, 2: Call = the planes of -sigma_K c (sigma_x, sigma_y, sigma_z),
// Chat untouched.
void launch_build_spinor_mats(int N, int n, const double *C, int K, double *Call, double *Chat,
                              hipStream_t s);
// Scatter the slice's spinor columns into G[p][q][c][d][re, im]: for pair
// i = 2 g + h (c <= d) of group g, columns 4 g + 2 h (V re) and + 1 (V im) give
// A and B (complex, planes x = 0, 1 of Gc), (pq|cd) = A + iB and (pq|dc) = A - iB.
void launch_pack_spinor(int n, const int32_t *rs, int nspair, int64_t c0, int nc,
                        const double *Gc, double *G, int accumulate, hipStream_t s);
// Scatter Gc[c][(x,p)][q] for MO-pair columns c of [c0, c0+nc) (c = 4 idx + y)
// into G[p][q][r][s][x][y] and its mirror G[p][q][s][r][x][y] = mirror * s_y * v,
// s = (+1,-1,-1,-1); accumulate = 1 adds to G instead of storing.  Coulomb
// (mirror = +1): Gc holds p <= q (p > q by G_pq^x = s_x G_qp^x); Gaunt
// (mirror = -1): Gc holds the first bra-density term T for every (p, q) and
// G_pq^x = T_pq^x - s_x T_qp^x.
void launch_pack(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc, double *G,
                 double mirror, int accumulate, hipStream_t s);
// Block output of the same slice: B[i][p][q][0][x][y] = v, B[i][p][q][1][x][y] =
// mirror * s_y * v (v itself when r = s) for the slice's MO pairs, i = pair
// index - b_i0.
void launch_pack_block(int n, const int32_t *rs, int64_t c0, int nc, const double *Gc,
                       double *B, int64_t b_i0, double mirror, int accumulate, hipStream_t s);

}  // namespace qdcb
