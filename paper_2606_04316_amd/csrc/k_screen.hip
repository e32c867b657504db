// k_screen.hip -- density-weighted Cauchy-Schwarz screening at tile level.
//
// Eq. (SchwarzDen): |(mn|kl) D_kl| <= Q_mn Q_kl ||D~_kl||_inf.  Pairs are
// ordered by decreasing Q, so a 64-pair tile has a tight maximum.  A
// (bra tile b, ket tile k) is kept when Qmax_b * Bmax_k >= tau, with
// Bmax_k = max over the tile of Q_kl Dmax_kl; every element is then masked
// individually by the exact directed predicate (Q_mn * Q_kl) * Dmax_kl >= tau
// when its integral tile is built.  The tile test carries a relative slack
// of 1e-12 so that rounding of the two different products can never drop a
// tile that still holds a kept element.
#include "kernels.h"

namespace qdcb {

__global__ void __launch_bounds__(64) k_tile_bounds(int ntiles, const double *Q,
                                                    const double *Dmax, double *Qmax,
                                                    double *Bmax, double *Dtmax) {
  int t = blockIdx.x;
  int64_t row = (int64_t)t * TILE + threadIdx.x;
  double q = Q[row];
  double d = Dmax[row];
  double b = q * d;
  q = wave_max(q);
  b = wave_max(b);
  d = wave_max(d);
  if (threadIdx.x == 0) {
    Qmax[t] = q;
    Bmax[t] = b;
    if (Dtmax) Dtmax[t] = d;
  }
}

void launch_tile_bounds(int ntiles, const double *Q, const double *Dmax, double *Qmax,
                        double *Bmax, double *Dtmax, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_tile_bounds, dim3(ntiles), dim3(64), 0, s, ntiles, Q, Dmax, Qmax, Bmax,
                     Dtmax);
}

__device__ __forceinline__ bool tile_kept(double qb, double bk, double tau) {
  return qb * bk >= tau * (1.0 - 1e-12);
}

__global__ void __launch_bounds__(256) k_screen_count(int ntiles, const double *Qmax,
                                                      const double *Bmax, double tau,
                                                      int32_t *count) {
  __shared__ int red[4];
  int b = blockIdx.x;
  double qb = Qmax[b];
  int c = 0;
  for (int k = threadIdx.x; k < ntiles; k += 256) c += tile_kept(qb, Bmax[k], tau) ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) count[b] = red[0] + red[1] + red[2] + red[3];
}

void launch_screen_count(int ntiles, const double *Qmax, const double *Bmax, double tau,
                         int32_t *count, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_screen_count, dim3(ntiles), dim3(256), 0, s, ntiles, Qmax, Bmax, tau,
                     count);
}

// Ordered compaction: chunks of 256 ket tiles, block-wide exclusive scan of
// the keep flags (wave ballots + per-wave offsets).
__global__ void __launch_bounds__(256) k_screen_fill(int b0, int ntiles, const double *Qmax,
                                                     const double *Bmax, double tau,
                                                     const int64_t *slot_base,
                                                     int32_t *tasks, int32_t *task_bra) {
  __shared__ int wsum[4];
  int b = b0 + blockIdx.x;
  double qb = Qmax[b];
  int64_t out = slot_base[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k0 = 0; k0 < ntiles; k0 += 256) {
    int k = k0 + threadIdx.x;
    bool keep = k < ntiles && tile_kept(qb, Bmax[k], tau);
    unsigned long long m = __ballot(keep);
    int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int i = 0; i < w; ++i) off += wsum[i];
    int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (keep) {
      tasks[out + off + before] = k;
      task_bra[out + off + before] = b;
    }
    out += total;
    __syncthreads();
  }
}

// Directed slot map: one workgroup per bra tile b, the same ordered
// compaction as k_screen_fill, writing dmap[b][k] = slot of task (b, k).
__global__ void __launch_bounds__(256) k_screen_fill_map(int ntiles, const double *Qmax,
                                                         const double *Bmax, double tau,
                                                         const int64_t *slot_base,
                                                         int32_t *dmap) {
  __shared__ int wsum[4];
  const int b = blockIdx.x;
  const double qb = Qmax[b];
  int64_t out = slot_base[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k0 = 0; k0 < ntiles; k0 += 256) {
    const int k = k0 + threadIdx.x;
    const bool keep = k < ntiles && tile_kept(qb, Bmax[k], tau);
    unsigned long long m = __ballot(keep);
    int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int i = 0; i < w; ++i) off += wsum[i];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (keep) dmap[(int64_t)b * ntiles + k] = (int32_t)(out + off + before);
    out += total;
    __syncthreads();
  }
}

void launch_screen_fill_map(int ntiles, const double *Qmax, const double *Bmax, double tau,
                            const int64_t *slot_base, int32_t *dmap, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_screen_fill_map, dim3(ntiles), dim3(256), 0, s, ntiles, Qmax, Bmax, tau,
                     slot_base, dmap);
}

// Unique (symmetric) tile pairs: (b, k) with k <= b is needed when either
// direction is kept, T[b][k] or T[k][b].  ucount[b] counts them per row.
__global__ void __launch_bounds__(256) k_screen_count_u(int ntiles, const double *Qmax,
                                                        const double *Bmax, double tau,
                                                        int32_t *ucount) {
  __shared__ int red[4];
  const int b = blockIdx.x;
  const double qb = Qmax[b], bb = Bmax[b];
  int c = 0;
  for (int k = threadIdx.x; k <= b; k += 256)
    c += (tile_kept(qb, Bmax[k], tau) || tile_kept(Qmax[k], bb, tau)) ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) ucount[b] = red[0] + red[1] + red[2] + red[3];
}

void launch_screen_count_u(int ntiles, const double *Qmax, const double *Bmax, double tau,
                           int32_t *ucount, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_screen_count_u, dim3(ntiles), dim3(256), 0, s, ntiles, Qmax, Bmax, tau,
                     ucount);
}

// Fill the unique pairs of row b in ascending k with their two directed
// slots (the directed map must be complete: same stream, launched before).
__global__ void __launch_bounds__(256) k_screen_fill_u(int ntiles, const double *Qmax,
                                                       const double *Bmax, double tau,
                                                       const int64_t *ubase,
                                                       const int32_t *dmap, int32_t *utask_k,
                                                       int32_t *utask_b, int32_t *uslot_bk,
                                                       int32_t *uslot_kb) {
  __shared__ int wsum[4];
  const int b = blockIdx.x;
  const double qb = Qmax[b], bb = Bmax[b];
  int64_t out = ubase[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k0 = 0; k0 <= b; k0 += 256) {
    const int k = k0 + threadIdx.x;
    const bool fwd = k <= b && tile_kept(qb, Bmax[k], tau);
    const bool rev = k < b && tile_kept(Qmax[k], bb, tau);
    const bool keep = fwd || rev;
    unsigned long long m = __ballot(keep);
    int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int i = 0; i < w; ++i) off += wsum[i];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (keep) {
      const int64_t slot = out + off + before;
      utask_k[slot] = k;
      utask_b[slot] = b;
      uslot_bk[slot] = fwd ? dmap[(int64_t)b * ntiles + k] : -1;
      uslot_kb[slot] = rev ? dmap[(int64_t)k * ntiles + b] : -1;
    }
    out += total;
    __syncthreads();
  }
}

void launch_screen_fill_u(int ntiles, const double *Qmax, const double *Bmax, double tau,
                          const int64_t *ubase, const int32_t *dmap, int32_t *utask_k,
                          int32_t *utask_b, int32_t *uslot_bk, int32_t *uslot_kb,
                          hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_screen_fill_u, dim3(ntiles), dim3(256), 0, s, ntiles, Qmax, Bmax, tau,
                     ubase, dmap, utask_k, utask_b, uslot_bk, uslot_kb);
}

// Tier split: one workgroup per bra tile, three ordered compactions of its
// task list (one per tier) into the same segment.
__global__ void __launch_bounds__(256) k_tier_split(
    int ntiles, const double *Qmax, const double *Bmax, const double *Dtmax, const double *sthr,
    double tau, int gbound, double t32, double t16, const int64_t *slot_base,
    const int32_t *count, const int32_t *tasks, int32_t *ttasks, int32_t *trank, int32_t *tdesc,
    int32_t *tcount, int32_t *toff) {
  __shared__ int wsum[4];
  const int b = blockIdx.x;
  // the bra tile's bound, raised to its pair partner's (tiles 2i and 2i + 1,
  // which the first half contracts in one workgroup): both tiles of a pair
  // then take every ket tile in the same tier, so the per-tier launches keep
  // the pair's shared staging
  const int bp = (b ^ 1) < ntiles ? (b ^ 1) : b;
  const double qb = gbound ? fmax(Bmax[b], Bmax[bp]) : fmax(Qmax[b], Qmax[bp]);
  const double qs = Qmax[b], tq = tau * (1.0 - 1e-12);
  const int64_t base = slot_base[b];
  const int n = count[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int out = 0;
  for (int tier = 0; tier < 3; ++tier) {
    const int first = out;
    for (int i0 = 0; i0 < n; i0 += 256) {
      const int i = i0 + threadIdx.x;
      int k = 0;
      bool keep = false;
      if (i < n) {
        k = tasks[base + i];
        const double B = qb * Bmax[k];
        const int t = B >= t32 ? 0 : (B >= t16 ? 1 : 2);
        keep = t == tier;
      }
      unsigned long long m = __ballot(keep);
      int before = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[w] = __popcll(m);
      __syncthreads();
      int off = 0;
      for (int j = 0; j < w; ++j) off += wsum[j];
      const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
      if (keep) {
        const int64_t e = base + out + off + before;
        ttasks[e] = k;
        trank[e] = i;
        int need = 4;
        if (sthr) {
          need = 1;
          for (int st = 1; st < 4; ++st)
            if (qs * sthr[(int64_t)k * 4 + st] >= tq) need = st + 1;
        }
        tdesc[e] = need | (scale_exp(qs * Qmax[k]) + 1024) << 3 |
                   (scale_exp(2.0 * Dtmax[k]) + 1024) << 14;
      }
      out += total;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      toff[tier * ntiles + b] = first;
      tcount[tier * ntiles + b] = out - first;
    }
  }
}

void launch_tier_split(int ntiles, const double *Qmax, const double *Bmax, const double *Dtmax,
                       const double *sthr, double tau, int gbound, double t32, double t16,
                       const int64_t *slot_base, const int32_t *count, const int32_t *tasks,
                       int32_t *ttasks, int32_t *trank, int32_t *tdesc, int32_t *tcount,
                       int32_t *toff, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_tier_split, dim3(ntiles), dim3(256), 0, s, ntiles, Qmax, Bmax, Dtmax, sthr,
                     tau, gbound, t32, t16, slot_base, count, tasks, ttasks, trank, tdesc, tcount,
                     toff);
}

// Device-side exclusive scan of the per-bra-tile counts (one workgroup of
// 1024 threads, each over a contiguous run of counts): slot_base, the total,
// and an overflow flag when the total exceeds the integral-panel capacity.
__global__ void __launch_bounds__(1024) k_scan_counts(int ntiles, const int32_t *count,
                                                      int64_t *slot_base, int64_t *total,
                                                      int64_t capacity, int32_t *overflow) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (ntiles + 1023) / 1024;
  const int i0 = t * per, i1 = min(ntiles, i0 + per);
  int64_t s = 0;
  for (int i = i0; i < i1; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int i = i0; i < i1; ++i) {
    slot_base[i] = run;
    run += count[i];
  }
  if (t == 1023) {
    *total = part[1023];
    *overflow = part[1023] > capacity ? 1 : 0;
  }
}

void launch_scan_counts(int ntiles, const int32_t *count, int64_t *slot_base, int64_t *total,
                        int64_t capacity, int32_t *overflow, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, ntiles, count, slot_base, total,
                     capacity, overflow);
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

void launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
}

// ---------------------------------------------------------------------------
// Longest-first order of the unique integral tiles (persistent schedule).  The
// cost class of a tile pair is floor(log2(P_b * P_k)), P_t the primitive pairs
// of tile t's 64 rows (P_b * P_k is the tile pair's primitive-quartet count
// when no element is masked); its index is the product's count of leading zero
// bits, so ascending indices run from the costliest tiles down.
__device__ __forceinline__ int lpt_class(const int64_t *row_first, int bt, int kt) {
  const int64_t pb = row_first[(int64_t)(bt + 1) * TILE] - row_first[(int64_t)bt * TILE];
  const int64_t pk = row_first[(int64_t)(kt + 1) * TILE] - row_first[(int64_t)kt * TILE];
  const unsigned long long c =
      (unsigned long long)max(pb, (int64_t)1) * (unsigned long long)max(pk, (int64_t)1);
  return __clzll((long long)c);  // c >= 1: 0..63
}

__device__ __forceinline__ int64_t lpt_n(int64_t n_host, const int64_t *d_total, int64_t cap) {
  return d_total ? min(*d_total, cap) : n_host;
}

// class sizes: work[c] += number of tasks of class c
__global__ void __launch_bounds__(256) k_lpt_count(int64_t n_host, const int64_t *d_total,
                                                   int64_t cap, const int32_t *tk,
                                                   const int32_t *tb, const int64_t *row_first,
                                                   unsigned long long *work) {
  __shared__ unsigned int h[LPT_CLASSES];
  if (threadIdx.x < LPT_CLASSES) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = lpt_n(n_host, d_total, cap);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    atomicAdd(&h[lpt_class(row_first, tb[i], tk[i])], 1u);
  __syncthreads();
  if (threadIdx.x < LPT_CLASSES && h[threadIdx.x])
    atomicAdd(&work[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// work[64 + c] = first position of class c; the queue counter work[128] = 0
__global__ void k_lpt_scan(unsigned long long *work) {
  if (threadIdx.x != 0) return;
  unsigned long long acc = 0;
  for (int c = 0; c < LPT_CLASSES; ++c) {
    work[LPT_CLASSES + c] = acc;
    acc += work[c];
  }
  work[2 * LPT_CLASSES] = 0;
}

// order[pos] = task index; each block reserves a range per class for its 256
// tasks with one atomic, then places them by their rank inside the block
__global__ void __launch_bounds__(256) k_lpt_scatter(int64_t n_host, const int64_t *d_total,
                                                     int64_t cap, const int32_t *tk,
                                                     const int32_t *tb, const int64_t *row_first,
                                                     unsigned long long *work, int32_t *order) {
  __shared__ unsigned int h[LPT_CLASSES];
  __shared__ unsigned long long base[LPT_CLASSES];
  const int64_t n = lpt_n(n_host, d_total, cap);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; i0 < n; i0 += (int64_t)gridDim.x * 256) {
    if (threadIdx.x < LPT_CLASSES) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = i0 + threadIdx.x;
    int c = -1;
    unsigned int r = 0;
    if (i < n) {
      c = lpt_class(row_first, tb[i], tk[i]);
      r = atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < LPT_CLASSES && h[threadIdx.x])
      base[threadIdx.x] =
          atomicAdd(&work[LPT_CLASSES + threadIdx.x], (unsigned long long)h[threadIdx.x]);
    __syncthreads();
    if (c >= 0) order[base[c] + r] = (int32_t)i;
    __syncthreads();
  }
}

void launch_lpt_order(int64_t n_host, const int64_t *d_total, int64_t cap, int64_t grid_cap,
                      const int32_t *task_k, const int32_t *task_b, const int64_t *row_first,
                      unsigned long long *work, int32_t *order, hipStream_t s) {
  launch_zero_u64(work, LPT_WORK, s);
  const int64_t m = d_total ? grid_cap : n_host;
  if (m <= 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>((m + 255) / 256, 2048);
  hipLaunchKernelGGL(k_lpt_count, dim3(nb), dim3(256), 0, s, n_host, d_total, cap, task_k,
                     task_b, row_first, work);
  hipLaunchKernelGGL(k_lpt_scan, dim3(1), dim3(64), 0, s, work);
  hipLaunchKernelGGL(k_lpt_scatter, dim3(nb), dim3(256), 0, s, n_host, d_total, cap, task_k,
                     task_b, row_first, work, order);
}

void launch_screen_fill(int b0, int b1, int ntiles, const double *Qmax, const double *Bmax,
                        double tau, const int64_t *slot_base, int32_t *tasks,
                        int32_t *task_bra, hipStream_t s) {
  if (b1 <= b0) return;
  hipLaunchKernelGGL(k_screen_fill, dim3(b1 - b0), dim3(256), 0, s, b0, ntiles, Qmax, Bmax, tau,
                     slot_base, tasks, task_bra);
}

// Intra-tile row order of a transform: within each 64-row tile the rows are
// ranked by decreasing bound B = Q Dmax (ties by row), one wavefront per
// tile.  perm[64 t + i] = the tile-local row at position i; sthr[4 t + s] =
// the B of position 16 s, the largest of the 16 rows of step s.
__global__ void __launch_bounds__(TILE) k_tile_order(int ntiles, const double *Q,
                                                     const double *Dmax, int32_t *perm,
                                                     double *sthr) {
  const int t = blockIdx.x, i = threadIdx.x;
  const int64_t row = (int64_t)t * TILE + i;
  const double b = Q[row] * Dmax[row];
  int rank = 0;
  for (int j = 0; j < TILE; ++j) {
    const double bj = __shfl(b, j, 64);
    rank += (bj > b || (bj == b && j < i)) ? 1 : 0;
  }
  perm[(int64_t)t * TILE + rank] = i;
  if (rank % 16 == 0) sthr[(int64_t)t * 4 + rank / 16] = b;
}

void launch_tile_order(int ntiles, const double *Q, const double *Dmax, int32_t *perm,
                       double *sthr, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_tile_order, dim3(ntiles), dim3(TILE), 0, s, ntiles, Q, Dmax, perm, sthr);
}

// Row data in that order, one wavefront per tile: Q, Dmax, class, pair
// functions and code of position i are those of row perm[i]; the primitive
// pairs of the tile keep
// their range [row_first[64 t], row_first[64 t + 64]) and are regrouped by
// position (wrow_first from a wavefront scan of the permuted counts), read
// contiguously, each written to its row's new place.
__global__ void __launch_bounds__(TILE) k_gather_rows(int ntiles, const int32_t *perm,
                                                      const double *Q, const double *Dmax,
                                                      const int32_t *cls, const int32_t *mu,
                                                      const int32_t *nu, const int32_t *code,
                                                      const int64_t *row_first, PrimPairsC pp,
                                                      double *wQ, double *wDmax, int32_t *wcls,
                                                      int32_t *wmu, int32_t *wnu,
                                                      int32_t *wcode, int64_t *wrow_first,
                                                      PrimPairs wpp) {
  __shared__ int64_t sfirst[TILE + 1];  // tile-local source offsets by row
  __shared__ int64_t dfirst[TILE];      // destination offset of each source row
  const int t = blockIdx.x, i = threadIdx.x;
  const int64_t base = (int64_t)t * TILE;
  const int src = perm[base + i];
  wQ[base + i] = Q[base + src];
  wDmax[base + i] = Dmax[base + src];
  wcls[base + i] = cls[base + src];
  wmu[base + i] = mu[base + src];
  wnu[base + i] = nu[base + src];
  if (code) wcode[base + i] = code[base + src];
  const int64_t t0 = row_first[base], t1 = row_first[base + TILE];
  sfirst[i] = row_first[base + i] - t0;
  if (i == 0) sfirst[TILE] = t1 - t0;
  __syncthreads();
  // exclusive scan of the counts in position order
  const int64_t c = sfirst[src + 1] - sfirst[src];
  int64_t x = c;
  for (int o = 1; o < TILE; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (i >= o) x += y;
  }
  const int64_t ex = x - c;
  wrow_first[base + i] = t0 + ex;
  if (t == ntiles - 1 && i == TILE - 1) wrow_first[base + TILE] = t1;
  dfirst[src] = ex;
  __syncthreads();
  // primitive pairs: source index g -> its row (search over sfirst) -> destination
  const int64_t n = t1 - t0;
  for (int64_t g = i; g < n; g += TILE) {
    int lo = 0, hi = TILE;  // last row with sfirst <= g
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sfirst[mid] <= g) lo = mid;
      else hi = mid;
    }
    while (lo + 1 < TILE && sfirst[lo + 1] <= g) ++lo;  // skip empty rows
    const int64_t from = t0 + g, to = t0 + dfirst[lo] + (g - sfirst[lo]);
    wpp.ip[to] = pp.ip[from];
    wpp.x[to] = pp.x[from];
    wpp.y[to] = pp.y[from];
    wpp.z[to] = pp.z[from];
    wpp.e[to] = pp.e[from];
    if (pp.pa) {
      wpp.pa[to] = pp.pa[from];
      wpp.pb[to] = pp.pb[from];
      wpp.ax[to] = pp.ax[from];
      wpp.ay[to] = pp.ay[from];
      wpp.az[to] = pp.az[from];
      wpp.bx[to] = pp.bx[from];
      wpp.by[to] = pp.by[from];
      wpp.bz[to] = pp.bz[from];
      for (int k = 0; k < PAIR_E; ++k) wpp.E[PAIR_E * to + k] = pp.E[PAIR_E * from + k];
    }
  }
}

void launch_gather_rows(int ntiles, const int32_t *perm, const double *Q, const double *Dmax,
                        const int32_t *cls, const int32_t *mu, const int32_t *nu,
                        const int32_t *code, const int64_t *row_first, PrimPairsC pp, double *wQ,
                        double *wDmax, int32_t *wcls, int32_t *wmu, int32_t *wnu,
                        int32_t *wcode, int64_t *wrow_first, PrimPairs wpp, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(ntiles), dim3(TILE), 0, s, ntiles, perm, Q, Dmax, cls,
                     mu, nu, code, row_first, pp, wQ, wDmax, wcls, wmu, wnu, wcode, wrow_first,
                     wpp);
}

// First-half work of the intra-tile order: the 16-row steps the contraction
// runs, summed over the directed tasks (bra tile b, ket tile k): 1 plus the
// steps s >= 1 with Qmax[b] sthr[4 k + s] >= tau (1 - 1e-12), as the
// first-half kernel counts them.  One workgroup per bra tile; *out += the sum.
__global__ void __launch_bounds__(256) k_step_work(int ntiles, const int64_t *slot_base,
                                                   const int32_t *count, const int32_t *tasks,
                                                   const double *Qmax, const double *sthr,
                                                   double tau, unsigned long long *out) {
  __shared__ unsigned long long red[4];
  const int b = blockIdx.x;
  const double qb = Qmax[b], tq = tau * (1.0 - 1e-12);
  const int64_t base = slot_base[b];
  unsigned long long sum = 0;
  for (int i = threadIdx.x; i < count[b]; i += 256) {
    const int64_t k = tasks[base + i];
    int ns = 1;
    for (int st = 1; st < 4; ++st)
      if (qb * sthr[k * 4 + st] >= tq) ns = st + 1;
    sum += (unsigned long long)ns;
  }
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, red[0] + red[1] + red[2] + red[3]);
}

void launch_step_work(int ntiles, const int64_t *slot_base, const int32_t *count,
                      const int32_t *tasks, const double *Qmax, const double *sthr, double tau,
                      unsigned long long *out, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_step_work, dim3(ntiles), dim3(256), 0, s, ntiles, slot_base, count,
                     tasks, Qmax, sthr, tau, out);
}

}  // namespace qdcb
