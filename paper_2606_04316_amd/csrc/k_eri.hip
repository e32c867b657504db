// k_eri.hip -- on-the-fly AO integral tiles for the first half.
//
// For every kept (bra tile, ket tile) a 64 x 64 block of contracted s-type
// ERIs (mn|kl) is generated from the primitive-pair data (Gaussian product
// theorem + Boys F0) and stored as panel[slot][ket j][bra m].  Each element
// is masked individually by the directed density-weighted Schwarz predicate
// of Eq. (SchwarzDen): it is computed only when (Q_mn * Q_kl) * Dmax_kl >= tau
// and is 0 otherwise, which is exactly the skip of that contribution.
//
// Work layout: 4 wavefronts x 16 ket rows each; lane = bra row.  The ket
// pair of a wavefront is uniform across its lanes, so its primitive data
// comes through scalar loads; the bra primitive data is per lane.  Stores are
// one 512-byte row of 64 bra values per ket row (coalesced).
#include "kernels.h"

namespace qdcb {

__global__ void __launch_bounds__(256) k_eri_tiles(EriTileArgs a) {
  const int64_t slot = a.slot0 + blockIdx.x;
  const int kt = a.tasks[slot];
  const int bt = a.task_bra[slot];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t brow = (int64_t)bt * TILE + lane;
  const double qb = a.Q[brow];
  const int cb = a.cls[brow];
  const int64_t bf0 = a.row_first[brow], bf1 = a.row_first[brow + 1];
  double *out = a.panel + (int64_t)blockIdx.x * TILE * TILE;
  long long kept[4] = {0, 0, 0, 0};
  for (int i = 0; i < TILE / 4; ++i) {
    const int j = w + 4 * i;
    const int64_t krow = (int64_t)kt * TILE + j;
    const double qk = a.Q[krow], dk = a.Dmax[krow];
    const int ck = a.cls[krow];
    const int64_t kf0 = a.row_first[krow], kf1 = a.row_first[krow + 1];
    double v = 0.0;
    if ((qb * qk) * dk >= a.tau) {
      v = contracted_eri(a.pp, bf0, bf1, a.pp, kf0, kf1);
      if (cb >= 0 && ck >= 0) kept[cb * 2 + ck] += 1;
    }
    out[j * TILE + lane] = v;
  }
  if (a.kept) {
    for (int c = 0; c < 4; ++c) {
      long long t = wave_sum_ll(kept[c]);
      if (lane == 0 && t) atomicAdd(a.kept + c, (unsigned long long)t);
    }
  }
}

void launch_eri_tiles(const EriTileArgs &a, int64_t nslots, hipStream_t s) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_eri_tiles, dim3((unsigned)nslots), dim3(256), 0, s, a);
}

}  // namespace qdcb
