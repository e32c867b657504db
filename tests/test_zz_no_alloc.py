"""GPU test of the allocation-free entry point qdcb_eri_quartets_noalloc
against qdcb_eri_quartets (the existing entry point with allocated staging):
the same integral kernels on the same inputs give the same bits.  Two calls
in a row, the second with fewer quartets (the array keeps the first call's
contents, which must not leak into the second), on an s-only and an s/p
basis pair; the size limit is refused before any device work."""
import numpy as np
import pytest

from paper_2606_04316_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


def _quartets(rng, na, nb, k):
    return np.stack([rng.integers(0, na, k), rng.integers(0, na, k),
                     rng.integers(0, nb, k), rng.integers(0, nb, k)], 1).astype(np.int32)


def test_noalloc_matches_allocating_entry_twice(q):
    ctx = q.Context(0)
    s = wl.cluster(seed=32, n_atoms=6, nl_per_atom=3, ns_per_atom=3, n=2, radius=5.0,
                   min_sep=1.0)
    sp = wl.sp_cluster(seed=41, n_atoms=4, edge=5.0, nprim=(1, 3), n=2, ham="DC")
    rng = np.random.default_rng(0)
    for La, Sb, label in ((s.L, s.S, "s"), (sp.L, sp.S, "s and p")):
        A, B = q.Basis(ctx, La), q.Basis(ctx, Sb)
        for k in (20000, 777):  # second call smaller than the first
            idx = _quartets(rng, La.nfunc, Sb.nfunc, k)
            ref = q.eri_quartets(A, B, idx)
            got = q.eri_quartets_noalloc(A, B, idx)
            print(f"{label}: {k} quartets, max|ref| {np.abs(ref).max():.3e}", flush=True)
            assert got.shape == ref.shape
            assert np.array_equal(got, ref), label
        A.close()
        B.close()
    ctx.close()


def test_noalloc_limits_and_arguments(q):
    ctx = q.Context(0)
    s = wl.small_ll(seed=39, n_atoms=2, nfunc=4, n=2)
    A = q.Basis(ctx, s.L)
    big = np.zeros((q.NOALLOC_MAX_QUARTETS + 1, 4), dtype=np.int32)
    with pytest.raises(q.QdcbError) as e:
        q.eri_quartets_noalloc(A, A, big)
    assert e.value.status == -1 and "limit" in str(e.value)
    bad = np.array([[0, 0, 0, 4]], dtype=np.int32)
    with pytest.raises(q.QdcbError):
        q.eri_quartets_noalloc(A, A, bad)
    assert q.eri_quartets_noalloc(A, A, np.zeros((0, 4), np.int32)).shape == (0,)
    # exactly at the limit
    full = np.zeros((q.NOALLOC_MAX_QUARTETS, 4), dtype=np.int32)
    full[:, 1] = np.arange(full.shape[0]) % 4
    assert np.array_equal(q.eri_quartets_noalloc(A, A, full), q.eri_quartets(A, A, full))
    A.close()
    ctx.close()
