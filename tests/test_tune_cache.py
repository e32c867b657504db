"""CPU checks of the tuning cache of the C-ABI library (host file access
only): lookups of stored keys, the last stored line winning, missing files,
malformed lines and rejected keys."""
import os

import pytest


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    if not os.path.exists(qdcb.LIB_PATH):
        from paper_2606_04316_amd import build
        build.build()
    return qdcb


KEY = "v1 ham=2 prec=0 n=128 NL=600 NS=1200 kL=6 kS=6 tau=1.000e-10 tC=6500 tG=11250 cu=256"


def test_store_then_lookup_last_line_wins(q, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    assert q.tune_cache_lookup(path, KEY) is None  # no file yet
    q.tune_cache_store(path, KEY, {"eri_sched": 1, "fh_order": 0, "sq_tile": 128})
    q.tune_cache_store(path, "other", {"eri_sched": 0, "fh_order": 1, "sq_tile": 64})
    assert q.tune_cache_lookup(path, KEY) == {"eri_sched": 1, "fh_order": 0, "sq_tile": 128}
    q.tune_cache_store(path, KEY, {"eri_sched": 0, "fh_order": 0, "sq_tile": 64})
    assert q.tune_cache_lookup(path, KEY) == {"eri_sched": 0, "fh_order": 0, "sq_tile": 64}
    assert q.tune_cache_lookup(path, "other") == {"eri_sched": 0, "fh_order": 1, "sq_tile": 64}
    assert q.tune_cache_lookup(path, "missing") is None
    # every line is one JSON object
    import json
    for line in open(path):
        d = json.loads(line)
        assert set(d) == {"key", "eri_sched", "fh_order", "sq_tile"}


def test_malformed_and_out_of_range_lines_are_ignored(q, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    with open(path, "w") as f:
        f.write('{"key": "%s", "eri_sched": 1, "fh_order": 0, "sq_tile": 128}\n' % KEY)
        f.write('{"key": "%s", "eri_sched": 7, "fh_order": 0, "sq_tile": 128}\n' % KEY)
        f.write('{"key": "%s", "eri_sched": 1, "sq_tile": 32}\n' % KEY)
        f.write("not json at all\n")
    assert q.tune_cache_lookup(path, KEY) == {"eri_sched": 1, "fh_order": 0, "sq_tile": 128}


def test_keys_that_would_break_the_line_are_rejected(q, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    for bad in ('a"b', "a\nb", "a\\b"):
        with pytest.raises(q.QdcbError):
            q.tune_cache_store(path, bad, {"eri_sched": 0, "fh_order": 0, "sq_tile": 64})
    assert not os.path.exists(path) or open(path).read() == ""
