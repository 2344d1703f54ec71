"""Persisted autotuner results: file format and validation (host only, on a
mock context, which holds a tuning cache like any other)."""
import os

import pytest

from paper_2509_17390_amd import Context
from paper_2509_17390_amd.rcast import RC_DEVICE_MOCK, RC_E_INVAL, RcastError

HEADER = "rcast-tuning-cache v2\n"
KEY = "gfx950:256cu|fmt1|tris2^20|pat32x1024|rays2^27|jobs2^0"
GOOD = KEY + " 0 0 64 0 16 4 4096 1 1 32\n"


def test_missing_file_is_an_empty_cache_and_save_roundtrips(tmp_path):
    c = Context(RC_DEVICE_MOCK)
    try:
        c.tuning_cache_load(str(tmp_path / "absent.txt"))
        out = tmp_path / "saved.txt"
        c.tuning_cache_save(str(out))
        assert out.read_text() == HEADER
        src = tmp_path / "src.txt"
        src.write_text(HEADER + GOOD + "# comment\n")
        c.tuning_cache_load(str(src))
        c.tuning_cache_save(str(out))
        assert out.read_text() == HEADER + GOOD
        assert not os.path.exists(str(out) + ".tmp")
    finally:
        c.close()


@pytest.mark.parametrize("body", [
    "not a cache\n" + GOOD,                                        # wrong version line
    HEADER + "key 0 0 64 0 16 4\n",                                # too few fields
    HEADER + GOOD.replace(" 16 4 4096", " 16 4 7"),                # chunk_max out of range
    HEADER + GOOD.replace(" 0 0 64", " 0 5 64"),                   # stack_lds not offered
    HEADER + GOOD.replace(" 1 1 32", " 1 1 65"),                   # leaf_batch out of range
    HEADER + GOOD.replace(" 1 1 32", " 1 1"),                      # v1 row in a v2 file
])
def test_malformed_or_out_of_range_entries_load_nothing(tmp_path, body):
    c = Context(RC_DEVICE_MOCK)
    try:
        p = tmp_path / "bad.txt"
        p.write_text(body)
        with pytest.raises(RcastError) as e:
            c.tuning_cache_load(str(p))
        assert e.value.status == RC_E_INVAL
        out = tmp_path / "after.txt"
        c.tuning_cache_save(str(out))
        assert out.read_text() == HEADER     # nothing from the bad file
    finally:
        c.close()


def test_version_1_files_load_with_leaf_tests_on_the_spot(tmp_path):
    """A cache written before the leaf_batch column (version 1 header, ten
    fields per row) loads with leaf_batch = 0 and is saved in version 2."""
    c = Context(RC_DEVICE_MOCK)
    try:
        src = tmp_path / "v1.txt"
        src.write_text("rcast-tuning-cache v1\n" + KEY + " 0 0 64 0 16 4 4096 1 1\n")
        c.tuning_cache_load(str(src))
        out = tmp_path / "v2.txt"
        c.tuning_cache_save(str(out))
        assert out.read_text() == HEADER + KEY + " 0 0 64 0 16 4 4096 1 1 0\n"
    finally:
        c.close()
