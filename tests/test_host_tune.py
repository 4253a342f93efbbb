"""The autotuner's table in its text form (no GPU needed): load, save, reset, errors."""
import os

import pytest


@pytest.fixture(scope="module")
def api():
    from paper_2605_02224_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmknn.so not built")
    from paper_2605_02224_amd import api as A
    return A


def test_table_round_trip(api, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text("mknn-tune 1\n0 1 1 19 3 6 4\n0 4 0 13 1 6 8\n0 2 0 20 2 6 4\n")
    api.tune_reset()
    api.tune_load(str(src))
    out = tmp_path / "out.txt"
    api.tune_save(str(out))
    lines = out.read_text().split("\n")
    assert lines[0] == "mknn-tune 1"
    assert sorted(l for l in lines[1:] if l) == sorted(
        ["0 1 1 19 3 6 4", "0 4 0 13 1 6 8", "0 2 0 20 2 6 4"])
    api.tune_reset()
    api.tune_save(str(out))
    assert out.read_text() == "mknn-tune 1\n"


@pytest.mark.parametrize("text", ["", "mknn-tune 2\n", "other 1\n", "mknn-tune 1\n0 1 1 19 3 6\n",
                                  "mknn-tune 1\n0 5 1 19 3 6 4\n", "mknn-tune 1\n0 1 1 19 4 6 4\n",
                                  "mknn-tune 1\n0 1 1 19 3 6 2\n"])
def test_malformed_tables_are_rejected_whole(api, tmp_path, text):
    from paper_2605_02224_amd._lib import MknnError, EINVAL
    api.tune_reset()
    bad = tmp_path / "bad.txt"
    bad.write_text(text)
    with pytest.raises(MknnError) as e:
        api.tune_load(str(bad))
    assert e.value.status == EINVAL
    out = tmp_path / "out.txt"
    api.tune_save(str(out))
    assert out.read_text() == "mknn-tune 1\n"


def test_missing_table(api, tmp_path):
    from paper_2605_02224_amd._lib import MknnError, ENOTFOUND
    with pytest.raises(MknnError) as e:
        api.tune_load(str(tmp_path / "nope.txt"))
    assert e.value.status == ENOTFOUND
