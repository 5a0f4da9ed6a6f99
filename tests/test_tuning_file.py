"""The autotuner's table as a file (perks_tuning_save / perks_tuning_load),
on the host: a file's entries load and save back unchanged, and a file
that is not a tuning file is rejected with nothing loaded."""
import pytest

import paper_2204_02064_amd as pk

HEADER = "perks-tuning 1\n"
ROWS = ["0 1 256 256 1 0 0 8 0 0 0 3 8\n",        # 2d5pt FP64 256^2: temporal blocking, K 8
        "2 0 258 258 258 0 0 0 16 0 0 0 0\n"]     # 3d7pt FP32 258^3: 16-plane columns


def _lib_or_skip():
    try:
        return pk.lib()
    except Exception as e:   # the library is not built in this checkout
        pytest.skip(str(e))


def test_tuning_file_round_trip(tmp_path):
    _lib_or_skip()
    src = tmp_path / "in.txt"
    src.write_text(HEADER + "".join(ROWS))
    pk.tuning_load(str(src))
    out = tmp_path / "out.txt"
    pk.tuning_save(str(out))
    lines = out.read_text().splitlines(keepends=True)
    assert lines[0] == HEADER
    for r in ROWS:
        assert r in lines[1:]


@pytest.mark.parametrize("text", ["not a tuning file\n", HEADER + "0 1 256 256 1 0 0 8 0 0 0 9 8\n",
                                  HEADER + "0 1 256\n", "perks-tuning 2\n"])
def test_malformed_tuning_files_are_rejected(tmp_path, text):
    _lib_or_skip()
    before = tmp_path / "before.txt"
    pk.tuning_save(str(before))
    bad = tmp_path / "bad.txt"
    bad.write_text(text)
    with pytest.raises(RuntimeError):
        pk.tuning_load(str(bad))
    after = tmp_path / "after.txt"
    pk.tuning_save(str(after))
    assert after.read_text() == before.read_text()
